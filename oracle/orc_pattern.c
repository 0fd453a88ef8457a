/*
 * Oracle (test infrastructure only): pattern compiler and exact counters.
 *
 * Sec. 4.2 keeps NS-prune unbiased by pruning only with a matching order and
 * symmetry breaking, because each restricted match is then one root-to-leaf
 * path of the subgraph tree.  The paper names the techniques but not an
 * algorithm, so the oracle fixes one reading:
 *   matching order: first the pattern vertex of largest degree (lowest index on
 *     ties), then its lowest-index neighbour of largest degree; then repeatedly
 *     the unmatched vertex with the most edges into the matched set (ties:
 *     larger pattern degree, then lower index);
 *   restrictions: the orbit/stabiliser chain over Aut(P) (Grochow and Kellis,
 *     RECOMB 2007): for each position i in order, if the current group moves i,
 *     require v_i > v_t for every other t in the orbit of i, then keep only the
 *     automorphisms that fix i.  For the 4-cycle this yields v0 = max and
 *     v3 < v1, the worked example of Sec. 4.2.
 * First-edge mode: when the plan orders v0 > v1 the first edge is drawn from
 * the m oriented edges (alpha starts at m, as in the paper's 4-cycle
 * algorithm); otherwise from the 2m arcs.
 */
#include "oracle.h"
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

static int build_adj(int k, int l, const int32_t* edges, uint8_t adj[8][8]) {
    memset(adj, 0, 64);
    for (int e = 0; e < l; e++) {
        int a = edges[2 * e], b = edges[2 * e + 1];
        if (a < 0 || b < 0 || a >= k || b >= k || a == b) return -1;
        adj[a][b] = adj[b][a] = 1;
    }
    return 0;
}

static int connected(int k, uint8_t adj[8][8]) {
    int seen = 1, grew = 1;
    while (grew) {
        grew = 0;
        for (int a = 0; a < k; a++)
            if (seen >> a & 1)
                for (int b = 0; b < k; b++)
                    if (adj[a][b] && !(seen >> b & 1)) { seen |= 1 << b; grew = 1; }
    }
    return seen == (1 << k) - 1;
}

/* all permutations of 0..k-1 in lexicographic order */
static int next_perm(int* p, int k) {
    int i = k - 2;
    while (i >= 0 && p[i] > p[i + 1]) i--;
    if (i < 0) return 0;
    int j = k - 1;
    while (p[j] < p[i]) j--;
    int t = p[i]; p[i] = p[j]; p[j] = t;
    for (int a = i + 1, b = k - 1; a < b; a++, b--) { t = p[a]; p[a] = p[b]; p[b] = t; }
    return 1;
}

static int is_aut(const int* p, int k, uint8_t adj[8][8]) {
    for (int a = 0; a < k; a++)
        for (int b = 0; b < k; b++)
            if (adj[a][b] != adj[p[a]][p[b]]) return 0;
    return 1;
}

int orc_automorphisms(int k, int l, const int32_t* edges) {
    uint8_t adj[8][8];
    if (k < 1 || k > 8 || build_adj(k, l, edges, adj)) return -1;
    int p[8], cnt = 0;
    for (int i = 0; i < k; i++) p[i] = i;
    do cnt += is_aut(p, k, adj); while (next_perm(p, k));
    return cnt;
}

int orc_compile(int k, int l, const int32_t* edges, int induced, orc_plan* out) {
    uint8_t adj[8][8];
    memset(out, 0, sizeof(*out));
    if (k < 2 || k > 8) return -4;
    if (build_adj(k, l, edges, adj)) return -1;
    if (!connected(k, adj)) return -4;
    int deg[8] = {0};
    for (int a = 0; a < k; a++)
        for (int b = 0; b < k; b++) deg[a] += adj[a][b];
    /* matching order */
    int order[8], used[8] = {0};
    int first = 0;
    for (int a = 1; a < k; a++)
        if (deg[a] > deg[first]) first = a;
    int second = -1;
    for (int b = 0; b < k; b++)
        if (adj[first][b] && (second < 0 || deg[b] > deg[second])) second = b;
    order[0] = first; order[1] = second;
    used[first] = used[second] = 1;
    for (int pos = 2; pos < k; pos++) {
        int best = -1, best_links = -1;
        for (int c = 0; c < k; c++) {
            if (used[c]) continue;
            int links = 0;
            for (int i = 0; i < pos; i++) links += adj[c][order[i]];
            if (links > best_links || (links == best_links && deg[c] > deg[best])) {
                best = c; best_links = links;
            }
        }
        if (best_links < 1) return -4;
        order[pos] = best;
        used[best] = 1;
    }
    /* automorphisms expressed on positions: gamma(i) = pos of perm(order[i]) */
    int posof[8];
    for (int i = 0; i < k; i++) posof[order[i]] = i;
    static int group[40320][8];
    int ng = 0;
    int p[8];
    for (int i = 0; i < k; i++) p[i] = i;
    do {
        if (is_aut(p, k, adj)) {
            for (int i = 0; i < k; i++) group[ng][i] = posof[p[order[i]]];
            ng++;
        }
    } while (next_perm(p, k));
    out->aut = ng;
    /* orbit / stabiliser chain */
    int alive[40320];
    for (int g = 0; g < ng; g++) alive[g] = 1;
    for (int i = 0; i < k; i++) {
        uint32_t orbit = 0;
        for (int g = 0; g < ng; g++)
            if (alive[g]) orbit |= 1u << group[g][i];
        for (int t = 0; t < k; t++)
            if (t != i && (orbit >> t & 1)) {
                /* v_i > v_t; t > i because positions before i are fixed */
                if (t > i) out->upper[t] |= (uint8_t)(1u << i);
                else out->lower[i] |= (uint8_t)(1u << t);
            }
        for (int g = 0; g < ng; g++)
            if (alive[g] && group[g][i] != i) alive[g] = 0;
    }
    out->k = k;
    out->induced = induced ? 1 : 0;
    for (int i = 0; i < k; i++) out->order[i] = order[i];
    for (int j = 0; j < k; j++)
        for (int i = 0; i < j; i++) {
            if (adj[order[i]][order[j]]) out->connect[j] |= (uint8_t)(1u << i);
            else if (induced) out->disconnect[j] |= (uint8_t)(1u << i);
        }
    out->oriented = (out->upper[1] & 1) ? 1 : 0;
    return 0;
}

/* ------------------------------------------------------------------ exact counters */

static int is_edge(const orc_graph* g, int64_t u, int64_t v) {
    int64_t lo = g->off[u], hi = g->off[u + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (g->nbr[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo < g->off[u + 1] && g->nbr[lo] == v;
}

/* Brute force: count injective maps V_P -> V_G preserving pattern edges (and,
 * when induced, non-edges); the occurrence count is that number / |Aut(P)|. */
void orc_brute_count(const orc_graph* g, int k, int l, const int32_t* edges, int induced,
                     uint64_t* injective_maps, uint64_t* count) {
    uint8_t adj[8][8];
    *injective_maps = 0; *count = 0;
    if (build_adj(k, l, edges, adj)) return;
    int64_t n = g->n;
    int64_t phi[8];
    uint64_t total = 0;
    /* odometer over n^k tuples with early rejection */
    int depth = 0;
    phi[0] = -1;
    while (depth >= 0) {
        phi[depth]++;
        if (phi[depth] >= n) { depth--; continue; }
        int ok = 1;
        for (int i = 0; i < depth && ok; i++) {
            if (phi[i] == phi[depth]) ok = 0;
            else {
                int e = is_edge(g, phi[i], phi[depth]);
                if (adj[i][depth] && !e) ok = 0;
                if (induced && !adj[i][depth] && e) ok = 0;
            }
        }
        if (!ok) continue;
        if (depth == k - 1) { total++; continue; }
        depth++;
        phi[depth] = -1;
    }
    int aut = orc_automorphisms(k, l, edges);
    *injective_maps = total;
    *count = aut > 0 ? total / (uint64_t)aut : 0;
}

/* Plan-based exact count: the number of tuples (v_0..v_{k-1}) that satisfy the
 * plan, i.e. the leaves of the pruned subgraph tree (Sec. 2.1, Sec. 4.2). */
typedef struct {
    const orc_graph* g; const orc_plan* p; uint64_t e0, e1; unsigned __int128 total;
} pc_job;

static unsigned __int128 pc_rec(const orc_graph* g, const orc_plan* p, int j, int32_t* v, int32_t* buf,
                                size_t stride) {
    int32_t* mine = buf + (size_t)j * stride;
    uint64_t cnt = orc_candidates(g, p, j, v, mine);
    if (j == p->k - 1) return cnt;
    unsigned __int128 t = 0;
    for (uint64_t i = 0; i < cnt; i++) {
        v[j] = mine[i];
        t += pc_rec(g, p, j + 1, v, buf, stride);
    }
    return t;
}

static void* pc_worker(void* arg) {
    pc_job* J = (pc_job*)arg;
    const orc_graph* g = J->g;
    const orc_plan* p = J->p;
    int64_t maxdeg = 0;
    for (int64_t u = 0; u < g->n; u++)
        if (g->off[u + 1] - g->off[u] > maxdeg) maxdeg = g->off[u + 1] - g->off[u];
    size_t stride = (size_t)maxdeg + 1;
    int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * 8 * stride);
    int32_t v[8];
    J->total = 0;
    for (uint64_t e = J->e0; e < J->e1; e++) {
        if (p->oriented) { v[0] = g->esrc[e]; v[1] = g->edst[e]; }
        else { v[0] = g->arow[e]; v[1] = g->nbr[e]; }
        if (p->k == 2) { J->total += 1; continue; }
        J->total += pc_rec(g, p, 2, v, buf, stride);
    }
    free(buf);
    return NULL;
}

void orc_plan_count(const orc_graph* g, const orc_plan* p, int nthreads, uint64_t* lo, uint64_t* hi) {
    uint64_t M = p->oriented ? (uint64_t)g->m : 2 * (uint64_t)g->m;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64];
    pc_job jobs[64];
    /* interleave ranges in 64 blocks per thread so skewed degree orders balance */
    unsigned __int128 total = 0;
    int nblocks = nthreads * 64;
    for (int base = 0; base < nblocks; base += nthreads) {
        for (int t = 0; t < nthreads; t++) {
            int b = base + t;
            jobs[t].g = g; jobs[t].p = p;
            jobs[t].e0 = M * (uint64_t)b / (uint64_t)nblocks;
            jobs[t].e1 = M * (uint64_t)(b + 1) / (uint64_t)nblocks;
            pthread_create(&th[t], NULL, pc_worker, &jobs[t]);
        }
        for (int t = 0; t < nthreads; t++) {
            pthread_join(th[t], NULL);
            total += jobs[t].total;
        }
    }
    *lo = (uint64_t)total;
    *hi = (uint64_t)(total >> 64);
}

/* Algorithmic bytes of the exact search (Sec. 4.4 nested loops; the work
 * measure of the GS cost model): the search tree's node at level j (a partial
 * match v_0..v_{j-1}) forms S_j, reading what one NS step reads from the same
 * partial match (orc_step_bytes: 16 per row first merged at this level of the
 * path, 4 per entry of every merged row inside the level's bounds); the sum
 * runs over every node of every level 2..k-1. */
typedef struct {
    const orc_graph* g; const orc_plan* p; uint64_t e0, e1; uint64_t bytes;
} pb_job;

static uint64_t pb_rec(const orc_graph* g, const orc_plan* p, int j, int32_t* v, uint32_t opened, int32_t* buf,
                       size_t stride) {
    uint64_t unused = 0;
    uint64_t b = orc_step_bytes(g, p, j, v, &opened, &unused);
    int32_t* mine = buf + (size_t)j * stride;
    uint64_t cnt = orc_candidates(g, p, j, v, mine);
    if (j == p->k - 1) return b;
    for (uint64_t i = 0; i < cnt; i++) {
        v[j] = mine[i];
        b += pb_rec(g, p, j + 1, v, opened, buf, stride);
    }
    return b;
}

static void* pb_worker(void* arg) {
    pb_job* J = (pb_job*)arg;
    const orc_graph* g = J->g;
    const orc_plan* p = J->p;
    int64_t maxdeg = 0;
    for (int64_t u = 0; u < g->n; u++)
        if (g->off[u + 1] - g->off[u] > maxdeg) maxdeg = g->off[u + 1] - g->off[u];
    size_t stride = (size_t)maxdeg + 1;
    int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * 8 * stride);
    int32_t v[8];
    J->bytes = 0;
    for (uint64_t e = J->e0; e < J->e1; e++) {
        if (p->oriented) { v[0] = g->esrc[e]; v[1] = g->edst[e]; }
        else { v[0] = g->arow[e]; v[1] = g->nbr[e]; }
        J->bytes += 8;  /* the first edge */
        if (p->k > 2) J->bytes += pb_rec(g, p, 2, v, 0u, buf, stride);
    }
    free(buf);
    return NULL;
}

uint64_t orc_plan_count_bytes(const orc_graph* g, const orc_plan* p, int nthreads) {
    uint64_t M = p->oriented ? (uint64_t)g->m : 2 * (uint64_t)g->m;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64];
    pb_job jobs[64];
    uint64_t total = 0;
    int nblocks = nthreads * 64;
    for (int base = 0; base < nblocks; base += nthreads) {
        for (int t = 0; t < nthreads; t++) {
            int b = base + t;
            jobs[t].g = g; jobs[t].p = p;
            jobs[t].e0 = M * (uint64_t)b / (uint64_t)nblocks;
            jobs[t].e1 = M * (uint64_t)(b + 1) / (uint64_t)nblocks;
            pthread_create(&th[t], NULL, pb_worker, &jobs[t]);
        }
        for (int t = 0; t < nthreads; t++) {
            pthread_join(th[t], NULL);
            total += jobs[t].bytes;
        }
    }
    return total;
}
