/*
 * Oracle (test infrastructure only): Philox4x32-10 and graph canonicalisation.
 *
 * Philox4x32-10 follows Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers:
 * As Easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64 multiplications
 * with multipliers 0xD2511F53 and 0xCD9E8D57, the key bumped between rounds by
 * the Weyl constants 0x9E3779B9 and 0xBB67AE85.
 *
 * The paper keeps its data graphs symmetric with no loops or duplicate edges
 * and orients them for cliques (Sec. 6, Table "Data graphs").  The oracle's
 * canonical form: symmetrise, drop loops, dedupe, relabel by degree
 * descending (ties: original id ascending), sort every row ascending.
 */
#include "oracle.h"
#include <stdlib.h>
#include <string.h>

static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(0xD2511F53u, c0, &hi0, &lo0);
        mulhilo32(0xCD9E8D57u, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Draw d of sample s: key = seed, counter = (s_lo, s_hi, d, tag), value = w1:w0. */
uint64_t orc_draw(uint64_t seed, uint64_t s, uint32_t d, uint32_t tag) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)s, (uint32_t)(s >> 32), d, tag};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return ((uint64_t)out[1] << 32) | (uint64_t)out[0];
}

/* Uniform index in [0, n): floor(n * r / 2^64). */
uint64_t orc_mulhi(uint64_t n, uint64_t r) {
    return (uint64_t)(((unsigned __int128)n * (unsigned __int128)r) >> 64);
}

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

void orc_graph_free(orc_graph* g) {
    free(g->off); free(g->nbr); free(g->esrc); free(g->edst); free(g->arow); free(g->perm);
    memset(g, 0, sizeof(*g));
}

/* Build off/nbr/esrc/edst/arow from a sorted, deduplicated, symmetric arc list. */
static int fill_from_arcs(int64_t n, int64_t narcs, const uint64_t* arcs, orc_graph* g) {
    g->n = n;
    g->m = narcs / 2;
    g->off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    g->nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(narcs ? narcs : 1));
    g->arow = (int32_t*)malloc(sizeof(int32_t) * (size_t)(narcs ? narcs : 1));
    g->esrc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->m ? g->m : 1));
    g->edst = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->m ? g->m : 1));
    if (!g->off || !g->nbr || !g->arow || !g->esrc || !g->edst) return -2;
    for (int64_t a = 0; a < narcs; a++) g->off[(arcs[a] >> 32) + 1]++;
    for (int64_t u = 0; u < n; u++) g->off[u + 1] += g->off[u];
    int64_t e = 0;
    for (int64_t a = 0; a < narcs; a++) {
        int32_t u = (int32_t)(arcs[a] >> 32), w = (int32_t)(uint32_t)arcs[a];
        g->nbr[a] = w;
        g->arow[a] = u;
        if (w < u) {
            g->esrc[e] = u;
            g->edst[e] = w;
            e++;
        }
    }
    return e == g->m ? 0 : -3;
}

typedef struct { int64_t deg; int64_t id; } deg_id;

static int cmp_deg_id(const void* a, const void* b) {
    const deg_id* x = (const deg_id*)a;
    const deg_id* y = (const deg_id*)b;
    if (x->deg != y->deg) return x->deg > y->deg ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

int orc_canon(int64_t n, const int64_t* in_off, const int32_t* in_nbr, orc_graph* g) {
    memset(g, 0, sizeof(*g));
    if (n < 0 || n > 0x7fffffffLL) return -1;
    if (in_off[0] != 0) return -1;
    for (int64_t u = 0; u < n; u++)
        if (in_off[u + 1] < in_off[u]) return -1;
    int64_t nin = in_off[n];
    for (int64_t i = 0; i < nin; i++)
        if (in_nbr[i] < 0 || in_nbr[i] >= n) return -1;
    /* symmetrise, drop loops */
    uint64_t* arcs = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(2 * nin + 1));
    if (!arcs) return -2;
    int64_t na = 0;
    for (int64_t u = 0; u < n; u++)
        for (int64_t i = in_off[u]; i < in_off[u + 1]; i++) {
            uint64_t v = (uint64_t)in_nbr[i];
            if (v == (uint64_t)u) continue;
            arcs[na++] = ((uint64_t)u << 32) | v;
            arcs[na++] = (v << 32) | (uint64_t)u;
        }
    qsort(arcs, (size_t)na, sizeof(uint64_t), cmp_u64);
    int64_t nd = 0;
    for (int64_t i = 0; i < na; i++)
        if (nd == 0 || arcs[i] != arcs[nd - 1]) arcs[nd++] = arcs[i];
    /* degree-descending relabel, ties by original id */
    deg_id* di = (deg_id*)malloc(sizeof(deg_id) * (size_t)(n ? n : 1));
    g->perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    if (!di || !g->perm) return -2;
    for (int64_t u = 0; u < n; u++) { di[u].deg = 0; di[u].id = u; }
    for (int64_t i = 0; i < nd; i++) di[arcs[i] >> 32].deg++;
    qsort(di, (size_t)n, sizeof(deg_id), cmp_deg_id);
    for (int64_t r = 0; r < n; r++) g->perm[di[r].id] = (int32_t)r;
    free(di);
    for (int64_t i = 0; i < nd; i++) {
        uint64_t u = (uint64_t)g->perm[arcs[i] >> 32], v = (uint64_t)g->perm[(uint32_t)arcs[i]];
        arcs[i] = (u << 32) | v;
    }
    qsort(arcs, (size_t)nd, sizeof(uint64_t), cmp_u64);
    int32_t* perm = g->perm;
    int rc = fill_from_arcs(n, nd, arcs, g);
    g->perm = perm;
    free(arcs);
    return rc;
}

/* Wrap an already canonical CSR (e.g. a sparsified graph) with the derived arrays. */
int orc_from_canonical(int64_t n, const int64_t* off, const int32_t* nbr, orc_graph* g) {
    memset(g, 0, sizeof(*g));
    int64_t na = off[n];
    uint64_t* arcs = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(na + 1));
    if (!arcs) return -2;
    for (int64_t u = 0; u < n; u++)
        for (int64_t i = off[u]; i < off[u + 1]; i++) arcs[i] = ((uint64_t)u << 32) | (uint32_t)nbr[i];
    int rc = fill_from_arcs(n, na, arcs, g);
    free(arcs);
    return rc;
}
