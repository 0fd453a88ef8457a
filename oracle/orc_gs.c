/*
 * Oracle (test infrastructure only): colour sparsification (GS path).
 *
 * Sec. 2.2 (subgraph sampling) and Sec. 5.2: colour every vertex uniformly
 * with one of c colours, keep only edges whose endpoints share a colour, count
 * the pattern exactly on the sparsified graph G' and scale.  For a connected
 * k-vertex pattern a match survives only when all k vertices share a colour,
 * which happens with probability c^(1-k); so the estimate is c^(k-1) * Y with
 * Y the exact count on G'.  (The paper writes the exponent with the number of
 * pattern edges; the two agree only for cycles.  The exhaustive-colouring test
 * settles the exponent.)  G' is the disjoint union of the colour classes, so
 * counting on G' equals summing over the classes.
 *
 * colour(v) = floor(c * r / 2^64) with r the Philox value of key = seed,
 * counter = (v mod 2^32, v div 2^32, 0, 0x40000000 | rep) on canonical ids.
 */
#include "oracle.h"
#include <stdlib.h>
#include <string.h>

int32_t orc_gs_colour(uint64_t seed, uint32_t rep, uint32_t c, int64_t v) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)v, (uint32_t)((uint64_t)v >> 32), 0u, 0x40000000u | rep};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    uint64_t r = ((uint64_t)out[1] << 32) | out[0];
    return (int32_t)orc_mulhi(c, r);
}

int orc_gs_sparsify(const orc_graph* g, const int32_t* colour, orc_graph* out) {
    int64_t n = g->n;
    int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * g->m + 1));
    if (!off || !nbr) return -2;
    int64_t w = 0;
    for (int64_t u = 0; u < n; u++) {
        for (int64_t e = g->off[u]; e < g->off[u + 1]; e++)
            if (colour[g->nbr[e]] == colour[u]) nbr[w++] = g->nbr[e];
        off[u + 1] = w;
    }
    int rc = orc_from_canonical(n, off, nbr, out);
    free(off);
    free(nbr);
    return rc;
}

void orc_gs_count(const orc_graph* g, const orc_plan* p, uint32_t c, uint64_t seed, uint32_t rep,
                  int nthreads, uint64_t* y_lo, uint64_t* y_hi) {
    int32_t* colour = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->n ? g->n : 1));
    for (int64_t v = 0; v < g->n; v++) colour[v] = orc_gs_colour(seed, rep, c, v);
    orc_graph sp;
    orc_gs_sparsify(g, colour, &sp);
    orc_plan_count(&sp, p, nthreads, y_lo, y_hi);
    orc_graph_free(&sp);
    free(colour);
}

/* the exact search's algorithmic bytes on colouring rep of the colour scheme */
uint64_t orc_gs_count_bytes(const orc_graph* g, const orc_plan* p, uint32_t c, uint64_t seed, uint32_t rep,
                            int nthreads) {
    int32_t* colour = (int32_t*)malloc(sizeof(int32_t) * (size_t)(g->n ? g->n : 1));
    for (int64_t v = 0; v < g->n; v++) colour[v] = orc_gs_colour(seed, rep, c, v);
    orc_graph sp;
    orc_gs_sparsify(g, colour, &sp);
    uint64_t b = orc_plan_count_bytes(&sp, p, nthreads);
    orc_graph_free(&sp);
    free(colour);
    return b;
}

/* Bernoulli edge sparsification (Sec. 2.2, the edge-sparsification algorithm
 * and the GS trade-off section): every edge is kept independently with
 * probability p = 1/c, so a match with l pattern edges survives with
 * probability p^l and the estimate is c^l * Y.  Non-edges are not preserved,
 * so only edge-induced patterns (no disconnect constraint) qualify.
 * keep({a, b}) with a > b: floor(c * r / 2^64) == 0, r the Philox value of
 * key = seed, counter = (a, b, 0, 0x20000000 | rep). */
int orc_bes_keep(uint64_t seed, uint32_t rep, uint32_t c, int32_t u, int32_t w) {
    uint32_t a = (uint32_t)(u > w ? u : w), b = (uint32_t)(u > w ? w : u);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {a, b, 0u, 0x20000000u | rep};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    uint64_t r = ((uint64_t)out[1] << 32) | out[0];
    return orc_mulhi(c, r) == 0;
}

int orc_bes_sparsify(const orc_graph* g, uint32_t c, uint64_t seed, uint32_t rep, orc_graph* out) {
    int64_t n = g->n;
    int64_t* off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * g->m + 1));
    if (!off || !nbr) return -2;
    int64_t w = 0;
    for (int64_t u = 0; u < n; u++) {
        for (int64_t e = g->off[u]; e < g->off[u + 1]; e++)
            if (orc_bes_keep(seed, rep, c, (int32_t)u, g->nbr[e])) nbr[w++] = g->nbr[e];
        off[u + 1] = w;
    }
    int rc = orc_from_canonical(n, off, nbr, out);
    free(off);
    free(nbr);
    return rc;
}

void orc_bes_count(const orc_graph* g, const orc_plan* p, uint32_t c, uint64_t seed, uint32_t rep,
                   int nthreads, uint64_t* y_lo, uint64_t* y_hi) {
    orc_graph sp;
    orc_bes_sparsify(g, c, seed, rep, &sp);
    orc_plan_count(&sp, p, nthreads, y_lo, y_hi);
    orc_graph_free(&sp);
}

/* pattern edges of a compiled plan */
int orc_plan_edges(const orc_plan* p) {
    int l = 0;
    for (int j = 1; j < p->k; j++) l += __builtin_popcount(p->connect[j]);
    return l;
}

/* GS estimate over repeated colourings: X_r = c^(k-1) * Y_r for rep r = 0, 1, ...
 * are i.i.d. unbiased estimates of the count.  The paper gives GS no online
 * confidence interval (Sec. 4.4 bounds its variance; Sec. 5.1 gives loose mode
 * no guarantee), and n is small here (a few colourings), so the interval is the
 * Student t interval of their mean: eps_hat = t_{n-1} sqrt(D / (n - 1)) / S1
 * with D = n S2 - S1^2, the unbiased variance and t_{n-1} the two-sided
 * quantile at the requested confidence.  Stop at the first n >= 3 with
 * eps_hat <= eps, or after reps_max colourings: two colourings of a small or
 * skewed count often give equal values, a zero variance and an interval of
 * width zero, so the test starts at the third. */
static void add_digits(uint32_t* acc, int nd, const uint64_t* cols, int nc) {
    unsigned __int128 carry = 0;
    for (int i = 0; i < nd; i++) {
        unsigned __int128 t = carry + acc[i];
        if (i < nc) t += cols[i];
        acc[i] = (uint32_t)t;
        carry = t >> 32;
    }
}

static int gs_run_scheme(const orc_graph* g, const orc_plan* p, uint32_t c, uint64_t seed, double eps,
                         double confidence, int reps_max, int nthreads, orc_gs_result* r, uint64_t* y_per_rep,
                         int bes) {
    memset(r, 0, sizeof(*r));
    double z = orc_t_ppf(confidence, 1);
    unsigned __int128 scale = 1;
    int expo = bes ? orc_plan_edges(p) : p->k - 1;
    for (int i = 0; i < expo; i++) scale *= c;
    for (int rep = 0; rep < reps_max; rep++) {
        uint64_t lo, hi;
        if (bes) orc_bes_count(g, p, c, seed, (uint32_t)rep, nthreads, &lo, &hi);
        else orc_gs_count(g, p, c, seed, (uint32_t)rep, nthreads, &lo, &hi);
        if (y_per_rep) y_per_rep[rep] = lo;
        unsigned __int128 y = ((unsigned __int128)hi << 64) | lo;
        unsigned __int128 x = y * scale;
        uint64_t d[4], sq[8];
        for (int i = 0; i < 4; i++) d[i] = (uint32_t)(x >> (32 * i));
        memset(sq, 0, sizeof(sq));
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) {
                uint64_t pr = d[a] * d[b];
                sq[a + b] += pr & 0xFFFFFFFFu;
                if (a + b + 1 < 8) sq[a + b + 1] += pr >> 32;
            }
        add_digits(r->s1, 8, d, 4);
        add_digits(r->s2, 12, sq, 8);
        r->reps++;
        if (y) r->nonzero++;
        if (r->reps >= 2) z = orc_t_ppf(confidence, (int)r->reps - 1);
        r->eps_hat = orc_eps_hat_t(z, r->reps, r->s1, 8, r->s2, 12);
        if (r->reps >= 3 && r->eps_hat <= eps) { r->converged = 1; break; }
    }
    /* estimate = S1 / n with S1 rounded once */
    r->estimate = orc_digits_to_double(r->s1, 8) / (double)r->reps;
    r->z = z;
    return 0;
}

int orc_gs_run(const orc_graph* g, const orc_plan* p, uint32_t c, uint64_t seed, double eps, double confidence,
               int reps_max, int nthreads, orc_gs_result* r, uint64_t* y_per_rep) {
    return gs_run_scheme(g, p, c, seed, eps, confidence, reps_max, nthreads, r, y_per_rep, 0);
}

/* The same over repeated Bernoulli edge sparsifications: X_r = c^l * Y_r. */
int orc_bes_run(const orc_graph* g, const orc_plan* p, uint32_t c, uint64_t seed, double eps, double confidence,
                int reps_max, int nthreads, orc_gs_result* r, uint64_t* y_per_rep) {
    return gs_run_scheme(g, p, c, seed, eps, confidence, reps_max, nthreads, r, y_per_rep, 1);
}
