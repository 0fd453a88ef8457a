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
