/*
 * Seeded synthetic graph generators (input synthesis only).
 *
 * This module produces the raw edge lists that both the HIP path and the CPU
 * oracle consume.  It holds none of the estimator's arithmetic: no Philox, no
 * canonical relabelling, no counting.  Its random numbers come from a
 * counter-based SplitMix64 stream (Steele, Lea, Flood, OOPSLA 2014): the
 * i-th value of stream `st` under `seed` is mix64(base(seed, st) + (i+1)*G),
 * G = 0x9E3779B97F4A7C15, so every generator is reproducible and can be split
 * over threads by index range without changing its output.
 *
 * Generators (the paper's inputs are real SNAP/web graphs, which these stand in
 * for; see the input recipe in the design notes):
 *   - Erdos-Renyi G(n, M): M distinct non-loop unordered pairs, drawn with
 *     rejection of repeats and loops, in draw order.
 *   - R-MAT (Chakrabarti, Zhan, Faloutsos 2004): per pair and level one uniform
 *     double in [0,1) picks a quadrant against cumulative (a, a+b, a+b+c).
 *   - Chung-Lu power law: weight_i = (i+1)^(-1/(gamma-1)); n*d/2 pairs with both
 *     endpoints drawn proportional to weight (Walker/Vose alias table).
 * Output: int32 pairs (u, v) as generated (duplicates and loops possible for
 * R-MAT and Chung-Lu); pairs_to_csr() packs them into a raw, unsorted CSR.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>

#define SX_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sx_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t sx_base(uint64_t seed, uint64_t stream) {
    return sx_mix(seed ^ sx_mix(stream * 0xD1B54A32D192ED03ULL + 0x632BE59BD9B4E019ULL));
}
static inline uint64_t sx_at(uint64_t base, uint64_t i) { return sx_mix(base + (i + 1) * SX_GAMMA); }
static inline uint64_t sx_below(uint64_t n, uint64_t r) {
    return (uint64_t)(((unsigned __int128)n * r) >> 64);
}
static inline double sx_unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* ---------------------------------------------------------------- ER G(n,M) */
/* open-addressing set of unordered pairs */
int64_t sgpm_gen_er(int64_t n, int64_t M, uint64_t seed, int32_t* out_pairs) {
    if (n < 2 || M < 0 || M > n * (n - 1) / 2) return -1;
    uint64_t cap = 1;
    while (cap < (uint64_t)M * 2 + 16) cap <<= 1;
    uint64_t* tab = (uint64_t*)calloc(cap, sizeof(uint64_t));
    if (!tab) return -2;
    uint64_t base = sx_base(seed, 1);
    int64_t got = 0;
    uint64_t i = 0;
    while (got < M) {
        uint64_t u = sx_below((uint64_t)n, sx_at(base, i++));
        uint64_t v = sx_below((uint64_t)n, sx_at(base, i++));
        if (u == v) continue;
        uint64_t a = u < v ? u : v, b = u < v ? v : u;
        uint64_t key = (a << 32 | b) + 1; /* never 0 */
        uint64_t h = sx_mix(key) & (cap - 1);
        int dup = 0;
        while (tab[h]) {
            if (tab[h] == key) { dup = 1; break; }
            h = (h + 1) & (cap - 1);
        }
        if (dup) continue;
        tab[h] = key;
        out_pairs[2 * got] = (int32_t)u;
        out_pairs[2 * got + 1] = (int32_t)v;
        got++;
    }
    free(tab);
    return got;
}

/* ---------------------------------------------------------------- R-MAT */
typedef struct {
    int scale; int64_t lo, hi; double a, ab, abc; uint64_t base; int32_t* out;
} rmat_job;

static void* rmat_worker(void* p) {
    rmat_job* j = (rmat_job*)p;
    for (int64_t e = j->lo; e < j->hi; e++) {
        uint64_t u = 0, v = 0;
        for (int l = 0; l < j->scale; l++) {
            double x = sx_unit(sx_at(j->base, (uint64_t)e * (uint64_t)j->scale + (uint64_t)l));
            uint64_t bu, bv;
            if (x < j->a) { bu = 0; bv = 0; }
            else if (x < j->ab) { bu = 0; bv = 1; }
            else if (x < j->abc) { bu = 1; bv = 0; }
            else { bu = 1; bv = 1; }
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        j->out[2 * e] = (int32_t)u;
        j->out[2 * e + 1] = (int32_t)v;
    }
    return NULL;
}

int64_t sgpm_gen_rmat(int scale, int64_t npairs, double a, double b, double c, uint64_t seed,
                      int32_t* out_pairs, int nthreads) {
    if (scale < 1 || scale > 30 || npairs < 0) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    pthread_t th[64];
    rmat_job jobs[64];
    uint64_t base = sx_base(seed, 2);
    for (int t = 0; t < nthreads; t++) {
        jobs[t].scale = scale;
        jobs[t].lo = npairs * t / nthreads;
        jobs[t].hi = npairs * (t + 1) / nthreads;
        jobs[t].a = a; jobs[t].ab = a + b; jobs[t].abc = a + b + c;
        jobs[t].base = base; jobs[t].out = out_pairs;
        pthread_create(&th[t], NULL, rmat_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    return npairs;
}

/* ---------------------------------------------------------------- Chung-Lu */
typedef struct {
    int64_t n, lo, hi; const double* prob; const int32_t* alias; uint64_t base; int32_t* out;
} cl_job;

static inline int32_t cl_draw(const cl_job* j, uint64_t i) {
    uint64_t r1 = sx_at(j->base, 2 * i), r2 = sx_at(j->base, 2 * i + 1);
    int64_t col = (int64_t)sx_below((uint64_t)j->n, r1);
    return sx_unit(r2) < j->prob[col] ? (int32_t)col : j->alias[col];
}

static void* cl_worker(void* p) {
    cl_job* j = (cl_job*)p;
    for (int64_t e = j->lo; e < j->hi; e++) {
        j->out[2 * e] = cl_draw(j, 2 * (uint64_t)e);
        j->out[2 * e + 1] = cl_draw(j, 2 * (uint64_t)e + 1);
    }
    return NULL;
}

int64_t sgpm_gen_chung_lu(int64_t n, int64_t npairs, double gamma, uint64_t seed,
                          int32_t* out_pairs, int nthreads) {
    if (n < 2 || npairs < 0 || gamma <= 1.0) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    double* w = (double*)malloc(sizeof(double) * n);
    double* prob = (double*)malloc(sizeof(double) * n);
    int32_t* alias = (int32_t*)malloc(sizeof(int32_t) * n);
    int64_t* small = (int64_t*)malloc(sizeof(int64_t) * n);
    int64_t* large = (int64_t*)malloc(sizeof(int64_t) * n);
    if (!w || !prob || !alias || !small || !large) return -2;
    double ex = -1.0 / (gamma - 1.0), tot = 0.0;
    for (int64_t i = 0; i < n; i++) { w[i] = pow((double)(i + 1), ex); tot += w[i]; }
    int64_t ns = 0, nl = 0;
    for (int64_t i = 0; i < n; i++) {
        w[i] = w[i] * (double)n / tot; /* scaled so the mean is 1 */
        alias[i] = (int32_t)i;
        if (w[i] < 1.0) small[ns++] = i; else large[nl++] = i;
    }
    while (ns > 0 && nl > 0) {
        int64_t s = small[--ns], l = large[--nl];
        prob[s] = w[s];
        alias[s] = (int32_t)l;
        w[l] = (w[l] + w[s]) - 1.0;
        if (w[l] < 1.0) small[ns++] = l; else large[nl++] = l;
    }
    while (nl > 0) prob[large[--nl]] = 1.0;
    while (ns > 0) prob[small[--ns]] = 1.0;
    pthread_t th[64];
    cl_job jobs[64];
    uint64_t base = sx_base(seed, 3);
    for (int t = 0; t < nthreads; t++) {
        jobs[t].n = n; jobs[t].lo = npairs * t / nthreads; jobs[t].hi = npairs * (t + 1) / nthreads;
        jobs[t].prob = prob; jobs[t].alias = alias; jobs[t].base = base; jobs[t].out = out_pairs;
        pthread_create(&th[t], NULL, cl_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(w); free(prob); free(alias); free(small); free(large);
    return npairs;
}

/* ---------------------------------------------------------------- packing */
/* Raw CSR: row u lists every v of every pair (u, v), in pair order.  No
 * symmetrisation, dedupe or sorting: that is the consumer's canonicalisation. */
int sgpm_pairs_to_csr(int64_t n, int64_t npairs, const int32_t* pairs, int64_t* off, int32_t* nbr) {
    memset(off, 0, sizeof(int64_t) * (n + 1));
    for (int64_t e = 0; e < npairs; e++) {
        int32_t u = pairs[2 * e];
        if (u < 0 || u >= n) return -1;
        off[u + 1]++;
    }
    for (int64_t i = 0; i < n; i++) off[i + 1] += off[i];
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
    if (!cur) return -2;
    memcpy(cur, off, sizeof(int64_t) * (n + 1));
    for (int64_t e = 0; e < npairs; e++) nbr[cur[pairs[2 * e]]++] = pairs[2 * e + 1];
    free(cur);
    return 0;
}
