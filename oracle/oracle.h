/*
 * CPU oracle for sampling-based approximate pattern counting (arXiv 2405.03488).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously correct
 * reference the HIP path is checked against.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no source
 * with the HIP library: its own Philox, canonicaliser, pattern compiler,
 * candidate sets, big integers, statistics and colour sparsification.
 *
 * Parity pins (see tests/test_oracle_*.py):
 *   Philox4x32-10 ...... rocRAND's host Philox4x32-10 generator (library routine)
 *   canonical graph .... invariants (symmetry, sortedness, degree order, perm)
 *   pattern compiler ... |Aut| of named patterns; restricted tuples x |Aut| equal
 *                        injective homomorphisms; the paper's 4-cycle plan (Sec. 4.2)
 *   exact counters ..... closed forms on K_n, rings, grids, hypercubes, K_ab,
 *                        Petersen, stars; degree identities; brute force
 *   NS sampler ......... exact expectation over every walk on tiny graphs equals
 *                        the brute-force count (Lemma, Sec. 4.2); k=2 zero variance
 *   statistics ......... hand-computed eps-hat; Phi^-1 against scipy
 *   colour GS .......... exhaustive colourings: mean of c^(k-1) Y equals C
 */
#ifndef SGPM_ORACLE_H
#define SGPM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Canonical graph (symmetric, loop-free, deduplicated, relabelled by degree
 * descending with ties by original id ascending, rows ascending). */
typedef struct {
    int64_t n, m;     /* vertices, undirected edges */
    int64_t* off;     /* [n+1] */
    int32_t* nbr;     /* [2m] */
    int32_t* esrc;    /* [m] oriented edge e = (esrc[e], edst[e]), edst < esrc, (u,w) order */
    int32_t* edst;    /* [m] */
    int32_t* arow;    /* [2m] row of arc a in full-CSR order */
    int32_t* perm;    /* [n] perm[original id] = canonical id (NULL for derived graphs) */
} orc_graph;

/* Compiled pattern: vertex order, per-position masks over earlier positions. */
typedef struct {
    int32_t k, induced, oriented, aut;
    int32_t order[8];      /* order[i] = pattern vertex matched at position i */
    uint8_t connect[8];    /* bit i of connect[j]: pattern edge between positions i < j */
    uint8_t disconnect[8]; /* induced only: no pattern edge between i < j */
    uint8_t upper[8];      /* bit i of upper[j]: restriction v_j < v_i */
    uint8_t lower[8];      /* bit i of lower[j]: restriction v_j > v_i */
} orc_plan;

/* One NS sample (trace record). */
typedef struct {
    uint64_t s;
    int32_t v[8];
    uint64_t size[8];      /* |S_j| for the steps that ran (size[0] = M) */
    int32_t k, hit, fail_step, overflow;
    uint64_t alpha_lo, alpha_hi;   /* X_s as a 128-bit integer (0 on a miss) */
    uint64_t bytes;        /* algorithmic bytes of this sample (measurement definition: every row merged) */
    uint64_t bytes_min;    /* the same with only the smallest connected row's entries (lower bound) */
} orc_rec;

typedef struct {
    double eps, confidence;
    uint64_t seed;
    uint32_t tag;
    int32_t nthreads;
    uint64_t fixed_n;      /* >0: one window of exactly fixed_n samples */
    uint64_t n_min, w_min, quantum, max_samples;
    double growth;
    int32_t sampler;       /* 0: NS-prune, 1: NS-base */
} orc_ns_opts;

typedef struct {
    double estimate, eps_hat, z;
    uint64_t n, hits, checksum, bytes;
    uint32_t s1[8], s2[12];   /* little-endian 32-bit digits of sum X, sum X^2 */
    int32_t windows, converged, overflow;
} orc_ns_result;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint64_t orc_draw(uint64_t seed, uint64_t s, uint32_t d, uint32_t tag);
uint64_t orc_mulhi(uint64_t n, uint64_t r);

int orc_canon(int64_t n, const int64_t* in_off, const int32_t* in_nbr, orc_graph* out);
int orc_from_canonical(int64_t n, const int64_t* off, const int32_t* nbr, orc_graph* out);
void orc_graph_free(orc_graph* g);

int orc_compile(int k, int l, const int32_t* edges, int induced, orc_plan* out);
int orc_automorphisms(int k, int l, const int32_t* edges);

void orc_brute_count(const orc_graph* g, int k, int l, const int32_t* edges, int induced,
                     uint64_t* injective_maps, uint64_t* count);
void orc_plan_count(const orc_graph* g, const orc_plan* p, int nthreads, uint64_t* lo, uint64_t* hi);
uint64_t orc_plan_count_bytes(const orc_graph* g, const orc_plan* p, int nthreads);
uint64_t orc_step_bytes(const orc_graph* g, const orc_plan* p, int j, const int32_t* v, uint32_t* opened,
                        uint64_t* min_b);
uint64_t orc_gs_count_bytes(const orc_graph* g, const orc_plan* p, uint32_t c, uint64_t seed, uint32_t rep,
                            int nthreads);

uint64_t orc_candidates(const orc_graph* g, const orc_plan* p, int j, const int32_t* v, int32_t* out);
void orc_ns_sample(const orc_graph* g, const orc_plan* p, uint64_t seed, uint32_t tag, uint64_t s,
                   const uint64_t* draws, orc_rec* r);
uint64_t orc_rec_hash(const orc_rec* r);
uint64_t orc_union_candidates(const orc_graph* g, const orc_plan* p, int j, const int32_t* v, int32_t* out);
void orc_ns_base_sample(const orc_graph* g, const orc_plan* p, uint64_t seed, uint32_t tag, uint64_t s,
                        const uint64_t* draws, orc_rec* r);
int orc_ns_base_trace(const orc_graph* g, const orc_plan* p, uint64_t seed, uint32_t tag,
                      uint64_t s0, uint64_t count, int nthreads, orc_rec* out);
int orc_ns_trace(const orc_graph* g, const orc_plan* p, uint64_t seed, uint32_t tag,
                 uint64_t s0, uint64_t count, int nthreads, orc_rec* out);
int orc_ns_run(const orc_graph* g, const orc_plan* p, const orc_ns_opts* o, orc_ns_result* r,
               double* eps_trace, uint64_t* n_trace, int trace_cap);

double orc_norm_ppf(double p);
double orc_digits_to_double(const uint32_t* d, int nd);
double orc_eps_hat(double z, uint64_t n, const uint32_t* s1, int n1, const uint32_t* s2, int n2);
double orc_t_ppf(double conf, int nu);
double orc_eps_hat_t(double t, uint64_t n, const uint32_t* s1, int n1, const uint32_t* s2, int n2);
uint64_t orc_window_next(uint64_t n_t, const orc_ns_opts* o);

typedef struct {
    double estimate, eps_hat, z;
    uint64_t reps, nonzero;
    uint32_t s1[8], s2[12];
    int32_t converged;
} orc_gs_result;

int orc_gs_run(const orc_graph* g, const orc_plan* p, uint32_t c, uint64_t seed, double eps, double confidence,
               int reps_max, int nthreads, orc_gs_result* r, uint64_t* y_per_rep);
int32_t orc_gs_colour(uint64_t seed, uint32_t rep, uint32_t c, int64_t v);
int orc_bes_keep(uint64_t seed, uint32_t rep, uint32_t c, int32_t u, int32_t w);
int orc_bes_sparsify(const orc_graph* g, uint32_t c, uint64_t seed, uint32_t rep, orc_graph* out);
void orc_bes_count(const orc_graph* g, const orc_plan* p, uint32_t c, uint64_t seed, uint32_t rep,
                   int nthreads, uint64_t* y_lo, uint64_t* y_hi);
int orc_plan_edges(const orc_plan* p);
int orc_bes_run(const orc_graph* g, const orc_plan* p, uint32_t c, uint64_t seed, double eps, double confidence,
                int reps_max, int nthreads, orc_gs_result* r, uint64_t* y_per_rep);
int orc_gs_sparsify(const orc_graph* g, const int32_t* colour, orc_graph* out);
void orc_gs_count(const orc_graph* g, const orc_plan* p, uint32_t c, uint64_t seed, uint32_t rep,
                  int nthreads, uint64_t* y_lo, uint64_t* y_hi);

int32_t orc_bucket(const orc_graph* g, int64_t v);
void orc_ns_sample_learned(const orc_graph* g, const orc_plan* p, const uint16_t* table, uint64_t seed,
                           uint32_t tag, uint64_t s, const uint64_t* draws, orc_rec* r, double* alpha_f);
double orc_bf16(double x);
void orc_learned_features(int pattern, int j, int b0, int bp, int bc, float* x);
void orc_learned_table(const float* params, int pattern, int k, int bf16, uint16_t* out);
int orc_mlp_nparams(void);
double orc_mlp(const float* params, const float* X, const float* y, int64_t N, int bf16, double* s_out,
               double* grads);

#ifdef __cplusplus
}
#endif
#endif
