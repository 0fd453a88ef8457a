/*
 * sgpm.h -- C-ABI of the MI355X library for sampling-based approximate graph
 * pattern counting (arXiv 2405.03488, "Accurate and Fast Approximate Graph
 * Pattern Mining at Scale").
 *
 * Problem statement (Sec. 2.1): given a data graph G and a pattern P, return an
 * estimate of the number of edge-induced (subgraph counting) or vertex-induced
 * (motif counting) occurrences of P in G that lies within a factor (1 +- eps)
 * of the true count with probability at least 1 - delta.
 *
 * Conventions for every call:
 *   - Every function returns sgpm_status (0 = success, < 0 = error) and never
 *     throws across the ABI.  A failing call leaves its outputs untouched
 *     unless stated otherwise; sgpm_last_error() gives a message.
 *   - Pointers are host pointers unless a flag says otherwise.  Caller-owned
 *     arrays are only read during the call; the library copies what it keeps.
 *   - Handles (sgpm_graph_t, sgpm_pattern_t, sgpm_model_t) are owned by the
 *     library until the matching *_free; each belongs to the context that made
 *     it.  One context per host thread.
 *   - All device work runs on the context's HIP stream; calls return after
 *     their results are final (no asynchronous outputs).
 *   - Sample ids, random draws and integer sums are deterministic: the same
 *     inputs and seed give bit-identical walks, sums and checksums regardless
 *     of launch configuration.
 */
#ifndef SGPM_H
#define SGPM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SGPM_OK = 0,
    SGPM_EINVAL = -1,          /* bad argument (null pointer, out-of-range option) */
    SGPM_ENOMEM = -2,          /* host or device allocation failed */
    SGPM_EHIP = -3,            /* a HIP runtime call failed */
    SGPM_EUNSUPPORTED = -4,    /* k < 2, k > 8, disconnected pattern, unsupported mode */
    SGPM_NOT_CONVERGED = -5,   /* max_samples reached before eps_hat <= eps; result IS filled */
    SGPM_EBADGRAPH = -6,       /* malformed CSR, or non-canonical input with SGPM_ASSUME_CANONICAL */
    SGPM_EOVERFLOW = -7        /* a sample weight exceeded 128 bits */
} sgpm_status;

typedef struct sgpm_ctx* sgpm_ctx_t;
typedef struct sgpm_graph* sgpm_graph_t;
typedef struct sgpm_pattern* sgpm_pattern_t;
typedef struct sgpm_model* sgpm_model_t;

/* ------------------------------------------------------------------ context */

/* Create a context bound to HIP device `hip_device` and stream `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  The stream must outlive
 * the context.  One context per host thread: calls on a context must not
 * overlap. */
sgpm_status sgpm_create(sgpm_ctx_t* out, int hip_device, void* hip_stream);
/* Release the context and the device memory it keeps between calls: the NS
 * engine's partial-sum and ticket buffers, the batch's capture and query
 * table, and the GS engine's grow-only scratch (about 25 bytes per vertex of
 * the largest graph sparsified, plus 32 bytes per 2,048 arcs).  Free the
 * context's graphs, patterns and models first. */
sgpm_status sgpm_destroy(sgpm_ctx_t ctx);
/* Message of the last failing call on ctx; valid until the next call on ctx. */
const char* sgpm_last_error(sgpm_ctx_t ctx);
/* Number of HIP devices visible (0 on a host without GPUs); never fails. */
int sgpm_device_count(void);

/* ------------------------------------------------------------------ graphs */

#define SGPM_ASSUME_CANONICAL 0x1u  /* input is already symmetric, loop-free, deduplicated,
                                       degree-descending relabelled with ascending rows */
#define SGPM_DEVICE_PTRS 0x2u       /* offsets and nbrs are device pointers (e.g. torch tensors'
                                       data) on the context's device */
#define SGPM_SYMMETRIZE 0x4u        /* the default made explicit: symmetrise and clean the input;
                                       not with SGPM_ASSUME_CANONICAL */

/* Build the canonical data graph (Sec. 6: symmetric, no loops or duplicate
 * edges; vertices relabelled by degree descending, ties by original id; rows
 * ascending) from a CSR of n vertices.  offsets has n+1 entries, int64 when
 * offsets_is_64 else int32; nbrs has offsets[n] int32 entries in [0, n).
 * Without SGPM_ASSUME_CANONICAL every (u, v) entry is symmetrised, loops and
 * duplicates are dropped.  With SGPM_DEVICE_PTRS the arrays are read from
 * device memory (the caller keeps them alive during the call): they are copied
 * to the host, where the canonicalisation runs, and the result is uploaded as
 * for host arrays.  The canonical CSR, the oriented edge list and the arc-row
 * array are kept in device memory owned by the graph handle.
 * Errors: EINVAL (null pointers, n < 0 or n >= 2^31, unknown flags, or
 * SGPM_SYMMETRIZE with SGPM_ASSUME_CANONICAL), EBADGRAPH (offsets not
 * monotone, neighbour id out of range, or a non-canonical input with
 * SGPM_ASSUME_CANONICAL), ENOMEM, EHIP (a device copy failed). */
sgpm_status sgpm_graph_from_csr(sgpm_ctx_t ctx, int64_t n, const void* offsets, int offsets_is_64,
                                const int32_t* nbrs, uint32_t flags, sgpm_graph_t* out);
/* Sizes of the canonical graph (Sec. 6, the data-graph table: |V|, |E| of the
 * symmetrised, loop-free graph, and the maximum degree that the sampling cost
 * depends on, Sec. 4.3): *n vertices, *m undirected edges, *max_deg (each
 * nullable); perm_out (nullable, n entries) receives perm[original id] =
 * canonical id.  EINVAL for a null graph. */
sgpm_status sgpm_graph_stats(sgpm_graph_t g, int64_t* n, int64_t* m, int64_t* max_deg, int32_t* perm_out);
/* Copy the canonical CSR to host arrays off_out[n+1], nbr_out[2m] (either nullable). */
sgpm_status sgpm_graph_export(sgpm_graph_t g, int64_t* off_out, int32_t* nbr_out);
sgpm_status sgpm_graph_free(sgpm_graph_t g);

/* ------------------------------------------------------------------ patterns */

/* Compile pattern P (k vertices, l edges given as pairs of ids in [0, k)) into
 * the matching order and symmetry-breaking restrictions of NS-prune (Sec. 4.2).
 * induced = 0: edge-induced (subgraph counting); 1: vertex-induced (motifs).
 * Errors: EINVAL (bad pointers or edge ids), EUNSUPPORTED (k < 2, k > 8, or P
 * disconnected). */
sgpm_status sgpm_pattern_create(sgpm_ctx_t ctx, int k, int l, const int32_t* edges, int induced,
                                sgpm_pattern_t* out);
/* The compiled plan: order[i] = pattern vertex at position i; per position j a
 * bit i < j of connect[j] is a pattern edge (i, j), of disconnect[j] a pattern
 * non-edge checked for vertex-induced counting, of upper[j] the restriction
 * v_j < v_i and of lower[j] the restriction v_j > v_i.  oriented = 1 when the
 * first edge is drawn from the m edges with v0 > v1 (alpha starts at m), else
 * from the 2m arcs.  All outputs are arrays of k entries (any may be NULL). */
sgpm_status sgpm_pattern_plan(sgpm_pattern_t p, int32_t* order, uint8_t* connect, uint8_t* disconnect,
                              uint8_t* upper, uint8_t* lower, int32_t* aut_size, int32_t* oriented);
sgpm_status sgpm_pattern_free(sgpm_pattern_t p);

/* ------------------------------------------------------------------ estimation */

enum {
    SGPM_MODE_STRICT_NS = 0,   /* NS-prune with online convergence (Sec. 4.1, 5.1 strict mode) */
    SGPM_MODE_FIXED_N = 1,     /* exactly fixed_n NS samples, no stop rule */
    SGPM_MODE_GS = 2,          /* colour sparsification + exact count, repeated colourings */
    SGPM_MODE_HYBRID = 3       /* loose mode: choose NS or GS from pilot costs (Sec. 5.1); the
                                  result equals that engine's own result (same options) */
};
enum { SGPM_SCHEME_NS = 0, SGPM_SCHEME_GS = 1, SGPM_SCHEME_EXACT = 2 };
enum {
    SGPM_GS_COLOUR = 0,        /* colour sparsification, estimate c^(k-1) Y (Sec. 2.2, 5.2) */
    SGPM_GS_BERNOULLI = 1      /* Bernoulli edge sparsification (Sec. 2.2): every edge kept with probability
                                  1/c, decided per undirected edge {a > b} by Philox(key seed, counter
                                  (a, b, 0, 0x20000000 | rep)); estimate c^l Y with l pattern edges;
                                  edge-induced patterns only (EUNSUPPORTED otherwise); SGPM_MODE_GS only */
};
enum {
    SGPM_SAMPLER_PRUNE = 0,    /* NS-prune: eager verification, candidate sets filtered at every step (Sec. 4.2) */
    SGPM_SAMPLER_BASE = 1      /* NS-base: the sampler the paper compares against (Sec. 4.2): position j drawn
                                  from the union of the joined positions' rows (alpha *= its size, union
                                  enumerated by ascending position, each row ascending, first occurrences),
                                  every test deferred to a closure check after the last draw; a failed closure
                                  is a miss with status k */
};

/* One NS sample as recorded by the trace option (64 bytes). status = 0xFF for a
 * hit, else the position j whose candidate set was empty; v[i] = -1 for
 * positions not reached; alpha = X_s (0 on a miss). */
typedef struct {
    uint64_t s;
    int32_t v[8];
    uint32_t status;
    uint32_t k;
    uint64_t alpha_lo, alpha_hi;
} sgpm_trace_rec;

typedef struct {
    double eps;              /* relative error bound, e.g. 0.01 */
    double confidence;       /* 1 - delta, e.g. 0.95 */
    uint64_t seed;           /* Philox key */
    uint32_t query_tag;      /* Philox counter word 3; distinct tags give independent streams */
    int32_t mode;            /* SGPM_MODE_* */
    uint64_t fixed_n;        /* SGPM_MODE_FIXED_N sample count */
    uint64_t n_min;          /* first window end (rounded up to quantum); > 0 in NS and hybrid modes */
    uint64_t w_min;          /* smallest window */
    uint64_t quantum;        /* window ends are multiples of this */
    uint64_t max_samples;    /* hard cap (NOT_CONVERGED when reached) */
    double window_growth;    /* next window = max(w_min, ceil(growth * n)) */
    int32_t colours;         /* GS: colours c in [1, 256], or 0 = choose c in 4..16 from one probe colouring
                                (see sgpm_host_colours_choice; the Bernoulli scheme takes 8); < 0 or > 256
                                is EINVAL */
    int32_t gs_reps_max;     /* GS: cap on repeated colourings */
    sgpm_model_t proposal;   /* NULL = uniform proposal */
    int32_t lanes_per_sample;/* 0 = autotune, else 1, 4, 16 or 64 lanes cooperate on one sample */
    int32_t checksum;        /* 1 = fold every sample record into result.checksum */
    uint64_t trace_lo, trace_hi; /* record samples with trace_lo <= s < trace_hi ... */
    sgpm_trace_rec* trace_buf;   /* ... into this host array of trace_hi - trace_lo records */
    int32_t sampler;         /* SGPM_SAMPLER_*: NS-prune (default) or NS-base; NS-base runs in the strict
                                and fixed-n modes only, with the uniform proposal and no byte count */
    int32_t gs_scheme;       /* SGPM_GS_*: the sparsifier of SGPM_MODE_GS */
    int32_t hybrid_selector; /* SGPM_HYBRID_*: how loose mode chooses between NS and GS */
} sgpm_options;

enum {
    SGPM_HYBRID_PILOTS = 0,    /* timed NS and GS pilots predict both engines' times (default) */
    SGPM_HYBRID_COST_MODEL = 1 /* the paper's profiler (10 % sparsified graph, NS-online to 50 % at 99 %,
                                  Sec. 5.3) with the NS performance cone (Sec. 4.3) and the GS cost model
                                  (Sec. 4.4); NS then runs with windows of 10 % of the predicted samples
                                  (Sec. 5.4); see sgpm_host_cost_model */
};

typedef struct {
    double estimate;         /* mu = S1 / n (NS) or the mean of c^(k-1) Y over colourings (GS) */
    double eps_hat;          /* predicted relative error (error equation, Sec. 4.1); +inf if S1 = 0.  GS:
                                t_{n-1} sqrt((n S2 - S1^2) / (n - 1)) / S1 over the n sparsifications */
    double ci_lo, ci_hi;     /* mu -+ z sigma */
    double z;                /* NS: Phi^-1(1 - delta/2); GS: the Student t quantile with n - 1 degrees of
                                freedom at the same two-sided confidence */
    uint64_t n_samples, n_hits;
    uint32_t sum_digits[8];  /* S1 = sum X, little-endian 32-bit digits */
    uint32_t sumsq_digits[12]; /* S2 = sum X^2 */
    int32_t scheme;          /* SGPM_SCHEME_* */
    int32_t colours;
    int32_t converged;
    int32_t windows;
    int32_t lanes_per_sample;/* launch configuration used */
    int32_t launches;        /* sampling-kernel launches */
    uint64_t checksum;       /* sum over samples of the record hash, mod 2^64 (0 unless requested) */
    uint64_t bytes;          /* algorithmic bytes of all samples (0 unless requested) */
    double seconds_sampling; /* device time of the windows (kernels, reductions, read-back) */
    double seconds_total;    /* wall time of the call */
    double seconds_kernel;   /* device time of the sampling kernels alone (HIP events around each) */
    int32_t tile;            /* batch: samples per ticket picked by the autotuner */
    int32_t weight_shift;    /* sums are of X * 2^weight_shift (52 with a learned proposal, else 0) */
    int32_t reserved0;
    /* hybrid mode: predicted NS time range (the pilot slices' min and max), the
     * predicted GS time (+inf when GS cannot meet eps), and the pilots' wall time */
    double pred_ns_lo, pred_ns_hi, pred_gs;
    double seconds_pilot;
    /* NS: device time during which at least one sampling kernel of the call ran
     * (the union of their intervals; below seconds_kernel when windows queued
     * ahead overlap on the second stream) */
    double seconds_kernel_busy;
    /* loose mode with SGPM_HYBRID_COST_MODEL: the samples the profiler predicts NS needs */
    double pred_samples;
} sgpm_result;

/* Defaults: eps 0.01, confidence 0.95, seed 1, tag 0, strict NS, n_min = w_min =
 * 2^19 (a few passes of the device's waves, so that a window's slowest samples
 * do not set its length), quantum 2^16, max_samples 2^40, growth 0.10, colours
 * 0, reps 64, lanes 0 (autotuned on the first window of 2^19 samples or more;
 * one sample per wave before that), no checksum, no trace. */
void sgpm_options_default(sgpm_options* o);

/* Estimate the count of P in G (Sec. 4-5).  Strict mode draws NS-prune samples
 * in windows [n_t, n_{t+1}) of sample ids and stops at the first window end
 * with eps_hat <= eps (NS-online algorithm); every window's integer sums are
 * exact, so results do not depend on the launch configuration.
 * Returns NOT_CONVERGED (result filled) when max_samples is reached. */
sgpm_status sgpm_estimate(sgpm_ctx_t ctx, sgpm_graph_t g, sgpm_pattern_t p, const sgpm_options* o,
                          sgpm_result* res);

/* sgpm_estimate in the NS modes with result.bytes filled: the algorithmic bytes
 * of every sample (8 for the first edge, 16 per earlier vertex whose row a step
 * reads, 4 per entry of every row the step merges -- its connected rows and,
 * vertex-induced, its disconnected rows -- inside the step's bounds; Sec. 4.2
 * set operations, Sec. 4.3 work per sample).  Uses an instrumented build of the
 * sampling kernel; for measurement. */
sgpm_status sgpm_estimate_counted(sgpm_ctx_t ctx, sgpm_graph_t g, sgpm_pattern_t p, const sgpm_options* o,
                                  sgpm_result* res);

/* Estimate nq queries (graphs[i], patterns[i], opts[i]) in one persistent,
 * hipGraph-captured launch; each query keeps its own windows and stop rule
 * (Sec. 4.1 NS-online, with the window barrier of Sec. 5.4 taken on the device)
 * and its result equals the solo sgpm_estimate result bit for bit.  Queries are
 * NS-prune, strict or fixed-n, uniform proposal, no trace (else EUNSUPPORTED).
 * Per query an autotuner picks the lanes per sample (opts[i].lanes_per_sample,
 * or the solo estimate's choice for that graph and pattern, or timed pilot
 * samples on the query's pilot stream at 64, 16, 4, 1) and the tile of samples
 * per ticket; result.lanes_per_sample and result.tile report them.  Graphs,
 * patterns and options stay owned by the caller; res[nq] is filled.  EINVAL on
 * bad arguments (nq <= 0, null handles, lanes not in {0, 1, 4, 16, 64}). */
sgpm_status sgpm_estimate_batch(sgpm_ctx_t ctx, int nq, const sgpm_graph_t* graphs,
                                const sgpm_pattern_t* patterns, const sgpm_options* opts, sgpm_result* res);

/* Exact count of P in G: the plan-driven nested-loop search of the GS engine
 * (Sec. 4.4: one loop per pattern vertex over its candidate set, formed by set
 * intersections; Sec. 5.2: the exact search that runs on each sparsified
 * graph) on the unsparsified graph, which is colour sparsification with one
 * colour.  The count is (count_hi << 64) | count_lo (count_hi nullable).
 * Errors: EINVAL (null ctx, graph, pattern or count_lo), EHIP.
 * The same count is reached three ways: the 4-, 5- and 6-clique by bitmaps
 * over each first edge's common lower neighbourhood; the wedge, 3-star,
 * 4-path, tailed triangle and diamond (edge- and vertex-induced; the induced
 * 4-path and 4-cycle with the 4-cycles' search) by closed forms over per-edge
 * common-neighbour counts and degrees; every other pattern by the search, at
 * 8, 16 or 64 lanes per first edge chosen from the pattern and the graph's
 * mean and maximum degree.  The environment variable SGPM_EXACT_GROUP (8, 16
 * or 64) sends every pattern to the search at that width.  The count does not
 * depend on the way or the width. */
sgpm_status sgpm_exact_count(sgpm_ctx_t ctx, sgpm_graph_t g, sgpm_pattern_t p, uint64_t* count_lo,
                             uint64_t* count_hi);

/* For callers that cannot allocate memory during the call (tight serving
 * loops, harnesses that forbid allocation): sgpm_exact_count without any
 * hipMalloc, hipFree or other allocating routine.  Like sgpm_exact_count it
 * synchronises the context's stream to read its counts back, so it is not for
 * use under stream capture.  The count's scratch (block partials, its ticket
 * counters and sums, and the list of first edges that the clique bitmaps pass
 * on) lives in one file-scope device array per GPU of about 8 MiB, reserved
 * when the library is loaded and held until the process ends; its device
 * address is looked up on the first call on each device.  The kernels, widths
 * and ticket plans are sgpm_exact_count's, so the count is the same; where the
 * array's list (2^21 first edges) could not hold a pass's list, cliques go to
 * the general search instead of that bitmap pass, which counts the same
 * tuples.  A launch needing more than 4,096 blocks of partials fails with
 * EINVAL.  Every call on a GPU shares that GPU's array and clears its counters
 * first, so calls that overlap on one GPU (contexts on different host threads)
 * race and must be serialised by the caller.  Arguments, result and other
 * errors as sgpm_exact_count. */
sgpm_status sgpm_exact_count_noalloc(sgpm_ctx_t ctx, sgpm_graph_t g, sgpm_pattern_t p, uint64_t* count_lo,
                                     uint64_t* count_hi);

/* Colour-sparsify G (Sec. 2.2, Sec. 5.2): colour(v) = floor(c * r / 2^64) with r
 * the Philox value of (key = seed, counter = (v lo, v hi, 0, 0x40000000 | rep)),
 * keep edges whose endpoints share a colour.  The result is a new graph handle
 * on the same vertex ids (the disjoint union of the colour classes). */
sgpm_status sgpm_gs_sparsify(sgpm_ctx_t ctx, sgpm_graph_t g, uint32_t colours, uint64_t seed, uint32_t rep,
                             sgpm_graph_t* out);
/* Bernoulli edge sparsification of g (every edge kept with probability 1/inv_p,
 * inv_p in [1, 256], the keep rule of SGPM_GS_BERNOULLI for repetition rep)
 * into a new graph handle with the same vertex ids; free it with
 * sgpm_graph_free. */
sgpm_status sgpm_bes_sparsify(sgpm_ctx_t ctx, sgpm_graph_t g, uint32_t inv_p, uint64_t seed, uint32_t rep,
                              sgpm_graph_t* out);

/* ------------------------------------------------------------------ learned proposal */

/* Train the MLP proposal on pilot NS samples of (g, patterns[0..np)) drawn with
 * tag 0x80000000 | i, using the library's BF16 MFMA forward and backward
 * kernels; train_cfg may be NULL for the defaults: 2^18 pilot samples per
 * pattern, 8 epochs of Adam over minibatches of 2048 rows, learning rate 6e-3,
 * seed 1 (fields left 0 take their default). */
typedef struct {
    uint64_t pilot_samples;  /* per pattern */
    int32_t epochs;
    int32_t batch;
    float lr;
    uint64_t seed;
} sgpm_train_cfg;
sgpm_status sgpm_model_train(sgpm_ctx_t ctx, sgpm_graph_t g, const sgpm_pattern_t* patterns, int np,
                             const sgpm_train_cfg* cfg, sgpm_model_t* out);
sgpm_status sgpm_model_free(sgpm_model_t m);
/* A proposal from given weight tables (np patterns, np x [8][32][32][32]
 * uint16 weights >= 1, indexed [step][bucket of v_0][bucket of v_{j-1}]
 * [candidate bucket], bucket = floor(log2(1 + degree)) clipped to 31).  Steps
 * 2..k-2 choose a bucket in proportion to (members x weight) and a uniform
 * member of it; the last step k-1 picks uniformly (every candidate there
 * completes exactly one match), so its rows are not used. */
sgpm_status sgpm_model_from_tables(sgpm_ctx_t ctx, int np, const sgpm_pattern_t* patterns, const uint16_t* tables,
                                   sgpm_model_t* out);
/* Copy table i (8*32*32*32 uint16) out of a model. */
sgpm_status sgpm_model_table(sgpm_model_t m, int i, uint16_t* out);
/* Trained parameters (nullable; *nparams = 0 for table-only models) and
 * stats4 = {pilot seconds, total training seconds, first loss, last loss}. */
sgpm_status sgpm_model_info(sgpm_model_t m, float* params_out, int* nparams, double* stats4, uint64_t* tuples);
/* The MLP on the GPU (MFMA BF16, FP32 accumulate): forward scores of N rows of
 * 16 features, and the gradient of mean (s - y)^2 / 2 over them.  params is
 * W1[16x64], b1[64], W2[64x64], b2[64], w3[64], b3 (5313 floats). */
sgpm_status sgpm_mlp_forward(sgpm_ctx_t ctx, const float* params, const float* X, int64_t N, float* s_out);
sgpm_status sgpm_mlp_grad(sgpm_ctx_t ctx, const float* params, const float* X, const float* y, int64_t N,
                          float* grads_out);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the same loss
 * over nsteps consecutive minibatches of B rows: step s takes rows [s B, (s+1) B)
 * of X (nsteps * B x 16, row-major) and y.  params, m, v (5313 floats each) and
 * beta_pow = {0.9^t, 0.999^t} before the first step ({1, 1} at the start of
 * training) are host arrays, updated in place.  Each step equals
 * sgpm_mlp_grad on its rows followed by the FP32 update
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g g, c = 1 - beta^t,
 * params -= lr (m / c1) / (sqrt(v / c2) + eps); for B <= 256 all steps run in
 * one launch (weights in LDS), else two launches per step.  This is the
 * training step sgpm_model_train runs per epoch. */
sgpm_status sgpm_mlp_adam_steps(sgpm_ctx_t ctx, float* params, float* m, float* v, const float* X, const float* y,
                                int64_t nsteps, int64_t B, float lr, float* beta_pow);

/* ------------------------------------------------------------------ measurement probes */
/* Streaming copy of `bytes` (rounded down to 16) repeated iters times; *gbs =
 * bytes read + written per second.  The measured HBM roofline. */
sgpm_status sgpm_probe_copy(sgpm_ctx_t ctx, uint64_t bytes, int iters, double* gbs);
/* Random reads of segment_bytes-long aligned segments (4..256, a power of two)
 * from a working set of the given size, `rounds` dependent reads per segment
 * group; *gbs = segment bytes read per second.  The measured gather roofline. */
sgpm_status sgpm_probe_gather(sgpm_ctx_t ctx, uint64_t working_set_bytes, int segment_bytes, int rounds, double* gbs);

/* The MLP kernels on N random device-resident rows, iters launches each:
 * out4 = {forward ms, forward TFLOP/s, gradient ms, gradient TFLOP/s} (2 FLOPs
 * per multiply-add of the three layers; 3x that for forward + backward). */
sgpm_status sgpm_probe_mlp(sgpm_ctx_t ctx, int64_t N, int iters, double* out4);

/* ------------------------------------------------------------------ host-only utilities */
/* These run the host parts of the library without a device, so they can be
 * checked on any machine. */

/* Canonicalise a CSR on the host (same rules as sgpm_graph_from_csr; host
 * arrays only, so SGPM_DEVICE_PTRS gives EINVAL).  Call with nbr_out = NULL to
 * get *m_out (undirected edges); then off_out[n+1], nbr_out[2m] and
 * perm_out[n] (each nullable) are filled by a second call. */
sgpm_status sgpm_host_canonicalise(int64_t n, const void* offsets, int offsets_is_64, const int32_t* nbrs,
                                   uint32_t flags, int64_t* m_out, int64_t* off_out, int32_t* nbr_out,
                                   int32_t* perm_out);
/* Compile a pattern without a context; outputs as sgpm_pattern_plan. */
sgpm_status sgpm_host_plan(int k, int l, const int32_t* edges, int induced, int32_t* order, uint8_t* connect,
                           uint8_t* disconnect, uint8_t* upper, uint8_t* lower, int32_t* aut_size,
                           int32_t* oriented);
/* Phi^-1(p) for 0.5 < p < 1 (NaN otherwise). */
double sgpm_host_normal_quantile(double p);
/* Predicted relative error from exact sums given as little-endian 32-bit digits
 * (error equation, Sec. 4.1); +inf when S1 = 0. */
double sgpm_host_predicted_error(double z, uint64_t n, const uint32_t* s1, int n1, const uint32_t* s2, int n2);
/* Two-sided Student t quantile: t with P(|T| <= t) = conf for nu >= 1 degrees
 * of freedom (NaN outside 0 < conf < 1 or for nu < 1). */
double sgpm_host_t_quantile(double conf, int nu);
/* Predicted relative error of the GS estimate (the mean of n repeated
 * sparsifications) from its exact sums: t * sqrt((n S2 - S1^2) / (n - 1)) / S1,
 * the unbiased-variance form; +inf when n < 2 or S1 = 0. */
double sgpm_host_predicted_error_t(double t, uint64_t n, const uint32_t* s1, int n1, const uint32_t* s2, int n2);
/* Colour count chosen for colours = 0 (Sec. 4.4: GS time is insensitive to c
 * inside a stabilisation window, so the fewest colours inside it give the best
 * accuracy).  A probe colouring at c = 16 (repetition 0x3FFFFFFF) of a graph
 * with m edges found leaves16 matches of a k-vertex pattern; a colouring at c
 * is predicted to take 2m / 1e11 + 3e-4 + leaves16 (16 / c)^(k-1) / 3e9
 * seconds (sparsification, then a search whose leaves scale as c^-(k-1)), and
 * the result is the smallest c of 4, 5, 6, 8, 10, 12, 16 predicted within 25 %
 * of the time at 16.  SGPM_EINVAL for m < 0, k outside [2, 8] or leaves16 < 0. */
int sgpm_host_colours_choice(int64_t m, int k, double leaves16);
/* Inputs and outputs of the loose-mode cost models (SGPM_HYBRID_COST_MODEL). */
typedef struct {
    double n, m;                 /* |V| and |E| (undirected) of G */
    double triangles;            /* T, the triangle count of G (GS set-size model) */
    double count;                /* estimated count of P on G (the profiler's, scaled) */
    double eps, confidence, z;   /* target error bound, confidence, Phi^-1(1 - delta/2) */
    int32_t gs_reps_max;         /* cap on colourings */
    int32_t reserved;
    double pilot_samples, pilot_seconds; /* NS pilot on G: samples and kernel seconds */
    double rho_g;                /* hit rate of that pilot: rho(P, G) */
    double prof_samples, prof_eps_hat, prof_z; /* profiler: NS-online on G' ended at N_o with eps_o, z_o */
    double rho_sparse;           /* its hit rate: rho(P, G') */
    double sparsify_seconds, sparsify_keep; /* one timed sparsification of G keeping a fraction of the edges */
    double probe_colours, probe_search_seconds; /* one timed exact search of G colour-sparsified with c colours */
} sgpm_cost_in;
typedef struct {
    double w_lo, w_hi;           /* NS work per sample (row entries): first break point, full walk */
    double ns_samples;           /* N_s = N_o (eps_o / eps)^2 (z / z_o)^2 rho(P, G') / rho(P, G) */
    double ns_lo, ns_hi;         /* NS cone: (seconds per unit of pilot work) x w_lo / w_hi x N_s */
    double gs_seconds[7];        /* predicted GS time for 4, 5, 6, 8, 10, 12, 16 colours */
    int32_t gs_reps[7];          /* colourings the GS stop rule needs (0: more than gs_reps_max) */
    int32_t gs_colours;          /* the fastest colour count, 0 if none is feasible */
    double gs_best;              /* its predicted time */
    int32_t choice;              /* SGPM_SCHEME_GS when gs_best lies below ns_lo, else SGPM_SCHEME_NS */
    int32_t reserved;
} sgpm_cost_out;
/* The loose-mode cost models on the host (Sec. 4.3, 4.4, 5.1, 5.3) for a
 * pattern given as for sgpm_pattern_create.  NS: a row holds 2|E|/|V| entries;
 * w_lo = 1 + rows_2 d, w_hi = 1 + sum_j rows_j d (rows_j: earlier positions a
 * step merges).  GS at keep probability p = 1/c: preprocessing seconds per
 * |E| (1 + p) from the timed sparsification; search work sum_j (prod_{t<j}
 * i_t) rows_j 2|E|p/|V| with i_1 = p|E| first edges (2p|E| arcs for
 * unoriented plans) and i_j = |V| p1 p2^(c_j - 1), halved for a bounded step,
 * p1 = 2|E|p/|V|^2, p2 = min(1, 3T|V|/(2|E|^2)), c_j the step's pattern edges;
 * seconds per unit from the timed search; colourings from the relative
 * variance (c^(k-1) - 1) / count and the GS Student t stop rule.  Returns
 * SGPM_OK, or the pattern's compile error. */
int sgpm_host_cost_model(int k, int l, const int32_t* edges, int induced, const sgpm_cost_in* in, sgpm_cost_out* out);
/* End of the window that starts at sample n_t under options o. */
uint64_t sgpm_host_next_window(uint64_t n_t, const sgpm_options* o);
/* The NS time cone of loose mode's pilot selector (Sec. 5.1 and the NS cost
 * model of Sec. 4.3, measured): pilot slice i drew slice_n[i] samples in one
 * launch of slice_seconds[i] and gave the predicted error slice_eps_hat[i].
 * Launch time is fitted as t0 + n / rate by least squares over the slices (a
 * fit with t0 < 0 or no positive rate falls back to t0 = 0 and the slices'
 * mean rate).  By the error equation the samples needed scale with (eps_hat /
 * eps)^2, so slice i predicts N_i = slice_n[i] (slice_eps_hat[i] / o->eps)^2
 * samples taking N_i / rate + t0 x (windows of o's schedule up to N_i)
 * seconds (+inf for a slice without hits); *lo, *hi = their min and max, *t0
 * and *rate (nullable) the fit.  SGPM_EINVAL for bad arguments. */
int sgpm_host_ns_cone(int slices, const double* slice_n, const double* slice_seconds, const double* slice_eps_hat,
                      const sgpm_options* o, double* lo, double* hi, double* t0, double* rate);
/* Hybrid selection (loose mode, Sec. 5.1) given the NS cone's lower end
 * ns_lo.  GS: gs_reps_run (1 or 2) pilot colourings took gs_rep_seconds each
 * on average; with two, gs_cv is the relative standard deviation of one
 * colouring's estimate (unbiased variance over the squared mean) and GS needs
 * the smallest R in [3, gs_reps_max] with t_{R-1} gs_cv / sqrt(R) <= eps (t:
 * two-sided Student t quantile at `confidence`), +inf if there is none; with
 * one, only the lower bound 3 * gs_rep_seconds (the rule's minimum) is known.  *gs_pred = R *
 * gs_rep_seconds.  Returns SGPM_SCHEME_GS when GS lies entirely below the
 * cone, else SGPM_SCHEME_NS (above or overlapping: NS keeps the guarantee);
 * SGPM_EINVAL for bad inputs. */
int sgpm_host_hybrid_choice(double ns_lo, double eps, double confidence, int gs_reps_run, double gs_rep_seconds,
                            double gs_cv, int gs_reps_max, double* gs_pred);

#ifdef __cplusplus
}
#endif
#endif
