// Internal types shared by the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sgpm.h"

namespace sgpm {

// Compiled pattern (NS-prune plan, Sec. 4.2); passed to kernels by value.
struct Plan {
    int32_t k, oriented, induced, aut;
    int32_t order[8];
    uint8_t connect[8], disconnect[8], upper[8], lower[8];
    uint8_t reuse[8];  // step j's constraints contain step j-1's: S_j is a subset of S_{j-1}
};

// Device-resident canonical graph.
struct DGraph {
    const int64_t* off;   // [n+1]
    const int32_t* nbr;   // [2m] rows ascending
    const int2* epair;    // [m] oriented edges (u, w), w < u, in (u, w) order
    const int32_t* arow;  // [2m] row of each arc
    int64_t n, m;
};

// Per-block partial record written by the sampling kernels.
enum {
    PF_S1 = 0,    // 6 normalised 32-bit digits of sum X
    PF_S2 = 6,    // 10 normalised 32-bit digits of sum X^2
    PF_HITS = 16,
    PF_CSUM = 17,
    PF_BYTES = 18,
    PF_OVF = 19,
    PF_N = 20
};

struct TraceArgs {
    sgpm_trace_rec* buf;  // device buffer
    uint64_t lo, hi;
    uint32_t* sizes;      // optional: |S_j| for j < 8 per traced sample (training pilots)
};

// Learned proposal: bucket b(v) = floor(log2(1 + deg v)) clipped to 31 is
// non-increasing in the canonical id, so b(v) = #{b < 31 : v < thr[b]} with
// thr[b] = the number of vertices whose bucket exceeds b.
struct LearnArgs {
    const uint16_t* table;  // [8][32][32][32] weights for the pattern, nullptr = uniform proposal
    const uint8_t* vb;      // [n] bucket floor(log2(1 + degree)) of every vertex, clipped to 31
    const int32_t* thr;     // [32] first id of the buckets <= b (buckets do not increase with the id)
    int32_t lane_thr;       // in the kernel: thr[lane] for lanes < 32
};

// Dynamic work distribution of the sampling kernels: NTK ticket counters,
// TK_STRIDE words apart, counter x handing out tickets x, x + NTK, ...
constexpr int NTK = 8;
constexpr int TK_STRIDE = 32;
// The launch's finish counts (after the ticket counters of a slot): blocks
// finish in groups of FIN_GROUP, one count per group and one over the groups,
// each in a 128-byte line of its own.
constexpr int FIN_GROUP = 64;
constexpr int FIN_MAX_GROUPS = 32;  // so a launch has at most 2048 blocks
constexpr int FIN_STRIDE = 16;
constexpr size_t SLOT_TK_WORDS = (size_t)NTK * TK_STRIDE + (size_t)(1 + FIN_MAX_GROUPS) * FIN_STRIDE;

struct LaunchCfg {
    int lanes;     // lanes cooperating on one sample: 1, 4, 16, 64
    int spl;       // samples per group per ticket
    int blocks;    // grid size
    int base = 0;  // 1: the NS-base sampler (one sample per wave only)
};

// kernels (ns_kernels.hip)
// One sampling launch over [s0, s1) of at most FIN_GROUP * FIN_MAX_GROUPS
// blocks: ticket = SLOT_TK_WORDS words (NTK counters TK_STRIDE words apart,
// then the finish counts), zero before the launch and left zero by it;
// partials = one 20-word partial per block and per finish group; out = the
// launch's 20-word sums (PF_* layout), written by its last block.
hipError_t launch_ns_window(const DGraph& g, const Plan& p, uint64_t seed, uint32_t tag, uint64_t s0, uint64_t s1,
                            const LaunchCfg& cfg, unsigned long long* ticket, unsigned long long* partials,
                            unsigned long long* out, int checksum, int count_bytes, const TraceArgs& tr,
                            const LearnArgs& la, hipStream_t st);
int ns_blocks_per_cu(int lanes);
int ns_clique_blocks_per_cu();  // the uniform clique kernels (compiled for more blocks)
bool plan_is_clique(const Plan& p);
bool wave_uses_clique_kernel(const Plan& p, const TraceArgs& tr, const LearnArgs& la, int count_bytes);
hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t st);

// persistent batch (batch_kernels.hip)
struct BatchQuery {
    DGraph g;
    Plan p;
    uint64_t seed;
    uint32_t tag;
    int32_t lanes;  // lanes per sample: 1, 4, 16 or 64
    int32_t mode;   // SGPM_MODE_STRICT_NS or SGPM_MODE_FIXED_N
    int32_t tile;   // samples per ticket
    int32_t window_cap;  // first window index that would hold >= 2^32 samples
    int32_t pad;
    uint64_t fixed_n, n_min, w_min, quantum, max_samples;
    double growth, eps, z;
};
// one ticket counter per XCD, each in a cache line of its own: counter c hands
// out tiles c, c + 8, c + 16, .. of the current window as epoch << 40 | k
struct alignas(128) BatchTicket {
    unsigned long long v;
    unsigned long long pad[15];
};
struct BatchState {
    BatchTicket ticket[8];
    alignas(128) unsigned long long done;  // samples whose sums are in win[]
    unsigned long long done_pad[15];
    int32_t finished, status, converged, windows;
    unsigned long long win[8][PF_N];         // current window's sum columns, one copy per XCD
    unsigned long long tot_s1[8], tot_s2[12];  // normalised 32-bit digits
    unsigned long long hits, csum, bytes, ovf;
    double eps_hat;
    uint64_t n;
};
int batch_blocks_per_cu(int kmax, bool clq, bool grp);
int batch_kmax(int k);
hipError_t launch_batch(const BatchQuery* q, BatchState* s, int nq, unsigned long long* active, int blocks,
                        int kmax, bool clq, bool grp, hipStream_t st);

struct NsExtra {
    LearnArgs la;        // learned proposal (table nullptr = uniform)
    uint32_t* d_sizes;   // pilot traces: |S_j| per traced sample
    // samples [0, prefix_n) of the estimation stream already drawn (the
    // loose-mode pilot): their window sums, kernel seconds and launches; used
    // by a strict run when prefix_n lies inside its first window or ends it
    uint64_t prefix_n;
    unsigned long long prefix_sums[PF_N];
    double prefix_kernel_s;
    int prefix_launches;
};

// MLP (mlp_kernels.hip)
int mlp_nparams();
int64_t mlp_grad_blocks(int64_t N);  // partial gradients mlp_grad / mlp_adam_steps write
hipError_t mlp_forward(const float* P, const float* X, int64_t N, float* s_out, hipStream_t st);
hipError_t mlp_grad(const float* P, const float* X, const float* y, int64_t N, float* gpart, float* g,
                    hipStream_t st);
hipError_t mlp_adam_steps(float* P, float* m, float* v, const float* X, const float* y, int64_t nsteps, int64_t B,
                          float lr, float* bpow, float* gpart, hipStream_t st);

// host helpers
struct HostGraph {
    int64_t n = 0, m = 0;
    std::vector<int64_t> off;
    std::vector<int32_t> nbr;
    std::vector<int32_t> perm;  // perm[original] = canonical
};
int canonicalise(int64_t n, const void* offsets, int off64, const int32_t* nbrs, bool assume_canonical,
                 HostGraph& out, std::string& err);
int compile_pattern(int k, int l, const int32_t* edges, int induced, Plan& out, std::string& err);

// exact big integers as little-endian 32-bit digits
struct Big {
    std::vector<uint32_t> d;
    explicit Big(size_t nd = 24) : d(nd, 0) {}
};
void big_add_digits(Big& a, const unsigned long long* digits, int nd);  // digits may exceed 32 bits
double big_to_double(const Big& a);
bool big_is_zero(const Big& a);
double normal_quantile(double p);
double predicted_error(double z, uint64_t n, const Big& S1, const Big& S2);
double student_t_quantile(double conf, int nu);
double predicted_error_t(double t, uint64_t n, const Big& S1, const Big& S2);
uint64_t next_window_end(uint64_t n_t, const sgpm_options& o);

// GS kernels (gs_kernels.hip)
hipError_t gs_colours(int64_t n, uint32_t c, uint64_t seed, uint32_t rep, uint8_t* col, hipStream_t st);
int64_t arc_tiles(int64_t narcs);
// col != nullptr: colour sparsification by col; else Bernoulli edge
// sparsification with probability 1/c for repetition rep
hipError_t gs_arc_counts(const DGraph& g, const uint8_t* col, uint32_t c, uint64_t seed, uint32_t rep, int64_t* tk,
                         int64_t* tl, hipStream_t st);
hipError_t gs_arc_write(const DGraph& g, const uint8_t* col, uint32_t c, uint64_t seed, uint32_t rep,
                        const int64_t* tko, const int64_t* tlo, int32_t* nnbr, int32_t* narow, int2* nepair,
                        int64_t* rstart, int64_t* rlow, int64_t* noff, int64_t* neoff, hipStream_t st);
int64_t scan_scratch_words(int64_t n);
hipError_t exclusive_scan(const int64_t* in, int64_t n, int64_t* out, int64_t* scratch, hipStream_t st);
// exclusive scans of a and b (n entries each, totals at oa[n], ob[n]); one
// block for n up to 65,536, else exclusive_scan twice
hipError_t exclusive_scan_pair(const int64_t* a, const int64_t* b, int64_t n, int64_t* oa, int64_t* ob,
                               int64_t* scratch, hipStream_t st);
hipError_t max_degree(const int64_t* off, int64_t n, unsigned long long* out, hipStream_t st);
// Work split of the count kernels: a wave (or lane group) takes ticket t from
// one counter and counts first edges [ticket_start(t), ticket_start(t + 1)).
// Ticket t holds base + floor(t / growth) edges roughly (growth 0: base
// each), so with growth the first tickets, over the highest-degree rows that
// lead the edge order, are short while the count of tickets (one atomic each
// on the shared counter) stays bounded.  growth > 0 needs nfirst < 2^32.
struct TicketPlan {
    uint64_t base, growth;
};
__host__ __device__ inline uint64_t ticket_start(const TicketPlan& tp, uint64_t t) {
    return t * tp.base + (tp.growth ? (t * (t - 1) / 2) / tp.growth : 0);
}
// group: lanes per first edge (8, 16 or 64); elist: nullptr for first edges
// [0, nfirst), else nfirst entries of first-edge ids
hipError_t launch_exact_count(const DGraph& g, const Plan& p, uint64_t nfirst, int group, int blocks, TicketPlan tp,
                              unsigned long long* ticket, unsigned long long* partials, unsigned long long* out2,
                              const uint32_t* elist, hipStream_t st);
int exact_blocks_per_cu(int group);
// the k-clique (k = 4, 5, 6; oriented first edges) by bitmaps over each first
// edge's candidate set of at most 64; first edges with larger sets are appended
// to overflow (count in *noverflow, both zero before the launch)
hipError_t launch_clique_bitmap(const DGraph& g, int k, uint64_t nfirst, int blocks, TicketPlan tp,
                                unsigned long long* ticket, unsigned long long* partials, unsigned long long* out2,
                                uint32_t* overflow, unsigned long long* noverflow, hipStream_t st);
int clique_bitmap_blocks_per_cu(int k);
// the same for the nlist first edges elist[] whose candidate sets hold up to
// 128 members (two-word masks); larger sets go to overflow
hipError_t launch_clique_bitmap128(const DGraph& g, int k, const uint32_t* elist, uint64_t nlist, int blocks,
                                   TicketPlan tp, unsigned long long* ticket, unsigned long long* partials,
                                   unsigned long long* out2, uint32_t* overflow, unsigned long long* noverflow,
                                   hipStream_t st);
int clique_bitmap128_blocks_per_cu(int k);
// Closed-form 4-vertex counts over edges: for every oriented edge (common
// neighbours t, endpoint degrees du, dw) the terms sel[0..2] of
//   0 C(t, 2), 1 t (du + dw - 4), 2 (du - 1)(dw - 1) - t,
//   3 C(du - 1, 2) + C(dw - 1, 2), 4 du + dw - 2, 5 du + dw - 2 - 2t
// (-1: none) are summed; out6[2k], out6[2k + 1] receive term k's low and high
// 32-bit halves' sums.  need_t: the terms use t (group 8 or 64 lanes per
// edge intersect the rows); else one lane per edge.  partials: 6 words per
// block.
hipError_t launch_edge_terms(const DGraph& g, int group, bool need_t, int blocks, TicketPlan tp, const int sel[3],
                             unsigned long long* ticket, unsigned long long* partials, unsigned long long* out6,
                             hipStream_t st);
int edge_terms_blocks_per_cu(int group, bool need_t);
// Scratch of the allocation-free exact count: one file-scope device array per
// GPU of kCountScratchWords 64-bit words, laid out as kCountScratchBlocks
// two-word block partials, then kCountCells counter and sum words, then a list of
// kCountScratchOvf 32-bit first-edge ids (8 MiB) for the bitmap count's first
// edges with more than 64 candidates.
constexpr size_t kCountScratchBlocks = 4096;
constexpr size_t kCountScratchOvf = size_t(1) << 21;
constexpr size_t kCountCells = 48;
constexpr size_t kCountScratchWords = 2 * kCountScratchBlocks + kCountCells + kCountScratchOvf / 2;
// that array's device address on `dev`, which must be the current device:
// looked up once per device (hipGetSymbolAddress), then reused
hipError_t count_scratch_address(int dev, unsigned long long** out);
// probes (probe_kernels.hip)
hipError_t probe_copy(const void* in, void* out, uint64_t bytes, int blocks, hipStream_t st);
hipError_t probe_gather(const int32_t* a, uint64_t words, int seg_bytes, int rounds, int blocks, uint64_t seed,
                        unsigned long long* sink, hipStream_t st);

}  // namespace sgpm

// ------------------------------------------------------------------ library handles
struct sgpm_ctx {
    int dev = 0;
    hipStream_t st = nullptr;
    std::string err;
    int cus = 256;
    // scratch reused across calls
    unsigned long long* d_partials = nullptr;
    unsigned long long* d_partials2 = nullptr;  // the second stream's
    size_t partial_blocks = 0;
    hipStream_t st2 = nullptr;  // a window queued ahead runs here, beside the one on st
    unsigned long long* h_slots = nullptr;   // pinned host slots: per launch its 20 sums (32 words a slot)
    unsigned long long* dh_slots = nullptr;  // the same memory as seen from the device
    unsigned long long* d_tickets = nullptr; // per slot: SLOT_TK_WORDS words of ticket counters and finish counts
    size_t nslots = 0;
    std::vector<hipEvent_t> kev;             // start/stop events around each sampling kernel
    // batch: autotuned lanes per (graph, plan), device/pinned tables, captured graph
    // batch (lanes per sample, tile) per (graph, plan, requested lanes)
    std::map<std::tuple<const void*, std::string, int>, std::pair<int, int>> tuned;
    std::map<std::tuple<const void*, std::string>, int> ns_tuned;  // solo lanes per sample per (graph, plan)
    int batch_nq = 0;
    int batch_kmax = 0;
    bool batch_clq = false;
    bool batch_grp = false;
    void* d_bq = nullptr;
    void* h_bq = nullptr;
    hipStream_t batch_stream = nullptr;
    hipGraph_t batch_graph = nullptr;
    hipGraphExec_t batch_exec = nullptr;
    // grow-only device scratch of the GS engine (sparsification temporaries,
    // count partials), reused by every colouring; freed with the context.  GS
    // calls finish (stream synchronised) before they return, so calls on one
    // context never share it in flight.
    std::vector<std::pair<void*, size_t>> gs_scratch;
};

struct sgpm_graph {
    sgpm_ctx* ctx = nullptr;
    int64_t n = 0, m = 0, maxdeg = 0;
    bool degree_ordered = false;  // canonical ids: degree non-increasing (bucket thresholds valid)
    int32_t bthr[32] = {0};          // host: vertices with bucket > b (bucket thresholds in id order)
    uint8_t* d_vb = nullptr;         // device: bucket of every vertex (canonical graphs)
    int32_t* d_bthr = nullptr;       // device: bthr
    std::vector<int32_t> perm;
    int64_t* d_off = nullptr;
    int32_t* d_nbr = nullptr;
    int2* d_epair = nullptr;
    int32_t* d_arow = nullptr;
    bool borrowed = false;  // the device arrays are the context's GS scratch: not freed here
    sgpm::DGraph view() const { return sgpm::DGraph{d_off, d_nbr, d_epair, d_arow, n, m}; }
    sgpm_graph() = default;
    sgpm_graph(const sgpm_graph&) = delete;
    sgpm_graph& operator=(const sgpm_graph&) = delete;
    // owns its device arrays, so a build that fails part way frees what it took
    ~sgpm_graph();
};

struct sgpm_pattern {
    sgpm::Plan plan;
};

struct sgpm_model {
    sgpm_ctx* ctx = nullptr;
    int np = 0;
    std::vector<sgpm::Plan> plans;
    std::vector<uint16_t> tables;  // np x [8][32][32][32]
    uint16_t* d_tables = nullptr;
    std::vector<float> params;     // trained MLP (empty for table-only models)
    double train_seconds = 0.0, pilot_seconds = 0.0, loss_first = 0.0, loss_last = 0.0;
    uint64_t tuples = 0;
    sgpm_model() = default;
    sgpm_model(const sgpm_model&) = delete;
    sgpm_model& operator=(const sgpm_model&) = delete;
    ~sgpm_model();  // frees d_tables
};


namespace sgpm {

// engines shared by the estimate entry points
struct GsPrefix {              // colourings 0..n-1 already counted (hybrid pilots)
    int n = 0;
    unsigned __int128 y[2] = {0, 0};
    double dev_seconds = 0.0;
};
sgpm_status gs_rep(sgpm_ctx* c, sgpm_graph* g, const Plan& p, uint32_t colours, uint64_t seed, uint32_t rep,
                   unsigned __int128* y, double* dev_seconds, bool bes = false);
// modelled seconds of one colour sparsification of a graph of m edges (two
// passes over the 2m arcs at the measured 1e11 arcs/s, plus 0.3 ms of launches)
double gs_sparsify_model_s(int64_t m);
uint32_t colours_from_probe(int64_t m, int k, double leaves16);
sgpm_status gs_resolve_colours(sgpm_ctx* c, sgpm_graph* g, const Plan& p, const sgpm_options& o, uint32_t* col);
sgpm_status gs_estimate(sgpm_ctx* c, sgpm_graph* g, const Plan& p, const sgpm_options& o, sgpm_result* res,
                        const GsPrefix* pre = nullptr);
sgpm_status ns_estimate_solo(sgpm_ctx* c, sgpm_graph* g, const Plan& p, const sgpm_options& o, sgpm_result* res,
                             int count_bytes, const NsExtra* ex = nullptr);
// NS pilot: `slices` equal consecutive id ranges of [0, n) under options o
// (the caller sets the tag); per slice the kernel seconds and predicted error,
// and the estimate of the count over the whole pilot
sgpm_status ns_pilot(sgpm_ctx* c, sgpm_graph* g, const Plan& p, const sgpm_options& o, const LearnArgs& la,
                     int slices, const uint64_t* slice_end, double* seconds, double* eps_hat, double* mean,
                     unsigned long long* sums_out);
// NS time cone from pilot slices (one launch each): launch time fitted as
// t0 + n / rate over the slices; slice i predicts n_i (eps_hat_i / eps)^2
// samples in N / rate + t0 x (windows of the schedule of o up to N) seconds
void ns_cone(int slices, const double* slice_n, const double* seconds, const double* eps_hat, const sgpm_options& o,
             double* lo, double* hi, double* t0_out, double* rate_out);
sgpm_status learn_args_for(sgpm_ctx* c, sgpm_graph* g, sgpm_pattern* p, sgpm_model* m, LearnArgs* la);
sgpm_status hybrid_estimate(sgpm_ctx* c, sgpm_graph* g, sgpm_pattern* p, const sgpm_options& o, sgpm_result* res);
sgpm_status model_hybrid_estimate(sgpm_ctx* c, sgpm_graph* g, sgpm_pattern* p, const sgpm_options& o,
                                  sgpm_result* res);
void cost_model(const Plan& p, const sgpm_cost_in& in, sgpm_cost_out* out);
// scratch_graph: the sparsified graph's arrays are the context's GS scratch
// (grown, never freed per call) and its max degree is not measured but taken
// as the source's over c; the handle must be freed before
// the next such call on the context
sgpm_status sparsify(sgpm_ctx* c, sgpm_graph* g, uint32_t colours, uint64_t seed, uint32_t rep, sgpm_graph** out,
                     bool bes = false, bool scratch_graph = false);
sgpm_status exact_count(sgpm_ctx* c, sgpm_graph* g, const Plan& p, unsigned __int128* out, double* seconds);
// patterns whose exact count is a closed form over per-edge terms (common
// neighbours and degrees of the edge's endpoints), by edge_shape; the
// vertex-induced 4-path and 4-cycle also take the 4-cycles' general search
enum EdgeShape { SHAPE_NONE, SHAPE_WEDGE, SHAPE_STAR3, SHAPE_PATH4, SHAPE_TAILED, SHAPE_DIAMOND, SHAPE_IPATH4, SHAPE_ICYCLE4 };
int edge_shape(const Plan& p);
// the edge-shaped patterns and the 4- to 6-clique: counted from per-edge terms
// or by bitmaps, whose time does not follow the number of leaves
bool count_not_by_leaves(const Plan& p);
int hybrid_choice(double ns_lo, double eps, double confidence, int gs_reps_run, double gs_rep_seconds, double gs_cv,
                  int gs_reps_max, double* gs_pred);
int gs_reps_needed(double cv, double eps, double confidence, int cap);
// the GS stop rule tests its interval from the third sparsification on
constexpr uint64_t kGsMinReps = 3;

inline sgpm_status fail(sgpm_ctx* c, sgpm_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                                 \
    do {                                                                                                   \
        hipError_t _e = (expr);                                                                            \
        if (_e != hipSuccess) return sgpm::fail((ctx), SGPM_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

// Device memory owned by a scope: freed on every return path (hipFree waits for
// the work still using it).
struct DeviceBuffer {
    void* p = nullptr;
    DeviceBuffer() = default;
    DeviceBuffer(const DeviceBuffer&) = delete;
    DeviceBuffer& operator=(const DeviceBuffer&) = delete;
    ~DeviceBuffer() {
        if (p) (void)hipFree(p);
    }
};

// N HIP events owned by a scope: create() makes them, the destructor releases
// those made, on every return path.
template <int N>
struct ScopedEvents {
    hipEvent_t e[N] = {};
    int made = 0;
    ScopedEvents() = default;
    ScopedEvents(const ScopedEvents&) = delete;
    ScopedEvents& operator=(const ScopedEvents&) = delete;
    hipError_t create() {
        for (; made < N; made++) {
            const hipError_t r = hipEventCreate(&e[made]);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
    ~ScopedEvents() {
        for (int i = 0; i < made; i++) (void)hipEventDestroy(e[i]);
    }
    hipEvent_t operator[](int i) const { return e[i]; }
};

}  // namespace sgpm
