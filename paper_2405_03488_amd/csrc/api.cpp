// C-ABI entry points: contexts, graphs, patterns and the NS estimation loop.
#include <algorithm>
#include <deque>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>

#include "sgpm_internal.h"

using namespace sgpm;

namespace sgpm {
}

namespace {

constexpr int SLOT_WORDS = 32;  // host slot of one launch: [1..20] its sums


sgpm_status ensure_scratch(sgpm_ctx* c, size_t blocks, size_t slots) {
    if (blocks > c->partial_blocks) {
        if (c->d_partials) (void)hipFree(c->d_partials);
        if (c->d_partials2) (void)hipFree(c->d_partials2);
        c->d_partials = c->d_partials2 = nullptr;
        c->partial_blocks = 0;
        // a partial per block and per finish group of the block
        HIP_TRY(c, hipMalloc(&c->d_partials, (blocks + FIN_MAX_GROUPS) * PF_N * sizeof(unsigned long long)));
        HIP_TRY(c, hipMalloc(&c->d_partials2, (blocks + FIN_MAX_GROUPS) * PF_N * sizeof(unsigned long long)));
        c->partial_blocks = blocks;
    }
    if (!c->st2) HIP_TRY(c, hipStreamCreateWithFlags(&c->st2, hipStreamNonBlocking));
    if (slots > c->nslots) {
        if (c->h_slots) (void)hipHostFree(c->h_slots);
        if (c->d_tickets) (void)hipFree(c->d_tickets);
        c->h_slots = nullptr;
        c->dh_slots = nullptr;
        c->d_tickets = nullptr;
        c->nslots = 0;
        size_t want = std::max<size_t>(slots, 1024);
        // pinned host slots the reduction kernel writes into directly: no copy
        // command follows a window, so queueing the next window never waits
        HIP_TRY(c, hipHostMalloc(&c->h_slots, want * SLOT_WORDS * sizeof(unsigned long long),
                                 hipHostMallocMapped | hipHostMallocCoherent));
        HIP_TRY(c, hipHostGetDevicePointer((void**)&c->dh_slots, c->h_slots, 0));
        // per slot: the ticket counters and the launch's finish counts, zero
        // between launches (each launch's last block clears them)
        HIP_TRY(c, hipMalloc(&c->d_tickets, want * SLOT_TK_WORDS * sizeof(unsigned long long)));
        HIP_TRY(c, hipMemsetAsync(c->d_tickets, 0, want * SLOT_TK_WORDS * sizeof(unsigned long long), c->st));
        HIP_TRY(c, hipStreamSynchronize(c->st));
        c->nslots = want;
    }
    return SGPM_OK;
}

int blocks_for(sgpm_ctx* c, int lanes, bool clique_kernel = false) {
    // enough 256-thread blocks to fill every CU at the kernel's occupancy
    return c->cus * (clique_kernel ? ns_clique_blocks_per_cu() : ns_blocks_per_cu(lanes));
}

int largest_grid(sgpm_ctx* c) {
    int m = blocks_for(c, 64, true);
    for (int l : {1, 4, 16, 64}) m = std::max(m, blocks_for(c, l));
    return m;
}

}  // namespace

sgpm_graph::~sgpm_graph() {
    // lane counts and tiles tuned for this graph must not carry over to a
    // later graph that happens to get the same address
    if (ctx) {
        for (auto it = ctx->ns_tuned.begin(); it != ctx->ns_tuned.end();)
            it = std::get<0>(it->first) == (const void*)this ? ctx->ns_tuned.erase(it) : std::next(it);
        for (auto it = ctx->tuned.begin(); it != ctx->tuned.end();)
            it = std::get<0>(it->first) == (const void*)this ? ctx->tuned.erase(it) : std::next(it);
    }
    if (borrowed || (!d_off && !d_nbr && !d_epair && !d_arow && !d_vb && !d_bthr)) return;
    if (ctx) (void)hipSetDevice(ctx->dev);
    for (void* q : {(void*)d_off, (void*)d_nbr, (void*)d_epair, (void*)d_arow, (void*)d_vb, (void*)d_bthr})
        if (q) (void)hipFree(q);
}

extern "C" {

int sgpm_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    return n;
}

sgpm_status sgpm_create(sgpm_ctx_t* out, int hip_device, void* hip_stream) {
    if (!out) return SGPM_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return SGPM_EHIP;
    auto* c = new (std::nothrow) sgpm_ctx();
    if (!c) return SGPM_ENOMEM;
    c->dev = hip_device;
    c->st = (hipStream_t)hip_stream;
    if (hipSetDevice(hip_device) != hipSuccess) {
        delete c;
        return SGPM_EHIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess && prop.multiProcessorCount > 0)
        c->cus = prop.multiProcessorCount;
    *out = c;
    return SGPM_OK;
}

sgpm_status sgpm_destroy(sgpm_ctx_t c) {
    if (!c) return SGPM_EINVAL;
    (void)hipSetDevice(c->dev);
    if (c->st2) (void)hipStreamSynchronize(c->st2);
    if (c->d_partials) (void)hipFree(c->d_partials);
    if (c->d_partials2) (void)hipFree(c->d_partials2);
    if (c->st2) (void)hipStreamDestroy(c->st2);
    if (c->h_slots) (void)hipHostFree(c->h_slots);
    if (c->d_tickets) (void)hipFree(c->d_tickets);
    for (hipEvent_t e : c->kev) (void)hipEventDestroy(e);
    if (c->batch_exec) (void)hipGraphExecDestroy(c->batch_exec);
    if (c->batch_graph) (void)hipGraphDestroy(c->batch_graph);
    if (c->batch_stream) (void)hipStreamDestroy(c->batch_stream);
    if (c->d_bq) (void)hipFree(c->d_bq);
    if (c->h_bq) (void)hipHostFree(c->h_bq);
    for (auto& b : c->gs_scratch)
        if (b.first) (void)hipFree(b.first);
    delete c;
    return SGPM_OK;
}

const char* sgpm_last_error(sgpm_ctx_t c) { return c ? c->err.c_str() : "null context"; }

void sgpm_options_default(sgpm_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->eps = 0.01;
    o->confidence = 0.95;
    o->seed = 1;
    o->query_tag = 0;
    o->mode = SGPM_MODE_STRICT_NS;
    o->n_min = 1ull << 19;
    o->w_min = 1ull << 19;
    o->quantum = 1ull << 16;
    o->max_samples = 1ull << 40;
    o->window_growth = 0.10;
    o->colours = 0;
    o->gs_reps_max = 64;
    o->lanes_per_sample = 0;
}

sgpm_status sgpm_graph_from_csr(sgpm_ctx_t c, int64_t n, const void* offsets, int offsets_is_64,
                                const int32_t* nbrs, uint32_t flags, sgpm_graph_t* out) {
    if (!c || !out || !offsets || n < 0 || n >= (1ll << 31)) return fail(c, SGPM_EINVAL, "bad graph arguments");
    if (flags & ~(SGPM_ASSUME_CANONICAL | SGPM_DEVICE_PTRS | SGPM_SYMMETRIZE))
        return fail(c, SGPM_EINVAL, "unknown graph flags");
    if ((flags & SGPM_ASSUME_CANONICAL) && (flags & SGPM_SYMMETRIZE))
        return fail(c, SGPM_EINVAL, "SGPM_SYMMETRIZE contradicts SGPM_ASSUME_CANONICAL");
    // device arrays: staged to the host, where the canonicalisation runs
    std::vector<unsigned char> h_off;
    std::vector<int32_t> h_nbr;
    if (flags & SGPM_DEVICE_PTRS) {
        HIP_TRY(c, hipSetDevice(c->dev));
        const size_t w = offsets_is_64 ? 8 : 4;
        h_off.resize(w * (size_t)(n + 1));
        HIP_TRY(c, hipMemcpy(h_off.data(), offsets, h_off.size(), hipMemcpyDefault));
        const int64_t cnt = offsets_is_64 ? ((const int64_t*)h_off.data())[n] : ((const int32_t*)h_off.data())[n];
        if (cnt < 0) return fail(c, SGPM_EBADGRAPH, "offsets[n] < 0");
        if (cnt > 0 && !nbrs) return fail(c, SGPM_EINVAL, "null neighbour array");
        h_nbr.resize((size_t)cnt);
        if (cnt > 0) HIP_TRY(c, hipMemcpy(h_nbr.data(), nbrs, sizeof(int32_t) * (size_t)cnt, hipMemcpyDefault));
        offsets = h_off.data();
        nbrs = h_nbr.data();
    }
    HostGraph h;
    std::string err;
    int rc = canonicalise(n, offsets, offsets_is_64, nbrs, (flags & SGPM_ASSUME_CANONICAL) != 0, h, err);
    if (rc != SGPM_OK) return fail(c, (sgpm_status)rc, err);
    auto g = std::make_unique<sgpm_graph>();
    g->ctx = c;
    g->n = h.n;
    g->m = h.m;
    for (int64_t u = 0; u < n; u++) g->maxdeg = std::max(g->maxdeg, h.off[(size_t)u + 1] - h.off[(size_t)u]);
    // oriented edges (u, w), w < u: the prefix of each ascending row below u
    std::vector<int2> ep((size_t)std::max<int64_t>(h.m, 1));
    std::vector<int32_t> arow((size_t)std::max<int64_t>(2 * h.m, 1));
    {
        int64_t e = 0;
        for (int64_t u = 0; u < n; u++)
            for (int64_t i = h.off[(size_t)u]; i < h.off[(size_t)u + 1]; i++) {
                arow[(size_t)i] = (int32_t)u;
                if (h.nbr[(size_t)i] < u) ep[(size_t)e++] = make_int2((int32_t)u, h.nbr[(size_t)i]);
            }
        if (e != h.m) return fail(c, SGPM_EBADGRAPH, "internal: oriented edge count mismatch");
    }
    HIP_TRY(c, hipSetDevice(c->dev));
    HIP_TRY(c, hipMalloc(&g->d_off, sizeof(int64_t) * (size_t)(n + 1)));
    HIP_TRY(c, hipMalloc(&g->d_nbr, sizeof(int32_t) * (size_t)std::max<int64_t>(2 * h.m, 1)));
    HIP_TRY(c, hipMalloc(&g->d_epair, sizeof(int2) * (size_t)std::max<int64_t>(h.m, 1)));
    HIP_TRY(c, hipMalloc(&g->d_arow, sizeof(int32_t) * (size_t)std::max<int64_t>(2 * h.m, 1)));
    HIP_TRY(c, hipMemcpy(g->d_off, h.off.data(), sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice));
    if (h.m > 0) {
        HIP_TRY(c, hipMemcpy(g->d_nbr, h.nbr.data(), sizeof(int32_t) * (size_t)(2 * h.m), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(g->d_epair, ep.data(), sizeof(int2) * (size_t)h.m, hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(g->d_arow, arow.data(), sizeof(int32_t) * (size_t)(2 * h.m), hipMemcpyHostToDevice));
    }
    // degree buckets b = floor(log2(1 + deg)) are non-increasing in the canonical id;
    // the learned proposal counts a sorted candidate set's buckets by searching
    // it for the first id of each bucket, and reads single candidates' buckets
    // from a byte per vertex
    g->degree_ordered = true;
    {
        int64_t cntb[32] = {0};
        std::vector<uint8_t> vb((size_t)std::max<int64_t>(n, 1), 0);
        for (int64_t u = 0; u < n; u++) {
            const int64_t d = h.off[(size_t)u + 1] - h.off[(size_t)u];
            int b = 0;
            while (b < 31 && ((d + 1) >> (b + 1)) > 0) b++;
            cntb[b]++;
            vb[(size_t)u] = (uint8_t)b;
        }
        int64_t above = 0;
        for (int b = 31; b >= 0; b--) {
            g->bthr[b] = (int32_t)above;  // vertices with bucket > b
            above += cntb[b];
        }
        HIP_TRY(c, hipMalloc(&g->d_vb, vb.size()));
        HIP_TRY(c, hipMemcpy(g->d_vb, vb.data(), vb.size(), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMalloc(&g->d_bthr, sizeof(g->bthr)));
        HIP_TRY(c, hipMemcpy(g->d_bthr, g->bthr, sizeof(g->bthr), hipMemcpyHostToDevice));
    }
    g->perm = std::move(h.perm);
    *out = g.release();
    return SGPM_OK;
}

sgpm_status sgpm_graph_stats(sgpm_graph_t g, int64_t* n, int64_t* m, int64_t* max_deg, int32_t* perm_out) {
    if (!g) return SGPM_EINVAL;
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (max_deg) *max_deg = g->maxdeg;
    if (perm_out && !g->perm.empty()) std::memcpy(perm_out, g->perm.data(), sizeof(int32_t) * g->perm.size());
    return SGPM_OK;
}

sgpm_status sgpm_graph_export(sgpm_graph_t g, int64_t* off_out, int32_t* nbr_out) {
    if (!g) return SGPM_EINVAL;
    sgpm_ctx* c = g->ctx;
    HIP_TRY(c, hipSetDevice(c->dev));
    if (off_out) HIP_TRY(c, hipMemcpy(off_out, g->d_off, sizeof(int64_t) * (size_t)(g->n + 1), hipMemcpyDeviceToHost));
    if (nbr_out && g->m > 0)
        HIP_TRY(c, hipMemcpy(nbr_out, g->d_nbr, sizeof(int32_t) * (size_t)(2 * g->m), hipMemcpyDeviceToHost));
    return SGPM_OK;
}

sgpm_status sgpm_graph_free(sgpm_graph_t g) {
    if (!g) return SGPM_EINVAL;
    delete g;
    return SGPM_OK;
}

sgpm_status sgpm_pattern_create(sgpm_ctx_t c, int k, int l, const int32_t* edges, int induced, sgpm_pattern_t* out) {
    if (!c || !out) return fail(c, SGPM_EINVAL, "null argument");
    Plan p;
    std::string err;
    int rc = compile_pattern(k, l, edges, induced, p, err);
    if (rc != SGPM_OK) return fail(c, (sgpm_status)rc, err);
    auto* h = new (std::nothrow) sgpm_pattern();
    if (!h) return SGPM_ENOMEM;
    h->plan = p;
    *out = h;
    return SGPM_OK;
}

sgpm_status sgpm_pattern_plan(sgpm_pattern_t p, int32_t* order, uint8_t* connect, uint8_t* disconnect, uint8_t* upper,
                              uint8_t* lower, int32_t* aut_size, int32_t* oriented) {
    if (!p) return SGPM_EINVAL;
    const Plan& q = p->plan;
    for (int i = 0; i < q.k; i++) {
        if (order) order[i] = q.order[i];
        if (connect) connect[i] = q.connect[i];
        if (disconnect) disconnect[i] = q.disconnect[i];
        if (upper) upper[i] = q.upper[i];
        if (lower) lower[i] = q.lower[i];
    }
    if (aut_size) *aut_size = q.aut;
    if (oriented) *oriented = q.oriented;
    return SGPM_OK;
}

sgpm_status sgpm_pattern_free(sgpm_pattern_t p) {
    if (!p) return SGPM_EINVAL;
    delete p;
    return SGPM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ NS engine
namespace {

struct NsState {
    Big S1{24}, S2{24};
    uint64_t n = 0, hits = 0, csum = 0, bytes = 0, ovf = 0;
};

void absorb(NsState& s, const unsigned long long* sums) {
    big_add_digits(s.S1, sums + PF_S1, 6);
    big_add_digits(s.S2, sums + PF_S2, 10);
    s.hits += sums[PF_HITS];
    s.csum += sums[PF_CSUM];
    s.bytes += sums[PF_BYTES];
    s.ovf += sums[PF_OVF];
}

// Launch [s0, s1) with the given lane count into slot `slot`; enqueue only.
// `span` is the length of the whole window the range belongs to: ticket sizes
// follow it, so a window split into pieces (autotuning, pilots) is launched
// as the whole window would be.
sgpm_status enqueue_range(sgpm_ctx* c, sgpm_graph* g, const Plan& p, const sgpm_options& o, uint64_t s0, uint64_t s1,
                          int lanes, size_t slot, const TraceArgs& tr, int count_bytes, const LearnArgs& la,
                          uint64_t span = 0, bool second_stream = false) {
    LaunchCfg cfg;
    cfg.lanes = lanes;
    cfg.base = o.sampler == SGPM_SAMPLER_BASE ? 1 : 0;
    cfg.blocks = blocks_for(c, lanes, lanes == 64 && !la.table && !cfg.base && wave_uses_clique_kernel(p, tr, la, count_bytes));
    // Tickets of about 1/16 of a wave's share of the window: few enough that
    // the single ticket counter (a device-scope atomic, about 8e7 per second
    // on one address) is not the bottleneck, many enough to balance skewed
    // per-sample work across waves.
    {
        const uint64_t waves = (uint64_t)cfg.blocks * 4, groups_per_wave = (uint64_t)(64 / lanes);
        const uint64_t len = std::max<uint64_t>(span, s1 - s0);
        const uint64_t per_group = len / (waves * groups_per_wave * 16);
        cfg.spl = (int)std::min<uint64_t>(256, std::max<uint64_t>(1, per_group));
        // one sample per wave: whole groups of 16 samples (the kernel's draw and
        // record groups)
        if (lanes == 64) cfg.spl = (cfg.spl + 15) / 16 * 16;
    }
    const uint64_t per_wave = (uint64_t)(64 / lanes) * (uint64_t)cfg.spl;
    const uint64_t tickets = (s1 - s0 + per_wave - 1) / per_wave;
    const uint64_t max_blocks = std::min<uint64_t>((tickets + 3) / 4, (uint64_t)FIN_GROUP * FIN_MAX_GROUPS);
    if ((uint64_t)cfg.blocks > max_blocks) cfg.blocks = (int)std::max<uint64_t>(1, max_blocks);
    // partials sized for the largest grid once, so no buffer in flight is freed
    sgpm_status st = ensure_scratch(c, (size_t)largest_grid(c), slot + 1);
    if (st != SGPM_OK) return st;
    hipStream_t sq = second_stream ? c->st2 : c->st;
    unsigned long long* parts = second_stream ? c->d_partials2 : c->d_partials;
    unsigned long long* tk = c->d_tickets + slot * SLOT_TK_WORDS;
    while (c->kev.size() < 3 * (slot + 1)) {
        hipEvent_t ev;
        HIP_TRY(c, hipEventCreate(&ev));
        c->kev.push_back(ev);
    }
    HIP_TRY(c, hipEventRecord(c->kev[3 * slot], sq));
    // the launch's last block adds the block partials into the slot's host-mapped words
    HIP_TRY(c, launch_ns_window(g->view(), p, o.seed, o.query_tag, s0, s1, cfg, tk, parts,
                                c->dh_slots + slot * SLOT_WORDS + 1, o.checksum, count_bytes, tr, la, sq));
    HIP_TRY(c, hipEventRecord(c->kev[3 * slot + 1], sq));
    HIP_TRY(c, hipEventRecord(c->kev[3 * slot + 2], sq));
    return SGPM_OK;
}

void fill_result(sgpm_result* r, const NsState& s, double z, int shift) {
    r->n_samples = s.n;
    r->n_hits = s.hits;
    for (int i = 0; i < 8; i++) r->sum_digits[i] = s.S1.d[(size_t)i];
    for (int i = 0; i < 12; i++) r->sumsq_digits[i] = s.S2.d[(size_t)i];
    // learned proposal: the sums are of alpha' * 2^shift (exact integers); the
    // predicted error is invariant to that power-of-two scale
    r->estimate = s.n ? std::ldexp(big_to_double(s.S1) / (double)s.n, -shift) : 0.0;
    r->weight_shift = shift;
    r->eps_hat = predicted_error(z, s.n, s.S1, s.S2);
    r->z = z;
    const double sigma = std::isfinite(r->eps_hat) ? r->estimate * r->eps_hat / z : INFINITY;
    r->ci_lo = r->estimate - z * sigma;
    r->ci_hi = r->estimate + z * sigma;
    r->checksum = s.csum;
    r->bytes = s.bytes;
}

sgpm_status ns_estimate(sgpm_ctx* c, sgpm_graph* g, const Plan& p, const sgpm_options& o, sgpm_result* res,
                        int count_bytes, const NsExtra* ex = nullptr) {
    LearnArgs la{nullptr, nullptr, nullptr, 0};
    if (ex) la = ex->la;
    const bool learned = la.table != nullptr;
    auto t_start = std::chrono::steady_clock::now();
    std::memset(res, 0, sizeof(*res));
    res->scheme = SGPM_SCHEME_NS;
    const double z = normal_quantile(1.0 - (1.0 - o.confidence) / 2.0);
    const uint64_t M = p.oriented ? (uint64_t)g->m : 2ull * (uint64_t)g->m;
    if (M == 0) {  // no edges: the count is exactly zero
        res->z = z;
        res->converged = 1;
        res->eps_hat = 0.0;
        return SGPM_OK;
    }
    HIP_TRY(c, hipSetDevice(c->dev));
    // trace buffer
    DeviceBuffer trace_buf;
    sgpm_trace_rec* d_trace = nullptr;
    TraceArgs tr{nullptr, 0, 0, nullptr};
    const uint64_t ntr = (o.trace_buf && o.trace_hi > o.trace_lo) ? o.trace_hi - o.trace_lo : 0;
    if (ntr) {
        HIP_TRY(c, hipMalloc(&trace_buf.p, ntr * sizeof(sgpm_trace_rec)));
        d_trace = (sgpm_trace_rec*)trace_buf.p;
        HIP_TRY(c, launch_fill_u64((unsigned long long*)d_trace, ntr * sizeof(sgpm_trace_rec) / 8, 0ull, c->st));
        tr = TraceArgs{d_trace, o.trace_lo, o.trace_hi, ex ? ex->d_sizes : nullptr};
    }
    ScopedEvents<1> ev;
    HIP_TRY(c, ev.create());
    const hipEvent_t e0 = ev[0];  // start of the first window
    NsState s;
    // a prefix of the estimation stream already drawn (the loose-mode pilot):
    // part of the first window, or the whole of it (then its stop test runs
    // below, before any launch)
    uint64_t prefix_n = 0;
    bool prefix_window = false;
    if (ex && ex->prefix_n && o.mode != SGPM_MODE_FIXED_N && ex->prefix_n <= next_window_end(0, o) && !ntr &&
        !count_bytes) {
        absorb(s, ex->prefix_sums);
        prefix_n = ex->prefix_n;
        prefix_window = prefix_n == next_window_end(0, o);
        s.n = prefix_n;
    }
    int lanes = o.lanes_per_sample;
    // the learned proposal, pilot sizes and NS-base run one sample per wave
    if (learned || tr.sizes || o.sampler == SGPM_SAMPLER_BASE) lanes = 64;
    // lane counts picked earlier for this (graph, plan) are reused
    const auto tune_key = std::make_tuple((const void*)g, std::string((const char*)&p, sizeof(Plan)));
    if (lanes == 0) {
        auto it = c->ns_tuned.find(tune_key);
        if (it != c->ns_tuned.end()) lanes = it->second;
    }
    double dev_seconds = 0.0, kernel_seconds = prefix_n ? ex->prefix_kernel_s : 0.0;
    std::vector<std::pair<float, float>> spans;  // sampling kernels' [start, end) in ms after e0
    int windows = 0, launches = prefix_n ? ex->prefix_launches : 0;
    bool converged = false;
    sgpm_status status = SGPM_OK;
    // Windows are decided in order, one at a time.  A launch ends with a tail
    // (its last tickets finish at different times) and the next one starts
    // with a ramp, about 0.1 ms together; so when the error of the windows so
    // far predicts that the next window cannot stop either (the samples needed,
    // n (eps_hat / eps)^2, exceed its end by 10 %), the window after it is
    // queued at once on the second stream, where it fills the CUs the first
    // one's tail leaves idle.  The stop rule is unchanged: a window queued
    // ahead is absorbed only if every earlier one missed, and otherwise waited
    // for and dropped.  Windows use slots 0 (stream st) and 1 (st2);
    // autotune pieces 2..9 (st).
    struct Win {
        uint64_t a, b;
        size_t slot0, nslots;
    };
    std::deque<Win> inflight;
    size_t depth = 1;
    const bool may_queue_ahead = o.mode != SGPM_MODE_FIXED_N && !ntr && !count_bytes;
    uint64_t queued = prefix_n;
    size_t last_done = SIZE_MAX;
    HIP_TRY(c, hipEventRecord(e0, c->st));
    // the stop test of a first window the prefix completed, as after any window
    bool done_early = false;
    if (prefix_window) {
        windows = 1;
        const double eh = predicted_error(z, s.n, s.S1, s.S2);
        if (s.ovf) {
            status = SGPM_EOVERFLOW;
            done_early = true;
        } else if (eh <= o.eps) {
            converged = true;
            done_early = true;
        } else if (o.max_samples && s.n >= o.max_samples) {
            done_early = true;
        } else if (may_queue_ahead && std::isfinite(eh) && eh > 0) {
            const double r = eh / o.eps, need = (double)s.n * r * r;
            if (need > 1.1 * (double)next_window_end(s.n, o)) depth = 2;
        }
    }
    for (; !done_early;) {
        while (inflight.size() < depth) {
            // the window that holds sample `queued` (a prefix may end inside the first window)
            // a prefix ends inside the first window, which then starts at the prefix's end
            const uint64_t nx = o.mode == SGPM_MODE_FIXED_N ? o.fixed_n
                                : next_window_end(queued == prefix_n && !prefix_window ? 0 : queued, o);
            if (nx <= queued || (o.mode == SGPM_MODE_FIXED_N && queued > 0)) break;
            if (lanes == 0 && nx - queued >= (1ull << 19)) {
                if (!inflight.empty()) break;  // tune once the queue has drained
                // autotune on the first long window: pieces of it go to the
                // candidate lane counts from wide to narrow, two rounds, each
                // candidate judged by its better piece (the first launch of a
                // kernel pays for loading its code and for cold caches); a
                // narrower count is tried only while narrowing has paid off, so
                // a slow one (one lane per sample at a hub's row) costs one
                // small piece at most.  The rest of the window runs at the
                // winner.  Every sample is still drawn exactly once, so results
                // are unchanged.
                static const int cand[4] = {64, 16, 4, 1};
                constexpr int kPieces = 16;
                const uint64_t len = nx - queued;
                float best_per[4] = {0, 0, 0, 0};
                bool seen[4] = {false, false, false, false};
                size_t used = 0;
                int ntry = 2;  // candidates in play
                uint64_t done_to = queued;
                for (int i = 0; i < 8; i++) {
                    const int ci = i % 4;
                    if (ci >= ntry) continue;
                    const uint64_t a = done_to, b = queued + len * (uint64_t)(used + 1) / kPieces;
                    done_to = b;
                    const size_t slot = 2 + used++;
                    status = enqueue_range(c, g, p, o, a, b, cand[ci], slot, tr, count_bytes, la, len);
                    if (status != SGPM_OK) return status;
                    // sampling-kernel time alone (the events enqueue_range records around it)
                    HIP_TRY(c, hipEventSynchronize(c->kev[3 * slot + 1]));
                    float ms = 0;
                    HIP_TRY(c, hipEventElapsedTime(&ms, c->kev[3 * slot], c->kev[3 * slot + 1]));
                    const float per = ms / (float)(b - a);
                    if (std::getenv("SGPM_DEBUG"))
                        std::fprintf(stderr, "sgpm autotune: lanes=%d %.3f ms for %llu samples (%.4g samples/s)\n",
                                     cand[ci], ms, (unsigned long long)(b - a), (double)(b - a) / (ms * 1e-3));
                    if (!seen[ci] || per < best_per[ci]) best_per[ci] = per;
                    seen[ci] = true;
                    // the narrower candidate won its first piece: try the next one too
                    if (i < 4 && ci >= 1 && ci + 1 == ntry && ntry < 4 && best_per[ci] < best_per[ci - 1]) ntry++;
                }
                int best = 64;
                float best_ms = 0;
                for (int ci = 0; ci < 4; ci++)
                    if (seen[ci] && (best_ms == 0 || best_per[ci] < best_ms)) {
                        best_ms = best_per[ci];
                        best = cand[ci];
                    }
                lanes = best;
                c->ns_tuned[tune_key] = best;
                if (done_to < nx) {  // the rest of the window at the winner
                    const size_t slot = 2 + used++;
                    status = enqueue_range(c, g, p, o, done_to, nx, best, slot, tr, count_bytes, la, len);
                    if (status != SGPM_OK) return status;
                }
                inflight.push_back(Win{queued, nx, 2, used});
                queued = nx;
                break;
            }
            // short windows before tuning: one sample per wave, not remembered;
            // the slot (and stream) no window in flight holds
            bool busy0 = false;
            for (const Win& w : inflight) busy0 = busy0 || w.slot0 == 0;
            const size_t slot = busy0 ? 1 : 0;
            status = enqueue_range(c, g, p, o, queued, nx, lanes ? lanes : 64, slot, tr, count_bytes, la, 0, slot == 1);
            if (status != SGPM_OK) return status;
            inflight.push_back(Win{queued, nx, slot, 1});
            queued = nx;
        }
        if (inflight.empty()) break;
        const Win w = inflight.front();
        inflight.pop_front();
        const size_t lastslot = w.slot0 + w.nslots - 1;
        HIP_TRY(c, hipEventSynchronize(c->kev[3 * lastslot + 2]));
        for (size_t k = w.slot0; k <= lastslot; k++) {
            absorb(s, c->h_slots + k * SLOT_WORDS + 1);
            float kms = 0, ka = 0, kb = 0;
            HIP_TRY(c, hipEventElapsedTime(&kms, c->kev[3 * k], c->kev[3 * k + 1]));
            HIP_TRY(c, hipEventElapsedTime(&ka, e0, c->kev[3 * k]));
            HIP_TRY(c, hipEventElapsedTime(&kb, e0, c->kev[3 * k + 1]));
            spans.emplace_back(ka, kb);
            kernel_seconds += kms * 1e-3;
            launches++;
        }
        last_done = lastslot;
        s.n = w.b;
        windows++;
        if (s.ovf) {
            status = SGPM_EOVERFLOW;
            break;
        }
        if (o.mode == SGPM_MODE_FIXED_N) break;
        const double eh = predicted_error(z, s.n, s.S1, s.S2);
        if (eh <= o.eps) {
            converged = true;
            break;
        }
        if (o.max_samples && s.n >= o.max_samples) break;
        depth = 1;
        if (may_queue_ahead && std::isfinite(eh) && eh > 0) {
            const uint64_t next_end = inflight.empty() ? next_window_end(s.n, o) : inflight.back().b;
            const double r = eh / o.eps, need = (double)s.n * r * r;
            if (need > 1.1 * (double)next_end) depth = 2;
        }
    }
    // windows queued ahead past the stop: wait for them (their slots and the
    // second stream are reused by the next call) and drop their sums
    for (const Win& w : inflight) HIP_TRY(c, hipEventSynchronize(c->kev[3 * (w.slot0 + w.nslots - 1) + 2]));
    if (last_done != SIZE_MAX) {
        float ms = 0;
        HIP_TRY(c, hipEventElapsedTime(&ms, e0, c->kev[3 * last_done + 2]));
        dev_seconds = ms * 1e-3;
    }
    fill_result(res, s, z, learned ? 52 : 0);
    res->windows = windows;
    res->lanes_per_sample = lanes ? lanes : 64;
    res->seconds_sampling = dev_seconds;
    res->seconds_kernel = kernel_seconds;
    {
        // union of the kernels' intervals (windows queued ahead overlap)
        std::sort(spans.begin(), spans.end());
        double busy = 0.0, a = -1.0, b = -1.0;
        for (const auto& sp : spans) {
            if (sp.first > b) {
                if (b > a) busy += b - a;
                a = sp.first;
                b = sp.second;
            } else if (sp.second > b) {
                b = sp.second;
            }
        }
        if (b > a) busy += b - a;
        // a prefix's launches ran before e0, one after another
        res->seconds_kernel_busy = busy * 1e-3 + (prefix_n ? ex->prefix_kernel_s : 0.0);
    }
    res->launches = launches;
    if (o.mode == SGPM_MODE_FIXED_N) converged = res->eps_hat <= o.eps;
    res->converged = converged ? 1 : 0;
    if (ntr) {
        HIP_TRY(c, hipMemcpy(o.trace_buf, d_trace, ntr * sizeof(sgpm_trace_rec), hipMemcpyDeviceToHost));
    }
    res->seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (status != SGPM_OK) return fail(c, status, "a sample weight exceeded 128 bits");
    if (!converged && o.mode != SGPM_MODE_FIXED_N) return fail(c, SGPM_NOT_CONVERGED, "max_samples reached");
    return SGPM_OK;
}

}  // namespace

namespace sgpm {
sgpm_status ns_estimate_solo(sgpm_ctx* c, sgpm_graph* g, const Plan& p, const sgpm_options& o, sgpm_result* res,
                             int count_bytes, const NsExtra* ex) {
    return ns_estimate(c, g, p, o, res, count_bytes, ex);
}

sgpm_status ns_pilot(sgpm_ctx* c, sgpm_graph* g, const Plan& p, const sgpm_options& o, const LearnArgs& la,
                     int slices, const uint64_t* slice_end, double* seconds, double* eps_hat, double* mean,
                     unsigned long long* sums_out) {
    HIP_TRY(c, hipSetDevice(c->dev));
    const double z = normal_quantile(1.0 - (1.0 - o.confidence) / 2.0);
    int lanes = o.lanes_per_sample;
    if (la.table) lanes = 64;
    if (lanes == 0) {
        auto it = c->ns_tuned.find(std::make_tuple((const void*)g, std::string((const char*)&p, sizeof(Plan))));
        lanes = it != c->ns_tuned.end() ? it->second : 64;
    }
    const TraceArgs tr{nullptr, 0, 0, nullptr};
    const uint64_t n = slice_end[slices - 1];
    for (int i = 0; i < slices; i++) {
        const uint64_t a = i ? slice_end[i - 1] : 0, b = slice_end[i];
        sgpm_status st = enqueue_range(c, g, p, o, a, b, lanes, (size_t)i, tr, 0, la, b - a);
        if (st != SGPM_OK) return st;
    }
    HIP_TRY(c, hipStreamSynchronize(c->st));
    NsState all;
    if (sums_out)
        for (int w = 0; w < PF_N; w++) sums_out[w] = 0;
    for (int i = 0; i < slices; i++) {
        const uint64_t a = i ? slice_end[i - 1] : 0, b = slice_end[i];
        const unsigned long long* sl = c->h_slots + (size_t)i * SLOT_WORDS + 1;
        NsState s;
        absorb(s, sl);
        absorb(all, sl);
        if (sums_out)
            for (int w = 0; w < PF_N; w++) sums_out[w] += sl[w];
        s.n = b - a;
        float ms = 0;
        HIP_TRY(c, hipEventElapsedTime(&ms, c->kev[3 * (size_t)i], c->kev[3 * (size_t)i + 1]));
        seconds[i] = ms * 1e-3;
        eps_hat[i] = predicted_error(z, s.n, s.S1, s.S2);
    }
    // the pilot's estimate of the count (learned: sums of alpha' * 2^52)
    if (mean) *mean = n ? std::ldexp(big_to_double(all.S1) / (double)n, la.table ? -52 : 0) : 0.0;
    return SGPM_OK;
}
}  // namespace sgpm

namespace {

sgpm_status check_options(sgpm_ctx* c, const sgpm_options* o) {
    if (!o) return fail(c, SGPM_EINVAL, "null options");
    if (!(o->eps > 0) || !(o->confidence > 0 && o->confidence < 1)) return fail(c, SGPM_EINVAL, "eps/confidence");
    if (o->mode == SGPM_MODE_FIXED_N && o->fixed_n == 0) return fail(c, SGPM_EINVAL, "fixed_n = 0");
    if ((o->mode == SGPM_MODE_STRICT_NS || o->mode == SGPM_MODE_HYBRID) && o->n_min == 0)
        return fail(c, SGPM_EINVAL, "n_min = 0: the first window would be empty");
    if (!(o->window_growth >= 0)) return fail(c, SGPM_EINVAL, "window_growth");
    const int l = o->lanes_per_sample;
    if (!(l == 0 || l == 1 || l == 4 || l == 16 || l == 64)) return fail(c, SGPM_EINVAL, "lanes_per_sample");
    if (o->trace_hi > o->trace_lo && !o->trace_buf) return fail(c, SGPM_EINVAL, "trace range without buffer");
    if (o->sampler != SGPM_SAMPLER_PRUNE && o->sampler != SGPM_SAMPLER_BASE) return fail(c, SGPM_EINVAL, "sampler");
    if (o->gs_scheme != SGPM_GS_COLOUR && o->gs_scheme != SGPM_GS_BERNOULLI) return fail(c, SGPM_EINVAL, "gs_scheme");
    if (o->gs_scheme == SGPM_GS_BERNOULLI && o->mode != SGPM_MODE_GS)
        return fail(c, SGPM_EUNSUPPORTED, "Bernoulli edge sparsification runs in the GS mode");
    if (o->sampler == SGPM_SAMPLER_BASE &&
        ((o->mode != SGPM_MODE_STRICT_NS && o->mode != SGPM_MODE_FIXED_N) || o->proposal))
        return fail(c, SGPM_EUNSUPPORTED, "NS-base runs in the strict and fixed-n modes with the uniform proposal");
    return SGPM_OK;
}

}  // namespace

extern "C" {

sgpm_status sgpm_estimate(sgpm_ctx_t c, sgpm_graph_t g, sgpm_pattern_t p, const sgpm_options* o, sgpm_result* res) {
    if (!c || !g || !p || !res) return fail(c, SGPM_EINVAL, "null argument");
    sgpm_status st = check_options(c, o);
    if (st != SGPM_OK) return st;
    switch (o->mode) {
        case SGPM_MODE_STRICT_NS:
        case SGPM_MODE_FIXED_N: {
            if (!o->proposal) return ns_estimate(c, g, p->plan, *o, res, 0);
            NsExtra ex{};
            sgpm_status st2 = learn_args_for(c, g, p, o->proposal, &ex.la);
            if (st2 != SGPM_OK) return st2;
            return ns_estimate(c, g, p->plan, *o, res, 0, &ex);
        }
        case SGPM_MODE_GS:
            return gs_estimate(c, g, p->plan, *o, res);
        case SGPM_MODE_HYBRID:
            return hybrid_estimate(c, g, p, *o, res);
        default:
            return fail(c, SGPM_EUNSUPPORTED, "mode not available");
    }
}

// Same as sgpm_estimate in NS modes, additionally filling result.bytes with the
// algorithmic bytes of every sample (measurement build of the kernel).
sgpm_status sgpm_estimate_counted(sgpm_ctx_t c, sgpm_graph_t g, sgpm_pattern_t p, const sgpm_options* o,
                                  sgpm_result* res) {
    if (!c || !g || !p || !res) return fail(c, SGPM_EINVAL, "null argument");
    sgpm_status st = check_options(c, o);
    if (st != SGPM_OK) return st;
    if (o->mode != SGPM_MODE_STRICT_NS && o->mode != SGPM_MODE_FIXED_N)
        return fail(c, SGPM_EUNSUPPORTED, "byte counting is for NS modes");
    if (o->proposal) return fail(c, SGPM_EUNSUPPORTED, "byte counting is for the uniform proposal");
    if (o->sampler == SGPM_SAMPLER_BASE) return fail(c, SGPM_EUNSUPPORTED, "byte counting is for NS-prune");
    return ns_estimate(c, g, p->plan, *o, res, 1);
}

}  // extern "C"

// ------------------------------------------------------------------ host-only utilities
extern "C" {

sgpm_status sgpm_host_canonicalise(int64_t n, const void* offsets, int offsets_is_64, const int32_t* nbrs,
                                   uint32_t flags, int64_t* m_out, int64_t* off_out, int32_t* nbr_out,
                                   int32_t* perm_out) {
    if (!offsets || n < 0 || n >= (1ll << 31)) return SGPM_EINVAL;
    if (flags & ~(SGPM_ASSUME_CANONICAL | SGPM_SYMMETRIZE)) return SGPM_EINVAL;  // host arrays only
    if ((flags & SGPM_ASSUME_CANONICAL) && (flags & SGPM_SYMMETRIZE)) return SGPM_EINVAL;
    HostGraph h;
    std::string err;
    int rc = canonicalise(n, offsets, offsets_is_64, nbrs, (flags & SGPM_ASSUME_CANONICAL) != 0, h, err);
    if (rc != SGPM_OK) return (sgpm_status)rc;
    if (m_out) *m_out = h.m;
    if (off_out) std::memcpy(off_out, h.off.data(), sizeof(int64_t) * (size_t)(n + 1));
    if (nbr_out && h.m) std::memcpy(nbr_out, h.nbr.data(), sizeof(int32_t) * (size_t)(2 * h.m));
    if (perm_out && n) std::memcpy(perm_out, h.perm.data(), sizeof(int32_t) * (size_t)n);
    return SGPM_OK;
}

sgpm_status sgpm_host_plan(int k, int l, const int32_t* edges, int induced, int32_t* order, uint8_t* connect,
                           uint8_t* disconnect, uint8_t* upper, uint8_t* lower, int32_t* aut_size,
                           int32_t* oriented) {
    sgpm_pattern p;
    std::string err;
    int rc = compile_pattern(k, l, edges, induced, p.plan, err);
    if (rc != SGPM_OK) return (sgpm_status)rc;
    return sgpm_pattern_plan(&p, order, connect, disconnect, upper, lower, aut_size, oriented);
}

double sgpm_host_normal_quantile(double p) { return normal_quantile(p); }

double sgpm_host_predicted_error(double z, uint64_t n, const uint32_t* s1, int n1, const uint32_t* s2, int n2) {
    Big S1(24), S2(24);
    for (int i = 0; i < n1 && i < 24; i++) S1.d[(size_t)i] = s1[i];
    for (int i = 0; i < n2 && i < 24; i++) S2.d[(size_t)i] = s2[i];
    return predicted_error(z, n, S1, S2);
}

double sgpm_host_t_quantile(double conf, int nu) { return student_t_quantile(conf, nu); }

double sgpm_host_predicted_error_t(double t, uint64_t n, const uint32_t* s1, int n1, const uint32_t* s2, int n2) {
    Big S1(24), S2(24);
    for (int i = 0; i < n1 && i < 24; i++) S1.d[(size_t)i] = s1[i];
    for (int i = 0; i < n2 && i < 24; i++) S2.d[(size_t)i] = s2[i];
    return predicted_error_t(t, n, S1, S2);
}

uint64_t sgpm_host_next_window(uint64_t n_t, const sgpm_options* o) { return o ? next_window_end(n_t, *o) : 0; }

int sgpm_host_colours_choice(int64_t m, int k, double leaves16) {
    if (m < 0 || k < 2 || k > 8 || !(leaves16 >= 0)) return SGPM_EINVAL;
    return (int)colours_from_probe(m, k, leaves16);
}

int sgpm_host_hybrid_choice(double ns_lo, double eps, double confidence, int gs_reps_run, double gs_rep_seconds,
                            double gs_cv, int gs_reps_max, double* gs_pred) {
    if (!(eps > 0) || !(confidence > 0 && confidence < 1)) return SGPM_EINVAL;
    return hybrid_choice(ns_lo, eps, confidence, gs_reps_run, gs_rep_seconds, gs_cv, gs_reps_max, gs_pred);
}

int sgpm_host_ns_cone(int slices, const double* slice_n, const double* slice_seconds, const double* slice_eps_hat,
                      const sgpm_options* o, double* lo, double* hi, double* t0, double* rate) {
    if (slices < 1 || !slice_n || !slice_seconds || !slice_eps_hat || !o || !lo || !hi || !(o->eps > 0))
        return SGPM_EINVAL;
    ns_cone(slices, slice_n, slice_seconds, slice_eps_hat, *o, lo, hi, t0, rate);
    return SGPM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ entry points built in later modules
extern "C" {
}

// ------------------------------------------------------------------ measurement probes
extern "C" {

sgpm_status sgpm_probe_copy(sgpm_ctx_t c, uint64_t bytes, int iters, double* gbs) {
    if (!c || !gbs || bytes < 16 || iters < 1) return fail(c, SGPM_EINVAL, "bad probe arguments");
    HIP_TRY(c, hipSetDevice(c->dev));
    bytes &= ~15ull;
    DeviceBuffer a, b;
    HIP_TRY(c, hipMalloc(&a.p, bytes));
    HIP_TRY(c, hipMalloc(&b.p, bytes));
    HIP_TRY(c, hipMemsetAsync(a.p, 1, bytes, c->st));
    const int blocks = c->cus * 8;
    HIP_TRY(c, probe_copy(a.p, b.p, bytes, blocks, c->st));  // warm
    ScopedEvents<2> ev;
    HIP_TRY(c, ev.create());
    HIP_TRY(c, hipEventRecord(ev[0], c->st));
    for (int i = 0; i < iters; i++) HIP_TRY(c, probe_copy(a.p, b.p, bytes, blocks, c->st));
    HIP_TRY(c, hipEventRecord(ev[1], c->st));
    HIP_TRY(c, hipEventSynchronize(ev[1]));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, ev[0], ev[1]));
    *gbs = 2.0 * (double)bytes * iters / (ms * 1e-3) / 1e9;
    return SGPM_OK;
}

sgpm_status sgpm_probe_gather(sgpm_ctx_t c, uint64_t working_set_bytes, int segment_bytes, int rounds, double* gbs) {
    if (!c || !gbs || segment_bytes < 4 || segment_bytes > 256 || (segment_bytes & (segment_bytes - 1)) ||
        working_set_bytes < (uint64_t)segment_bytes || rounds < 1)
        return fail(c, SGPM_EINVAL, "bad probe arguments");
    HIP_TRY(c, hipSetDevice(c->dev));
    const uint64_t words = working_set_bytes / 4;
    DeviceBuffer ab, sb;
    HIP_TRY(c, hipMalloc(&ab.p, words * 4));
    HIP_TRY(c, hipMalloc(&sb.p, 8));
    int32_t* a = (int32_t*)ab.p;
    unsigned long long* sink = (unsigned long long*)sb.p;
    HIP_TRY(c, hipMemsetAsync(a, 3, words * 4, c->st));
    const int blocks = c->cus * 8;
    HIP_TRY(c, probe_gather(a, words, segment_bytes, rounds, blocks, 1, sink, c->st));
    ScopedEvents<2> ev;
    HIP_TRY(c, ev.create());
    HIP_TRY(c, hipEventRecord(ev[0], c->st));
    HIP_TRY(c, probe_gather(a, words, segment_bytes, rounds, blocks, 2, sink, c->st));
    HIP_TRY(c, hipEventRecord(ev[1], c->st));
    HIP_TRY(c, hipEventSynchronize(ev[1]));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, ev[0], ev[1]));
    const double segs = (double)blocks * 256.0 / (segment_bytes / 4) * rounds;
    *gbs = segs * segment_bytes / (ms * 1e-3) / 1e9;
    return SGPM_OK;
}

}  // extern "C"
