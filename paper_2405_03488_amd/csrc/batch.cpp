// Batched estimation: many (graph, pattern) NS queries in one persistent,
// hipGraph-captured launch, each query sampled with its own lane count (one
// sample per wave, or groups of 16, 4 or 1 lanes per sample), with an
// autotuner that picks each query's lane count and ticket size from timed
// pilot samples.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>

#include "sgpm_internal.h"

namespace sgpm {

namespace {

// Autotuner: pick a query's lanes per sample and its ticket size from timed
// pilot samples (Philox tag 0x80000000 | tag, so they never overlap estimation
// samples).  Lane counts: the caller's lanes_per_sample if set, else the count
// the solo estimate chose for this (graph, plan) if it ran, else candidates
// from wide to narrow (64, 16, 4, 1), two timed rounds each (the first launch
// of a kernel pays for its code and cold caches), a narrower count tried only
// while narrowing paid off.  The tile (samples per ticket) is sized to about
// 400 us of wave time at the chosen count, so uneven queries hand out tickets
// of similar cost and the persistent grid drains evenly: for G lanes per sample
// a wave holds 64/G samples at once, so its samples per lane are tile / (64/G).
sgpm_status autotune_query(sgpm_ctx* c, sgpm_graph* g, const Plan& p, const sgpm_options& o, int* lanes_out,
                           int* tile) {
    sgpm_options po = o;
    po.mode = SGPM_MODE_FIXED_N;
    po.query_tag = 0x80000000u | (o.query_tag & 0x7FFFFFFFu);
    po.checksum = 0;
    po.trace_buf = nullptr;
    po.trace_lo = po.trace_hi = 0;
    int cand[4] = {64, 16, 4, 1};
    int ncand = 4;
    if (o.lanes_per_sample) {
        cand[0] = o.lanes_per_sample;
        ncand = 1;
    } else {
        auto it = c->ns_tuned.find(std::make_tuple((const void*)g, std::string((const char*)&p, sizeof(Plan))));
        if (it != c->ns_tuned.end()) {
            cand[0] = it->second;
            ncand = 1;
        }
    }
    double best[4] = {0, 0, 0, 0};
    int ntry = ncand == 1 ? 1 : 2;  // candidates in play
    for (int round = 0; round < 2; round++)
        for (int ci = 0; ci < ntry; ci++) {
            po.lanes_per_sample = cand[ci];
            po.fixed_n = cand[ci] == 64 ? (1u << 18) : (1u << 17);
            sgpm_result r;
            sgpm_status st = ns_estimate_solo(c, g, p, po, &r, 0);
            if (st != SGPM_OK && st != SGPM_NOT_CONVERGED) return st;
            const double per = r.seconds_kernel / (double)po.fixed_n;
            if (std::getenv("SGPM_DEBUG"))
                std::fprintf(stderr, "sgpm batch autotune: lanes=%d %.4g s per sample\n", cand[ci], per);
            if (round == 0 || per < best[ci]) best[ci] = per;
            // the narrower count won its first run: the next one is tried too
            if (round == 0 && ci >= 1 && ci + 1 == ntry && ntry < ncand && best[ci] < best[ci - 1]) ntry++;
        }
    int bi = 0;
    for (int ci = 1; ci < ntry; ci++)
        if (best[ci] < best[bi]) bi = ci;
    const int L = cand[bi];
    const bool clq = L == 64 && wave_uses_clique_kernel(p, TraceArgs{}, LearnArgs{}, 0);
    const double waves = (double)c->cus * (double)(clq ? ns_clique_blocks_per_cu() : ns_blocks_per_cu(L)) * 4.0;
    const double wave_time_per_sample = best[bi] * waves;
#ifndef SGPM_TILE_US
#define SGPM_TILE_US 400
#endif
    // at least 16 samples (a sample per wave: one group of the draw and
    // first-edge prefetch; smaller tiles were slower even for queries whose
    // samples take a wave a millisecond on hub rows) and a round of the
    // wave's lane groups
    const int per_round = 64 / L;  // samples a wave holds at once
    const int tmin = std::max(16, per_round), tmax = std::max(1024, 256 * per_round);
    double t = wave_time_per_sample > 0 ? SGPM_TILE_US * 1e-6 / wave_time_per_sample : (double)tmax;
    int tl = tmin;
    while (tl < tmax && tl * 2 <= 1.5 * t) tl *= 2;  // the power of two nearest t
    *tile = tl;
    *lanes_out = L;
    if (std::getenv("SGPM_DEBUG"))
        std::fprintf(stderr, "sgpm batch autotune: lanes %d, %.3g us wave time per sample -> tile %d\n", L,
                     wave_time_per_sample * 1e6, tl);
    return SGPM_OK;
}

}  // namespace

sgpm_status batch_estimate(sgpm_ctx* c, int nq, const sgpm_graph_t* graphs, const sgpm_pattern_t* patterns,
                           const sgpm_options* opts, sgpm_result* res) {
    auto t0 = std::chrono::steady_clock::now();
    if (nq <= 0 || !graphs || !patterns || !opts || !res) return fail(c, SGPM_EINVAL, "bad batch arguments");
    HIP_TRY(c, hipSetDevice(c->dev));
    std::vector<BatchQuery> hq((size_t)nq);
    std::vector<BatchState> hs((size_t)nq);
    std::memset(hs.data(), 0, sizeof(BatchState) * (size_t)nq);
    unsigned long long active = 0;
    for (int i = 0; i < nq; i++) {
        const sgpm_options& o = opts[i];
        if (!graphs[i] || !patterns[i]) return fail(c, SGPM_EINVAL, "null graph or pattern in batch");
        if (o.mode != SGPM_MODE_STRICT_NS && o.mode != SGPM_MODE_FIXED_N)
            return fail(c, SGPM_EUNSUPPORTED, "batch queries must be NS (strict or fixed-n)");
        if (o.trace_buf || o.proposal) return fail(c, SGPM_EUNSUPPORTED, "batch queries take no trace or proposal");
        if (o.sampler != SGPM_SAMPLER_PRUNE) return fail(c, SGPM_EUNSUPPORTED, "batch queries use NS-prune");
        const int l = o.lanes_per_sample;
        if (!(l == 0 || l == 1 || l == 4 || l == 16 || l == 64)) return fail(c, SGPM_EINVAL, "lanes_per_sample");
        if (!(o.eps > 0) || !(o.confidence > 0 && o.confidence < 1)) return fail(c, SGPM_EINVAL, "eps/confidence");
        if (o.mode == SGPM_MODE_FIXED_N && o.fixed_n == 0) return fail(c, SGPM_EINVAL, "fixed_n = 0");
        // every window must hold a tile, or its query would never complete
        if (o.mode == SGPM_MODE_STRICT_NS && o.n_min == 0)
            return fail(c, SGPM_EINVAL, "n_min = 0: the first window would be empty");
        // Window columns hold sums of 32-bit digits, so a window must stay
        // below 2^32 samples: window_cap = the first window that would not.
        int window_cap = 0x7FFFFFFF;
        {
            uint64_t n = 0;
            for (int t = 0; t < 1000000; t++) {
                const uint64_t nx = o.mode == SGPM_MODE_FIXED_N ? o.fixed_n : next_window_end(n, o);
                if (nx <= n) break;
                if (nx - n >= (1ull << 32)) {
                    window_cap = t;
                    break;
                }
                n = nx;
                if (o.mode == SGPM_MODE_FIXED_N) break;
            }
            if (window_cap == 0) return fail(c, SGPM_EUNSUPPORTED, "batch windows must stay below 2^32 samples");
        }
        sgpm_graph* g = graphs[i];
        const Plan& p = patterns[i]->plan;
        BatchQuery& Q = hq[(size_t)i];
        Q.g = g->view();
        Q.p = p;
        Q.seed = o.seed;
        Q.tag = o.query_tag;
        Q.mode = o.mode;
        Q.fixed_n = o.fixed_n;
        Q.n_min = o.n_min;
        Q.w_min = o.w_min;
        Q.quantum = o.quantum;
        Q.max_samples = o.max_samples;
        Q.growth = o.window_growth;
        Q.eps = o.eps;
        Q.z = normal_quantile(1.0 - (1.0 - o.confidence) / 2.0);
        const uint64_t M = p.oriented ? (uint64_t)g->m : 2ull * (uint64_t)g->m;
        int tile = 64, lanes = o.lanes_per_sample ? o.lanes_per_sample : 64;
        if (M > 0) {
            auto key = std::make_tuple((const void*)g, std::string((const char*)&p, sizeof(Plan)), o.lanes_per_sample);
            auto it = c->tuned.find(key);
            if (it != c->tuned.end()) {
                lanes = it->second.first;
                tile = it->second.second;
            } else {
                sgpm_status st = autotune_query(c, g, p, o, &lanes, &tile);
                if (st != SGPM_OK) return st;
                c->tuned[key] = std::make_pair(lanes, tile);
            }
        }
        Q.lanes = lanes;
        Q.tile = tile;
        Q.window_cap = window_cap;
        if (M == 0) {
            hs[(size_t)i].finished = 1;
            hs[(size_t)i].converged = 1;
        } else {
            active++;
        }
    }
    // device buffers and the captured graph, rebuilt when the batch shape changes
    const size_t qbytes = sizeof(BatchQuery) * (size_t)nq, sbytes = sizeof(BatchState) * (size_t)nq;
    int kmax = 2;
    for (int i = 0; i < nq; i++) kmax = std::max(kmax, patterns[i]->plan.k);
    kmax = batch_kmax(kmax);
    // some query with fewer than 64 lanes per sample: the build with the
    // lane-group samplers; else, every query a clique of at most 6 vertices:
    // tiles run the clique sampler
    bool grp = false;
    for (int i = 0; i < nq; i++) grp = grp || hq[(size_t)i].lanes != 64;
    bool clq = kmax <= 6 && !grp;
    for (int i = 0; i < nq; i++)
        clq = clq && plan_is_clique(patterns[i]->plan) && patterns[i]->plan.k >= 3 && patterns[i]->plan.k <= kmax;
    if (c->batch_nq != nq || c->batch_kmax != kmax || c->batch_clq != clq || c->batch_grp != grp) {
        if (c->batch_exec) (void)hipGraphExecDestroy(c->batch_exec);
        if (c->batch_graph) (void)hipGraphDestroy(c->batch_graph);
        c->batch_exec = nullptr;
        c->batch_graph = nullptr;
        if (c->d_bq) (void)hipFree(c->d_bq);
        if (c->h_bq) (void)hipHostFree(c->h_bq);
        c->d_bq = c->h_bq = nullptr;
        const size_t total = qbytes + sbytes + 64;
        HIP_TRY(c, hipMalloc(&c->d_bq, total));
        HIP_TRY(c, hipHostMalloc(&c->h_bq, total, hipHostMallocDefault));
        if (!c->batch_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->batch_stream, hipStreamNonBlocking));
        const int blocks = c->cus * batch_blocks_per_cu(kmax, clq, grp);
        char* d = (char*)c->d_bq;
        char* h = (char*)c->h_bq;
        BatchQuery* dq = (BatchQuery*)d;
        BatchState* ds = (BatchState*)(d + qbytes);
        unsigned long long* dact = (unsigned long long*)(d + qbytes + sbytes);
        HIP_TRY(c, hipStreamBeginCapture(c->batch_stream, hipStreamCaptureModeThreadLocal));
        HIP_TRY(c, hipMemcpyAsync(d, h, qbytes + sbytes + 8, hipMemcpyHostToDevice, c->batch_stream));
        HIP_TRY(c, launch_batch(dq, ds, nq, dact, blocks, kmax, clq, grp, c->batch_stream));
        HIP_TRY(c, hipMemcpyAsync(h + qbytes, d + qbytes, sbytes, hipMemcpyDeviceToHost, c->batch_stream));
        HIP_TRY(c, hipStreamEndCapture(c->batch_stream, &c->batch_graph));
        HIP_TRY(c, hipGraphInstantiate(&c->batch_exec, c->batch_graph, nullptr, nullptr, 0));
        c->batch_nq = nq;
        c->batch_kmax = kmax;
        c->batch_clq = clq;
        c->batch_grp = grp;
    }
    char* h = (char*)c->h_bq;
    std::memcpy(h, hq.data(), qbytes);
    std::memcpy(h + qbytes, hs.data(), sbytes);
    std::memcpy(h + qbytes + sbytes, &active, 8);
    ScopedEvents<2> ev;
    HIP_TRY(c, ev.create());
    HIP_TRY(c, hipEventRecord(ev[0], c->batch_stream));
    if (active > 0) HIP_TRY(c, hipGraphLaunch(c->batch_exec, c->batch_stream));
    HIP_TRY(c, hipEventRecord(ev[1], c->batch_stream));
    HIP_TRY(c, hipStreamSynchronize(c->batch_stream));
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    const BatchState* out = (const BatchState*)(h + qbytes);
    const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    sgpm_status worst = SGPM_OK;
    for (int i = 0; i < nq; i++) {
        const BatchState& S = active > 0 ? out[i] : hs[(size_t)i];
        const BatchQuery& Q = hq[(size_t)i];
        sgpm_result* r = &res[i];
        std::memset(r, 0, sizeof(*r));
        r->scheme = SGPM_SCHEME_NS;
        r->z = Q.z;
        r->n_samples = S.n;
        r->n_hits = S.hits;
        Big S1(24), S2(24);
        for (int k = 0; k < 8; k++) S1.d[(size_t)k] = (uint32_t)S.tot_s1[k];
        for (int k = 0; k < 12; k++) S2.d[(size_t)k] = (uint32_t)S.tot_s2[k];
        for (int k = 0; k < 8; k++) r->sum_digits[k] = S1.d[(size_t)k];
        for (int k = 0; k < 12; k++) r->sumsq_digits[k] = S2.d[(size_t)k];
        r->estimate = S.n ? big_to_double(S1) / (double)S.n : 0.0;
        r->eps_hat = S.n ? predicted_error(Q.z, S.n, S1, S2) : 0.0;
        const double sigma = std::isfinite(r->eps_hat) ? r->estimate * r->eps_hat / Q.z : INFINITY;
        r->ci_lo = r->estimate - Q.z * sigma;
        r->ci_hi = r->estimate + Q.z * sigma;
        r->converged = S.converged;
        r->windows = S.windows;
        r->lanes_per_sample = Q.lanes;
        r->tile = Q.tile;
        r->launches = 1;
        r->checksum = opts[i].checksum ? S.csum : 0;
        r->seconds_kernel = ms * 1e-3;
        r->seconds_sampling = ms * 1e-3;
        r->seconds_total = wall;
        sgpm_status st = SGPM_OK;
        if (active > 0 && !S.finished) st = SGPM_EHIP;  // the launch's watchdog ended it
        else if (S.status) st = (sgpm_status)S.status;
        else if (S.n && memcmp(&r->eps_hat, &S.eps_hat, sizeof(double)) != 0 &&
                 !(std::isinf(r->eps_hat) && std::isinf(S.eps_hat)))
            st = SGPM_EHIP;  // the device's stop test disagrees with the host's arithmetic
        else if (!S.converged && Q.mode != SGPM_MODE_FIXED_N)
            st = SGPM_NOT_CONVERGED;
        if (st != SGPM_OK && (worst == SGPM_OK || worst == SGPM_NOT_CONVERGED)) worst = st;
    }
    if (worst == SGPM_EHIP) return fail(c, worst, "device stop test differs from the host's, or the batch watchdog fired");
    if (worst == SGPM_EUNSUPPORTED) return fail(c, worst, "a query needed a window of 2^32 samples or more");
    if (worst == SGPM_EOVERFLOW) return fail(c, worst, "a sample weight exceeded 128 bits");
    if (worst == SGPM_NOT_CONVERGED) return fail(c, worst, "a query reached max_samples");
    return SGPM_OK;
}

}  // namespace sgpm

extern "C" sgpm_status sgpm_estimate_batch(sgpm_ctx_t c, int nq, const sgpm_graph_t* graphs,
                                           const sgpm_pattern_t* patterns, const sgpm_options* opts,
                                           sgpm_result* res) {
    if (!c) return SGPM_EINVAL;
    return sgpm::batch_estimate(c, nq, graphs, patterns, opts, res);
}
