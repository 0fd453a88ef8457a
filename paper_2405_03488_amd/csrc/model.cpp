// Learned proposal: model handles, the training driver and test hooks.
//
// Training (all compute on the GPU): for every pattern, 2^18 pilot NS samples
// (uniform proposal, Philox tag 0x80000000 | pattern index) are traced with
// their per-step candidate-set sizes.  Each step j that chose a vertex gives a
// tuple: features (candidate bucket, buckets of v_0 and v_{j-1}, step,
// pattern one-hot) and target log2(1 + Y), Y = prod_{t > j} |S_t| for a hit
// (the number of completions the walk's remaining choices represent) and 0
// for a miss.  The MLP regresses the target with Adam on the MFMA kernels.
// The weight table is the MLP evaluated on every (step, b0, b_prev, b_cand):
// w = clamp(round(2^(s - max_cand s + 15)), 1, 65535) per (step, b0, b_prev),
// so only the relative scores of candidate buckets matter.  The table is
// frozen before any estimation sample is drawn.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>

#include "sgpm_internal.h"

namespace sgpm {

namespace {

constexpr size_t TABLE = 8 * 32 * 32 * 32;
constexpr int NFEAT = 16;

bool same_plan(const Plan& a, const Plan& b) {
    return a.k == b.k && a.oriented == b.oriented && a.induced == b.induced &&
           !memcmp(a.connect, b.connect, 8) && !memcmp(a.disconnect, b.disconnect, 8) && !memcmp(a.upper, b.upper, 8) &&
           !memcmp(a.lower, b.lower, 8);
}

int bucket_host(const sgpm_graph* g, int32_t v) {
    int b = 0;
    while (b < 31 && v < g->bthr[b]) b++;
    return b;
}

void features(float* x, int pattern, int j, int b0, int bp, int bc) {
    x[0] = bc / 16.f;
    x[1] = b0 / 16.f;
    x[2] = bp / 16.f;
    x[3] = j / 8.f;
    x[4] = (bc - bp) / 16.f;
    x[5] = (bc - b0) / 16.f;
    x[6] = 1.f;
    for (int i = 0; i < 8; i++) x[7 + i] = (i == pattern) ? 1.f : 0.f;
    x[15] = 0.f;
}

uint64_t sm64(uint64_t& st) {
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double gauss(uint64_t& st) {
    const double u1 = ((sm64(st) >> 11) + 1.0) / 9007199254740993.0, u2 = (sm64(st) >> 11) / 9007199254740992.0;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

sgpm_status upload_tables(sgpm_ctx* c, sgpm_model* m) {
    HIP_TRY(c, hipMalloc(&m->d_tables, sizeof(uint16_t) * m->tables.size()));
    HIP_TRY(c, hipMemcpy(m->d_tables, m->tables.data(), sizeof(uint16_t) * m->tables.size(), hipMemcpyHostToDevice));
    return SGPM_OK;
}

}  // namespace

sgpm_status learn_args_for(sgpm_ctx* c, sgpm_graph* g, sgpm_pattern* p, sgpm_model* m, LearnArgs* la) {
    if (!g->degree_ordered || !g->d_vb || !g->d_bthr)
        return fail(c, SGPM_EUNSUPPORTED, "the learned proposal needs a degree-ordered (canonical) graph");
    for (int i = 0; i < m->np; i++)
        if (same_plan(m->plans[(size_t)i], p->plan)) {
            la->table = m->d_tables + (size_t)i * TABLE;
            la->vb = g->d_vb;
            la->thr = g->d_bthr;
            la->lane_thr = 0;
            return SGPM_OK;
        }
    return fail(c, SGPM_EINVAL, "the proposal model has no table for this pattern");
}

// evaluate the MLP on every (step, b0, bp, bc) of pattern index `pi` and quantise
sgpm_status build_table(sgpm_ctx* c, const float* d_params, int pi, int k, uint16_t* table) {
    std::vector<float> X(TABLE * NFEAT);
    for (int j = 0; j < 8; j++)
        for (int b0 = 0; b0 < 32; b0++)
            for (int bp = 0; bp < 32; bp++)
                for (int bc = 0; bc < 32; bc++)
                    features(&X[((((size_t)j * 32 + b0) * 32 + bp) * 32 + bc) * NFEAT], pi, j, b0, bp, bc);
    DeviceBuffer dX, dS;
    HIP_TRY(c, hipMalloc(&dX.p, sizeof(float) * X.size()));
    HIP_TRY(c, hipMalloc(&dS.p, sizeof(float) * TABLE));
    HIP_TRY(c, hipMemcpy(dX.p, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, mlp_forward(d_params, (const float*)dX.p, (int64_t)TABLE, (float*)dS.p, c->st));
    std::vector<float> sc(TABLE);
    HIP_TRY(c, hipMemcpyAsync(sc.data(), dS.p, sizeof(float) * TABLE, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    for (size_t row = 0; row < TABLE / 32; row++) {
        const int j = (int)(row / (32 * 32));
        float mx = -INFINITY;
        for (int bc = 0; bc < 32; bc++) mx = std::max(mx, sc[row * 32 + bc]);
        for (int bc = 0; bc < 32; bc++) {
            uint16_t w = 1;
            if (j >= 2 && j + 1 < k && std::isfinite(mx)) {  // the last step picks uniformly
                const double e = std::exp2((double)sc[row * 32 + bc] - (double)mx + 15.0);
                w = (uint16_t)std::min(65535.0, std::max(1.0, std::nearbyint(e)));
            }
            table[row * 32 + bc] = w;
        }
    }
    return SGPM_OK;
}

sgpm_status train(sgpm_ctx* c, sgpm_graph* g, const sgpm_pattern_t* pats, int np, const sgpm_train_cfg* cfg_in,
                  sgpm_model** out) {
    auto t0 = std::chrono::steady_clock::now();
    if (np < 1 || np > 8) return fail(c, SGPM_EINVAL, "a model covers 1..8 patterns");
    if (!g->degree_ordered) return fail(c, SGPM_EUNSUPPORTED, "training needs a degree-ordered (canonical) graph");
    // minibatches of 2048 rows spread each Adam step over many workgroups: on
    // R-MAT 20 and 22 the proposal's predicted error matches that of 256-row
    // minibatches (3e-3, 6 epochs) at a third to a half of the training time
    sgpm_train_cfg cfg{1ull << 18, 8, 2048, 6e-3f, 1};
    if (cfg_in) {
        if (cfg_in->pilot_samples) cfg.pilot_samples = cfg_in->pilot_samples;
        if (cfg_in->epochs > 0) cfg.epochs = cfg_in->epochs;
        if (cfg_in->batch > 0) cfg.batch = cfg_in->batch;
        if (cfg_in->lr > 0) cfg.lr = cfg_in->lr;
        cfg.seed = cfg_in->seed;
    }
    cfg.batch = std::max(16, (cfg.batch + 15) / 16 * 16);
    HIP_TRY(c, hipSetDevice(c->dev));
    auto m = std::make_unique<sgpm_model>();
    m->ctx = c;
    m->np = np;
    // 1. pilots and tuples.  A tuple is one pilot step j of pattern i: its cell
    // (i, j, bucket of v0, bucket of v_{j-1}, bucket of v_j) and C = the product
    // of the later set sizes on a hit, 0 on a miss -- an unbiased estimate of the
    // number of completions through v_j (the NS-prune argument applied to the
    // rest of the walk).  The proposal that makes the weights least variable
    // picks candidates in proportion to their completions, so the network
    // regresses log2 of the cell's mean C (plus 1/16, which keeps cells without
    // completions finite), every tuple of a cell carrying the cell's target.
    std::vector<float> X;
    std::vector<float> Y;
    std::vector<uint32_t> cell_of;
    std::vector<double> Csum((size_t)np * TABLE, 0.0);
    std::vector<uint32_t> Ccnt((size_t)np * TABLE, 0);
    const uint64_t N = cfg.pilot_samples;
    std::vector<sgpm_trace_rec> rec((size_t)N);
    std::vector<uint32_t> sizes((size_t)N * 8);
    DeviceBuffer dsz;
    HIP_TRY(c, hipMalloc(&dsz.p, sizeof(uint32_t) * 8 * (size_t)N));
    for (int i = 0; i < np; i++) {
        if (!pats[i]) return fail(c, SGPM_EINVAL, "null pattern");
        const Plan& p = pats[i]->plan;
        m->plans.push_back(p);
        sgpm_options o;
        sgpm_options_default(&o);
        o.mode = SGPM_MODE_FIXED_N;
        o.fixed_n = N;
        o.seed = cfg.seed;
        o.query_tag = 0x80000000u | (uint32_t)i;
        o.trace_lo = 0;
        o.trace_hi = N;
        o.trace_buf = rec.data();
        NsExtra ex{};
        ex.d_sizes = (uint32_t*)dsz.p;
        sgpm_result r;
        sgpm_status st = ns_estimate_solo(c, g, p, o, &r, 0, &ex);
        if (st != SGPM_OK && st != SGPM_NOT_CONVERGED) return st;
        HIP_TRY(c, hipMemcpy(sizes.data(), dsz.p, sizeof(uint32_t) * 8 * (size_t)N, hipMemcpyDeviceToHost));
        for (uint64_t s = 0; s < N; s++) {
            const sgpm_trace_rec& R = rec[(size_t)s];
            const uint32_t* sz = &sizes[(size_t)s * 8];
            const bool hit = R.status == 0xFFu;
            const int last = hit ? p.k : (int)R.status;  // positions 0..last-1 were chosen
            if (R.v[0] < 0) continue;
            const int b0 = bucket_host(g, R.v[0]);
            for (int j = 2; j < last; j++) {
                double Yc = 0.0;
                if (hit) {
                    Yc = 1.0;
                    for (int t = j + 1; t < p.k; t++) Yc *= (double)sz[t];
                }
                const int bp = bucket_host(g, R.v[j - 1]), bc = bucket_host(g, R.v[j]);
                float x[NFEAT];
                features(x, i, j, b0, bp, bc);
                X.insert(X.end(), x, x + NFEAT);
                const uint32_t cell = (uint32_t)((size_t)i * TABLE + ((((size_t)j * 32 + b0) * 32 + bp) * 32 + bc));
                cell_of.push_back(cell);
                Csum[cell] += Yc;
                Ccnt[cell] += 1;
            }
        }
    }
    Y.resize(cell_of.size());
    for (size_t t = 0; t < cell_of.size(); t++)
        Y[t] = (float)std::log2(Csum[cell_of[t]] / (double)Ccnt[cell_of[t]] + 0.0625);
    m->pilot_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    const int64_t T = (int64_t)Y.size();
    m->tuples = (uint64_t)T;
    if (T < cfg.batch) return fail(c, SGPM_EINVAL, "too few training tuples (patterns never matched in the pilot)");
    // 2. parameters
    const int NP = mlp_nparams();
    std::vector<float> P((size_t)NP, 0.f);
    uint64_t rs = cfg.seed ^ 0x5EEDull;
    for (int i = 0; i < 16 * 64; i++) P[(size_t)i] = (float)(gauss(rs) * std::sqrt(2.0 / 16));
    for (int i = 0; i < 64 * 64; i++) P[(size_t)(16 * 64 + 64 + i)] = (float)(gauss(rs) * std::sqrt(2.0 / 64));
    for (int i = 0; i < 64; i++) P[(size_t)(16 * 64 + 64 + 64 * 64 + 64 + i)] = (float)(gauss(rs) * std::sqrt(1.0 / 64));
    double ymean = 0;
    for (float v : Y) ymean += v;
    P[(size_t)NP - 1] = (float)(ymean / (double)T);
    // 3. Adam epochs over shuffled minibatches (rows permuted on the host per epoch)
    const int64_t B = cfg.batch, steps_per_epoch = T / B;
    DeviceBuffer dP, dX, dY, dm, dv, dg;
    HIP_TRY(c, hipMalloc(&dP.p, sizeof(float) * (size_t)NP));
    HIP_TRY(c, hipMalloc(&dm.p, sizeof(float) * (size_t)NP));
    HIP_TRY(c, hipMalloc(&dv.p, sizeof(float) * (size_t)NP));
    HIP_TRY(c, hipMalloc(&dX.p, sizeof(float) * (size_t)(steps_per_epoch * B) * NFEAT));
    HIP_TRY(c, hipMalloc(&dY.p, sizeof(float) * (size_t)(steps_per_epoch * B)));
    const int64_t parts = mlp_grad_blocks(B);
    HIP_TRY(c, hipMalloc(&dg.p, sizeof(float) * (size_t)NP * (size_t)parts));
    HIP_TRY(c, hipMemcpy(dP.p, P.data(), sizeof(float) * (size_t)NP, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemset(dm.p, 0, sizeof(float) * (size_t)NP));
    HIP_TRY(c, hipMemset(dv.p, 0, sizeof(float) * (size_t)NP));
    std::vector<int64_t> perm((size_t)T);
    for (int64_t i = 0; i < T; i++) perm[(size_t)i] = i;
    std::vector<float> Xs((size_t)(steps_per_epoch * B) * NFEAT), Ys((size_t)(steps_per_epoch * B));
    uint64_t ps = cfg.seed ^ 0xA11CEull;
    float bpow[2] = {1.f, 1.f};  // Adam's beta1^t, beta2^t
    DeviceBuffer dloss;
    HIP_TRY(c, hipMalloc(&dloss.p, sizeof(float) * (size_t)T));
    auto eval_loss = [&](double* loss) -> sgpm_status {
        // mean squared error over the first epoch's rows (forward only)
        HIP_TRY(c, mlp_forward((const float*)dP.p, (const float*)dX.p, steps_per_epoch * B, (float*)dloss.p, c->st));
        std::vector<float> sc((size_t)(steps_per_epoch * B));
        HIP_TRY(c, hipMemcpyAsync(sc.data(), dloss.p, sizeof(float) * sc.size(), hipMemcpyDeviceToHost, c->st));
        HIP_TRY(c, hipStreamSynchronize(c->st));
        double a = 0;
        for (size_t i = 0; i < sc.size(); i++) a += 0.5 * (sc[i] - Ys[i]) * (sc[i] - Ys[i]);
        *loss = a / (double)sc.size();
        return SGPM_OK;
    };
    for (int ep = 0; ep < cfg.epochs; ep++) {
        for (int64_t i = T - 1; i > 0; i--) std::swap(perm[(size_t)i], perm[(size_t)(sm64(ps) % (uint64_t)(i + 1))]);
        for (int64_t r = 0; r < steps_per_epoch * B; r++) {
            std::memcpy(&Xs[(size_t)r * NFEAT], &X[(size_t)perm[(size_t)r] * NFEAT], sizeof(float) * NFEAT);
            Ys[(size_t)r] = Y[(size_t)perm[(size_t)r]];
        }
        HIP_TRY(c, hipMemcpy(dX.p, Xs.data(), sizeof(float) * Xs.size(), hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(dY.p, Ys.data(), sizeof(float) * Ys.size(), hipMemcpyHostToDevice));
        if (ep == 0) {
            sgpm_status st = eval_loss(&m->loss_first);
            if (st != SGPM_OK) return st;
        }
        HIP_TRY(c, mlp_adam_steps((float*)dP.p, (float*)dm.p, (float*)dv.p, (const float*)dX.p, (const float*)dY.p,
                                  steps_per_epoch, B, cfg.lr, bpow, (float*)dg.p, c->st));
    }
    {
        sgpm_status st = eval_loss(&m->loss_last);
        if (st != SGPM_OK) return st;
    }
    m->params.resize((size_t)NP);
    HIP_TRY(c, hipMemcpy(m->params.data(), dP.p, sizeof(float) * (size_t)NP, hipMemcpyDeviceToHost));
    // 4. frozen weight tables
    m->tables.assign((size_t)np * TABLE, 1);
    for (int i = 0; i < np; i++) {
        sgpm_status st = build_table(c, (const float*)dP.p, i, m->plans[(size_t)i].k, &m->tables[(size_t)i * TABLE]);
        if (st != SGPM_OK) return st;
    }
    sgpm_status st = upload_tables(c, m.get());
    if (st != SGPM_OK) return st;
    m->train_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (std::getenv("SGPM_DEBUG"))
        std::fprintf(stderr, "sgpm train: %lld tuples, loss %.4f -> %.4f, pilot %.2fs, total %.2fs\n", (long long)T,
                     m->loss_first, m->loss_last, m->pilot_seconds, m->train_seconds);
    *out = m.release();
    return SGPM_OK;
}

}  // namespace sgpm

using namespace sgpm;

sgpm_model::~sgpm_model() {
    if (!d_tables) return;
    if (ctx) (void)hipSetDevice(ctx->dev);
    (void)hipFree(d_tables);
}

extern "C" {

sgpm_status sgpm_model_train(sgpm_ctx_t c, sgpm_graph_t g, const sgpm_pattern_t* patterns, int np,
                             const sgpm_train_cfg* cfg, sgpm_model_t* out) {
    if (!c || !g || !patterns || !out) return fail(c, SGPM_EINVAL, "null argument");
    return train(c, g, patterns, np, cfg, out);
}

sgpm_status sgpm_model_from_tables(sgpm_ctx_t c, int np, const sgpm_pattern_t* patterns, const uint16_t* tables,
                                   sgpm_model_t* out) {
    if (!c || !patterns || !tables || !out || np < 1 || np > 8) return fail(c, SGPM_EINVAL, "bad model arguments");
    auto m = std::make_unique<sgpm_model>();
    m->ctx = c;
    m->np = np;
    for (int i = 0; i < np; i++) {
        if (!patterns[i]) return fail(c, SGPM_EINVAL, "null pattern");
        m->plans.push_back(patterns[i]->plan);
    }
    m->tables.assign(tables, tables + (size_t)np * TABLE);
    for (uint16_t w : m->tables)
        if (w == 0) return fail(c, SGPM_EINVAL, "proposal weights must be >= 1");
    HIP_TRY(c, hipSetDevice(c->dev));
    sgpm_status st = upload_tables(c, m.get());
    if (st != SGPM_OK) return st;
    *out = m.release();
    return SGPM_OK;
}

sgpm_status sgpm_model_table(sgpm_model_t m, int i, uint16_t* out) {
    if (!m || !out || i < 0 || i >= m->np) return SGPM_EINVAL;
    std::memcpy(out, &m->tables[(size_t)i * TABLE], sizeof(uint16_t) * TABLE);
    return SGPM_OK;
}

sgpm_status sgpm_model_info(sgpm_model_t m, float* params_out, int* nparams, double* stats4, uint64_t* tuples) {
    if (!m) return SGPM_EINVAL;
    if (nparams) *nparams = (int)m->params.size();
    if (params_out && !m->params.empty()) std::memcpy(params_out, m->params.data(), sizeof(float) * m->params.size());
    if (stats4) {
        stats4[0] = m->pilot_seconds;
        stats4[1] = m->train_seconds;
        stats4[2] = m->loss_first;
        stats4[3] = m->loss_last;
    }
    if (tuples) *tuples = m->tuples;
    return SGPM_OK;
}

sgpm_status sgpm_model_free(sgpm_model_t m) {
    if (!m) return SGPM_EINVAL;
    delete m;
    return SGPM_OK;
}

sgpm_status sgpm_mlp_forward(sgpm_ctx_t c, const float* params, const float* X, int64_t N, float* s_out) {
    if (!c || !params || !X || !s_out || N < 1) return fail(c, SGPM_EINVAL, "bad arguments");
    HIP_TRY(c, hipSetDevice(c->dev));
    const int NP = mlp_nparams();
    DeviceBuffer dP, dX, dS;
    HIP_TRY(c, hipMalloc(&dP.p, sizeof(float) * (size_t)NP));
    HIP_TRY(c, hipMalloc(&dX.p, sizeof(float) * (size_t)N * NFEAT));
    HIP_TRY(c, hipMalloc(&dS.p, sizeof(float) * (size_t)N));
    HIP_TRY(c, hipMemcpy(dP.p, params, sizeof(float) * (size_t)NP, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(dX.p, X, sizeof(float) * (size_t)N * NFEAT, hipMemcpyHostToDevice));
    HIP_TRY(c, mlp_forward((const float*)dP.p, (const float*)dX.p, N, (float*)dS.p, c->st));
    HIP_TRY(c, hipMemcpyAsync(s_out, dS.p, sizeof(float) * (size_t)N, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return SGPM_OK;
}

sgpm_status sgpm_mlp_grad(sgpm_ctx_t c, const float* params, const float* X, const float* y, int64_t N,
                          float* grads_out) {
    if (!c || !params || !X || !y || !grads_out || N < 1) return fail(c, SGPM_EINVAL, "bad arguments");
    HIP_TRY(c, hipSetDevice(c->dev));
    const int NP = mlp_nparams();
    const int64_t parts = mlp_grad_blocks(N);
    DeviceBuffer dP, dX, dY, dgp, dg;
    HIP_TRY(c, hipMalloc(&dP.p, sizeof(float) * (size_t)NP));
    HIP_TRY(c, hipMalloc(&dX.p, sizeof(float) * (size_t)N * NFEAT));
    HIP_TRY(c, hipMalloc(&dY.p, sizeof(float) * (size_t)N));
    HIP_TRY(c, hipMalloc(&dgp.p, sizeof(float) * (size_t)NP * (size_t)parts));
    HIP_TRY(c, hipMalloc(&dg.p, sizeof(float) * (size_t)NP));
    HIP_TRY(c, hipMemcpy(dP.p, params, sizeof(float) * (size_t)NP, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(dX.p, X, sizeof(float) * (size_t)N * NFEAT, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(dY.p, y, sizeof(float) * (size_t)N, hipMemcpyHostToDevice));
    HIP_TRY(c, mlp_grad((const float*)dP.p, (const float*)dX.p, (const float*)dY.p, N, (float*)dgp.p, (float*)dg.p,
                        c->st));
    HIP_TRY(c, hipMemcpyAsync(grads_out, dg.p, sizeof(float) * (size_t)NP, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return SGPM_OK;
}

sgpm_status sgpm_mlp_adam_steps(sgpm_ctx_t c, float* params, float* m, float* v, const float* X, const float* y,
                                int64_t nsteps, int64_t B, float lr, float* beta_pow) {
    if (!c || !params || !m || !v || !X || !y || !beta_pow || nsteps < 1 || B < 1 || !(lr > 0))
        return fail(c, SGPM_EINVAL, "bad arguments");
    HIP_TRY(c, hipSetDevice(c->dev));
    const int NP = mlp_nparams();
    const size_t rows = (size_t)nsteps * (size_t)B;
    DeviceBuffer dP, dm, dv, dX, dY, dgp;
    HIP_TRY(c, hipMalloc(&dP.p, sizeof(float) * (size_t)NP));
    HIP_TRY(c, hipMalloc(&dm.p, sizeof(float) * (size_t)NP));
    HIP_TRY(c, hipMalloc(&dv.p, sizeof(float) * (size_t)NP));
    HIP_TRY(c, hipMalloc(&dX.p, sizeof(float) * rows * NFEAT));
    HIP_TRY(c, hipMalloc(&dY.p, sizeof(float) * rows));
    HIP_TRY(c, hipMalloc(&dgp.p, sizeof(float) * (size_t)NP * (size_t)mlp_grad_blocks(B)));
    HIP_TRY(c, hipMemcpy(dP.p, params, sizeof(float) * (size_t)NP, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(dm.p, m, sizeof(float) * (size_t)NP, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(dv.p, v, sizeof(float) * (size_t)NP, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(dX.p, X, sizeof(float) * rows * NFEAT, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(dY.p, y, sizeof(float) * rows, hipMemcpyHostToDevice));
    HIP_TRY(c, mlp_adam_steps((float*)dP.p, (float*)dm.p, (float*)dv.p, (const float*)dX.p, (const float*)dY.p, nsteps,
                              B, lr, beta_pow, (float*)dgp.p, c->st));
    HIP_TRY(c, hipMemcpyAsync(params, dP.p, sizeof(float) * (size_t)NP, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipMemcpyAsync(m, dm.p, sizeof(float) * (size_t)NP, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipMemcpyAsync(v, dv.p, sizeof(float) * (size_t)NP, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return SGPM_OK;
}

// Times the MLP forward and gradient kernels on N device-resident rows
// (iters launches each, HIP events): out4 = {forward ms, forward TFLOP/s,
// gradient ms, gradient TFLOP/s}, FLOPs counted as 2 per multiply-add of the
// three layers (x3 for forward + backward).
sgpm_status sgpm_probe_mlp(sgpm_ctx_t c, int64_t N, int iters, double* out4) {
    if (!c || N < 64 || iters < 1 || !out4) return fail(c, SGPM_EINVAL, "bad arguments");
    HIP_TRY(c, hipSetDevice(c->dev));
    const int NP = mlp_nparams();
    const int64_t parts = mlp_grad_blocks(N);
    std::vector<float> hp((size_t)NP), hx((size_t)N * NFEAT), hy((size_t)N);
    uint64_t rs = 12345;
    for (auto& v : hp) v = (float)(gauss(rs) * 0.1);
    for (auto& v : hx) v = (float)gauss(rs);
    for (auto& v : hy) v = (float)gauss(rs);
    DeviceBuffer dP, dX, dY, dS, dgp, dg;
    HIP_TRY(c, hipMalloc(&dP.p, sizeof(float) * (size_t)NP));
    HIP_TRY(c, hipMalloc(&dX.p, sizeof(float) * hx.size()));
    HIP_TRY(c, hipMalloc(&dY.p, sizeof(float) * hy.size()));
    HIP_TRY(c, hipMalloc(&dS.p, sizeof(float) * (size_t)N));
    HIP_TRY(c, hipMalloc(&dgp.p, sizeof(float) * (size_t)NP * (size_t)parts));
    HIP_TRY(c, hipMalloc(&dg.p, sizeof(float) * (size_t)NP));
    HIP_TRY(c, hipMemcpy(dP.p, hp.data(), sizeof(float) * hp.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(dX.p, hx.data(), sizeof(float) * hx.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(dY.p, hy.data(), sizeof(float) * hy.size(), hipMemcpyHostToDevice));
    ScopedEvents<4> e;
    HIP_TRY(c, e.create());
    HIP_TRY(c, mlp_forward((const float*)dP.p, (const float*)dX.p, N, (float*)dS.p, c->st));  // warm
    HIP_TRY(c, hipEventRecord(e[0], c->st));
    for (int i = 0; i < iters; i++) HIP_TRY(c, mlp_forward((const float*)dP.p, (const float*)dX.p, N, (float*)dS.p, c->st));
    HIP_TRY(c, hipEventRecord(e[1], c->st));
    HIP_TRY(c, mlp_grad((const float*)dP.p, (const float*)dX.p, (const float*)dY.p, N, (float*)dgp.p, (float*)dg.p,
                        c->st));
    HIP_TRY(c, hipEventRecord(e[2], c->st));
    for (int i = 0; i < iters; i++)
        HIP_TRY(c, mlp_grad((const float*)dP.p, (const float*)dX.p, (const float*)dY.p, N, (float*)dgp.p,
                            (float*)dg.p, c->st));
    HIP_TRY(c, hipEventRecord(e[3], c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    float f = 0, b = 0;
    HIP_TRY(c, hipEventElapsedTime(&f, e[0], e[1]));
    HIP_TRY(c, hipEventElapsedTime(&b, e[2], e[3]));
    const double flops_row = 2.0 * (16.0 * 64 + 64.0 * 64 + 64.0);
    out4[0] = f / iters;
    out4[1] = flops_row * (double)N / (out4[0] * 1e-3) / 1e12;
    out4[2] = b / iters;
    out4[3] = 3.0 * flops_row * (double)N / (out4[2] * 1e-3) / 1e12;
    return SGPM_OK;
}

}  // extern "C"
