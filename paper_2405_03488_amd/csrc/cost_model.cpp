// Loose mode with the paper's profiler and cost models (Sec. 4.3, 4.4, 5.1,
// 5.3, 5.4): the alternative to the timed-pilot selector of hybrid.cpp.
//
// NS cost model (Sec. 4.3): time = c W N_s, with the per-sample work W bounded
// by a cone: the lower slope is the work up to the first break point (the
// first set operation, step 2), the upper slope the work of a walk that never
// breaks.  Work counts row entries read by the set operations; a row is taken
// to hold the average degree 2|E|/|V| entries.  The hardware constant c
// (seconds per unit of work) is measured once per graph on a small pilot.
//
// Profiler (Sec. 5.3): the graph is sparsified to 10 % of its edges (Bernoulli
// edge sparsification) and NS-online runs on it to a 50 % error bound at 99 %
// confidence, ending after N_o samples with predicted error eps_o.  The
// samples needed on G follow the error equation: N_s = N_o (eps_o / eps)^2
// (z / z_o)^2 rho(P, G') / rho(P, G), where rho is the probability that an NS
// sample of P is a hit (the per-sample relative variance of a hit-or-miss
// weight scales as 1 / rho); rho(P, G') is the profiler run's hit rate and
// rho(P, G) the pilot's.
//
// GS cost model (Sec. 4.4), for c colours (keep probability p = 1/c):
// preprocessing |E| (w1 + p w2) with w1 one read and w2 one write per edge,
// and the nested-loop search of the sparsified graph: level 1 iterates the
// i_1 = p m first edges (2 p m arcs when the plan does not orient them), level
// j >= 2 computes its candidate set from rows_j rows of the average
// sparsified degree 2 |E| p / |V| (o_j = rows_j 2|E|p/|V| entries per parent)
// and iterates i_j = |V| p1 p2^(c_j - 1) of them, halved when the step has a
// symmetry-breaking bound, with p1 = 2 |E| p / |V|^2 and p2 = 3 T |V| / (2
// |E|^2) (capped at 1; T the triangle count of G, unchanged by sparsification
// since T' = T p^2 and |E'| = |E| p).  Total work = sum_j (prod_{t<j} i_t) o_j.
// Seconds per unit of preprocessing and search work come from one timed
// sparsification and one timed search.  The colourings needed follow the GS
// variance (Sec. 4.4) without its covariance term: relative variance of one
// colouring (c^(k-1) - 1) / C with C the profiler's count estimate, and the GS
// stop rule's Student t interval (at least three colourings).
//
// Selection (Sec. 5.1): the best colour count minimises the predicted GS time;
// GS runs only when that lies entirely below the NS cone, otherwise NS runs with
// windows of 10 % of N_s (Sec. 5.4).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "sgpm_internal.h"

namespace sgpm {

static const int kColourCands[7] = {4, 5, 6, 8, 10, 12, 16};

void cost_model(const Plan& p, const sgpm_cost_in& in, sgpm_cost_out* out) {
    std::memset(out, 0, sizeof(*out));
    const double n = in.n, m = in.m;
    const double dbar = n > 0 ? 2.0 * m / n : 0.0;
    int l = 0;
    for (int j = 1; j < p.k; j++) l += __builtin_popcount((unsigned)p.connect[j]);
    // NS: work per sample, the cone's two slopes
    auto rows = [&](int j) { return (double)__builtin_popcount((unsigned)(p.connect[j] | p.disconnect[j])); };
    double w_hi = 1.0;
    for (int j = 2; j < p.k; j++) w_hi += rows(j) * dbar;
    const double w_lo = p.k > 2 ? 1.0 + rows(2) * dbar : 1.0;
    out->w_lo = w_lo;
    out->w_hi = w_hi;
    // samples needed (profiler); infinite without hits on either graph
    double ns = INFINITY;
    if (in.prof_samples > 0 && std::isfinite(in.prof_eps_hat) && in.rho_g > 0 && in.rho_sparse > 0 && in.z > 0 &&
        in.prof_z > 0) {
        const double r = in.prof_eps_hat / in.eps, q = in.z / in.prof_z;
        ns = in.prof_samples * r * r * q * q * (in.rho_sparse / in.rho_g);
    }
    if (p.k <= 2) ns = 1.0;  // an edge pattern: every sample is exact
    out->ns_samples = ns;
    // seconds per unit of NS work from the pilot (geometric mean of the slopes)
    const double c_ns = in.pilot_samples > 0 ? in.pilot_seconds / (in.pilot_samples * std::sqrt(w_lo * w_hi)) : 0.0;
    out->ns_lo = std::isfinite(ns) ? c_ns * w_lo * ns : INFINITY;
    out->ns_hi = std::isfinite(ns) ? c_ns * w_hi * ns : INFINITY;
    // GS search work on the graph colour-sparsified with keep probability pk
    const double p2 = m > 0 ? std::min(1.0, 3.0 * in.triangles * n / (2.0 * m * m)) : 0.0;
    auto search_work = [&](double pk) {
        const double p1 = n > 0 ? 2.0 * m * pk / (n * n) : 0.0, dk = dbar * pk;
        double reach = (p.oriented ? 1.0 : 2.0) * pk * m;  // tuples at the current level
        double work = 0.0;
        for (int j = 2; j < p.k; j++) {
            work += reach * rows(j) * dk;
            const int cj = __builtin_popcount((unsigned)p.connect[j]);
            double ij = n * p1 * std::pow(p2, (double)(cj - 1));
            if (p.upper[j] || p.lower[j]) ij *= 0.5;
            reach *= ij;
        }
        return work;
    };
    const double c_pre = m > 0 ? in.sparsify_seconds / (m * (1.0 + in.sparsify_keep)) : 0.0;
    const double ws_probe = search_work(1.0 / in.probe_colours);
    const double c_s = ws_probe > 0 ? in.probe_search_seconds / ws_probe : 0.0;
    out->gs_best = INFINITY;
    out->gs_colours = 0;
    for (int i = 0; i < 7; i++) {
        const double c = kColourCands[i], pk = 1.0 / c;
        const double t_pre = c_pre * m * (1.0 + pk);
        const double t_search = c_s * search_work(pk);
        const double cv = in.count > 0 ? std::sqrt((std::pow(c, (double)(p.k - 1)) - 1.0) / in.count) : INFINITY;
        const int reps = in.count > 0 ? gs_reps_needed(cv, in.eps, in.confidence, in.gs_reps_max > 0 ? in.gs_reps_max : 64)
                                      : (int)kGsMinReps;
        const double t = reps > 0 ? reps * (t_pre + t_search) : INFINITY;
        out->gs_seconds[i] = t;
        out->gs_reps[i] = reps;
        if (t < out->gs_best) {
            out->gs_best = t;
            out->gs_colours = (int)c;
        }
    }
    // GS only when entirely below the NS cone (above or overlapping: NS)
    out->choice = (std::isfinite(out->gs_best) && out->gs_best < out->ns_lo) ? SGPM_SCHEME_GS : SGPM_SCHEME_NS;
    (void)l;
}

namespace {

constexpr uint32_t kProfilerTag = 0xA0000000u;
constexpr uint32_t kProfilerRep = 0x0FFFFFFFu;
constexpr uint32_t kProbeRep = 0x3FFFFFFFu;

}  // namespace

sgpm_status model_hybrid_estimate(sgpm_ctx* c, sgpm_graph* g, sgpm_pattern* pat, const sgpm_options& o,
                                  sgpm_result* res) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    const Plan& p = pat->plan;
    const uint64_t M = p.oriented ? (uint64_t)g->m : 2ull * (uint64_t)g->m;
    if (M == 0 || p.k <= 2) {
        sgpm_options no = o;
        no.mode = SGPM_MODE_STRICT_NS;
        return ns_estimate_solo(c, g, p, no, res, 0);
    }
    sgpm_cost_in in{};
    in.n = (double)g->n;
    in.m = (double)g->m;
    in.eps = o.eps;
    in.confidence = o.confidence;
    in.z = normal_quantile(1.0 - (1.0 - o.confidence) / 2.0);
    in.gs_reps_max = o.gs_reps_max;
    auto base = [&]() {
        sgpm_options q;
        sgpm_options_default(&q);
        q.seed = o.seed;
        q.lanes_per_sample = 64;
        return q;
    };
    sgpm_result r;
    // triangle count of G (the GS set-size model's p2): a 5 % NS estimate
    {
        Plan tri;
        std::string err;
        const int32_t e3[6] = {0, 1, 1, 2, 0, 2};
        if (compile_pattern(3, 3, e3, 0, tri, err) != SGPM_OK) return fail(c, SGPM_EINVAL, err);
        sgpm_options q = base();
        q.eps = 0.05;
        q.n_min = q.w_min = 1u << 16;
        q.quantum = 1u << 12;
        q.max_samples = 1ull << 24;
        q.query_tag = kProfilerTag | 1u;
        sgpm_status st = ns_estimate_solo(c, g, tri, q, &r, 0);
        if (st != SGPM_OK && st != SGPM_NOT_CONVERGED) return st;
        in.triangles = r.estimate;
    }
    // pilot on G: hit rate and the seconds per unit of NS work
    {
        sgpm_options q = base();
        q.mode = SGPM_MODE_FIXED_N;
        q.fixed_n = 1u << 16;
        q.query_tag = kProfilerTag | 2u;
        sgpm_status st = ns_estimate_solo(c, g, p, q, &r, 0);
        if (st != SGPM_OK && st != SGPM_NOT_CONVERGED) return st;
        in.pilot_samples = (double)r.n_samples;
        in.pilot_seconds = r.seconds_kernel;
        in.rho_g = (double)r.n_hits / (double)r.n_samples;
    }
    // profiler: 10 % of the edges, NS-online to 50 % at 99 %
    {
        const auto ta = clk::now();
        sgpm_graph* sp = nullptr;
        sgpm_status st = sparsify(c, g, 10, o.seed, kProfilerRep, &sp, true);
        if (st != SGPM_OK) return st;
        HIP_TRY(c, hipStreamSynchronize(c->st));
        in.sparsify_seconds = std::chrono::duration<double>(clk::now() - ta).count();
        in.sparsify_keep = 0.1;
        int l = 0;
        for (int j = 1; j < p.k; j++) l += __builtin_popcount((unsigned)p.connect[j]);
        sgpm_options q = base();
        q.eps = 0.5;
        q.confidence = 0.99;
        q.n_min = q.w_min = 1u << 14;
        q.quantum = 1u << 10;
        q.max_samples = 1ull << 26;
        q.query_tag = kProfilerTag | 3u;
        st = sp->m > 0 ? ns_estimate_solo(c, sp, p, q, &r, 0) : SGPM_OK;
        const bool ran = sp->m > 0;
        sgpm_graph_free(sp);
        if (st != SGPM_OK && st != SGPM_NOT_CONVERGED) return st;
        if (ran) {
            in.prof_samples = (double)r.n_samples;
            in.prof_eps_hat = r.eps_hat;
            in.prof_z = r.z;
            in.rho_sparse = r.n_samples ? (double)r.n_hits / (double)r.n_samples : 0.0;
            in.count = r.estimate * std::pow(10.0, (double)l);  // Bernoulli scaling c^l with c = 10
        }
    }
    // one timed search at 16 colours (the seconds per unit of search work)
    {
        sgpm_graph* sp = nullptr;
        sgpm_status st = sparsify(c, g, 16, o.seed, kProbeRep, &sp);
        if (st != SGPM_OK) return st;
        unsigned __int128 y = 0;
        double secs = 0.0;
        st = exact_count(c, sp, p, &y, &secs);
        sgpm_graph_free(sp);
        if (st != SGPM_OK) return st;
        in.probe_colours = 16.0;
        in.probe_search_seconds = secs;
    }
    sgpm_cost_out mo;
    cost_model(p, in, &mo);
    const double profile_s = std::chrono::duration<double>(clk::now() - t0).count();
    sgpm_status st;
    if (mo.choice == SGPM_SCHEME_GS) {
        sgpm_options go = o;
        go.mode = SGPM_MODE_GS;
        if (go.colours <= 0) go.colours = mo.gs_colours;
        st = gs_estimate(c, g, p, go, res);
    } else {
        // windows of 10 % of the predicted samples (Sec. 5.4)
        sgpm_options no = o;
        no.mode = SGPM_MODE_STRICT_NS;
        if (std::isfinite(mo.ns_samples)) {
            const uint64_t q = o.quantum ? o.quantum : 1;
            const uint64_t w = std::max<uint64_t>(q, (uint64_t)std::ceil(0.1 * mo.ns_samples / (double)q) * q);
            no.n_min = no.w_min = w;
            no.window_growth = 0.0;
        }
        st = ns_estimate_solo(c, g, p, no, res, 0);
    }
    res->pred_ns_lo = mo.ns_lo;
    res->pred_ns_hi = mo.ns_hi;
    res->pred_gs = mo.gs_best;
    res->pred_samples = mo.ns_samples;
    res->seconds_pilot = profile_s;
    res->seconds_total += profile_s;
    return st;
}

}  // namespace sgpm

using namespace sgpm;

extern "C" int sgpm_host_cost_model(int k, int l, const int32_t* edges, int induced, const sgpm_cost_in* in,
                                    sgpm_cost_out* out) {
    if (!in || !out) return SGPM_EINVAL;
    Plan p;
    std::string err;
    const int rc = compile_pattern(k, l, edges, induced, p, err);
    if (rc != SGPM_OK) return rc;
    cost_model(p, *in, out);
    return SGPM_OK;
}
