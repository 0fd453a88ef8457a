// Loose mode: choose the NS or the GS engine from short pilots (Sec. 5.1).
//
// The paper predicts NS time as work per sample times the number of samples
// (NS cost model, Sec. 4.3), bounded by a cone whose slopes are the cheapest
// (first step fails) and the dearest (no step fails) sample, and predicts GS
// time from a cost model of sparsification plus the nested-loop search
// (Sec. 4.4).  GS is chosen only when its prediction lies entirely below the
// NS cone; above it, or overlapping it, NS runs, since only NS carries the
// confidence guarantee.  Its profiler and GS cost formulas are not usable as
// printed, so both predictions here come from measurements on this device:
//
//  * NS: a pilot of the estimation stream itself (tag q): its first window,
//    in two slices (the first quarter and the rest), one launch each.  Their
//    kernel times fit t0 + n / rate (the launch's fixed cost and the steady
//    rate).  By the error equation (Sec. 4.1) the samples needed for eps scale
//    as (eps_hat / eps)^2, so slice i predicts N_i = n_i (eps_hat_i / eps)^2
//    samples taking N_i / rate plus t0 per window of the schedule up to N_i;
//    the slices' minimum and maximum are the cone.  When NS runs, the pilot is
//    its first window (its stop test is the first one the estimate applies).
//  * GS: colourings 0 and 1 of the GS engine itself (timed end to end:
//    sparsification and count).  Their relative spread (the unbiased standard
//    deviation of one colouring's estimate over their mean, cv) gives the
//    colourings needed under the GS stop rule: the smallest R >= 3 with
//    t_{R-1} cv / sqrt(R) <= eps (t the two-sided Student t quantile), and the
//    prediction is R times the mean colouring time.  When one colouring already takes a third
//    of the cone's lower end GS cannot lie below it and the second is skipped.  Before
//    any colouring, the NS pilot's estimate C bounds GS from below: one
//    colouring's search reaches about C / c^(k-1) leaves, and three colourings
//    (each its sparsification at the modelled device rate the colour choice
//    uses, plus its leaves at an optimistic rate) taking at least the cone's
//    lower end rule GS out without running it (a large graph's exact count can
//    take minutes; a small one's colouring is mostly its sparsification; the
//    per-edge closed forms (wedge, 3-star, 4-path, tailed triangle, diamond)
//    and the 4- to 6-clique's bitmaps count many leaves per instruction, up
//    to 2e12 leaves/s and more, so they are charged their pass over
//    the about m / c kept edges at 2e9 edges/s instead, above the 0.8e9 to
//    1.4e9 measured).  The rate is
//    1e11 leaves per second when the sparsified graph is sparse (mean degree
//    2m / (n c) below 16; the general search measures 2e9 to 3e10 there) and
//    1e12 otherwise (long rows: 4e10 measured for the general search's
//    4-clique on the whole R-MAT 20 graph).
//
// The engine then runs exactly as in its own mode with the same options (NS
// continues the pilot's stream, GS reuses the two pilot colourings, which are
// its first two), so a hybrid result equals the strict-NS or GS result bit for
// bit.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "sgpm_internal.h"

namespace sgpm {

// colourings the GS stop rule needs when one colouring's estimate has relative
// standard deviation cv: the smallest R in [3, cap] with t_{R-1} cv / sqrt(R)
// <= eps, or 0 when none is
int gs_reps_needed(double cv, double eps, double confidence, int cap) {
    if (!std::isfinite(cv) || !(eps > 0)) return 0;
    for (int R = (int)kGsMinReps; R <= cap; R++)
        if (student_t_quantile(confidence, R - 1) * cv / std::sqrt((double)R) <= eps) return R;
    return 0;
}

void ns_cone(int slices, const double* slice_n, const double* seconds, const double* eps_hat, const sgpm_options& o,
             double* lo, double* hi, double* t0_out, double* rate_out) {
    // least-squares fit of t = t0 + n / rate; a fit without a positive rate or
    // with a negative fixed cost falls back to the plain rate of all slices
    double sn = 0, st = 0, snn = 0, snt = 0;
    for (int i = 0; i < slices; i++) {
        sn += slice_n[i];
        st += seconds[i];
        snn += slice_n[i] * slice_n[i];
        snt += slice_n[i] * seconds[i];
    }
    const double den = slices * snn - sn * sn;
    double slope = den > 0 ? (slices * snt - sn * st) / den : 0.0;
    double t0 = slices > 0 ? (st - slope * sn) / slices : 0.0;
    if (!(slope > 0) || !(t0 >= 0)) {
        t0 = 0.0;
        slope = sn > 0 ? st / sn : 0.0;
    }
    double l = INFINITY, h = 0.0;
    for (int i = 0; i < slices; i++) {
        const double r = eps_hat[i] / o.eps;
        double t = INFINITY;
        if (std::isfinite(r)) {
            const double need = slice_n[i] * r * r;
            // windows of the schedule up to `need` samples (at least one)
            int w = 0;
            uint64_t e = 0;
            while (w < 100000) {
                const uint64_t nx = next_window_end(e, o);
                w++;
                if ((double)nx >= need || nx <= e) break;
                e = nx;
            }
            t = need * slope + t0 * w;
        }
        l = std::min(l, t);
        h = std::max(h, t);
    }
    if (slices == 0) l = h = INFINITY;
    *lo = l;
    *hi = h;
    if (t0_out) *t0_out = t0;
    if (rate_out) *rate_out = slope > 0 ? 1.0 / slope : 0.0;
}

int hybrid_choice(double ns_lo, double eps, double confidence, int gs_reps_run, double gs_rep_seconds, double gs_cv,
                  int gs_reps_max, double* gs_pred) {
    double gs = INFINITY;
    if (gs_reps_run >= 2) {
        const int need = gs_reps_needed(gs_cv, eps, confidence, gs_reps_max > 0 ? gs_reps_max : 64);
        if (need > 0) gs = need * gs_rep_seconds;
    } else if (gs_reps_run == 1) {
        gs = (double)kGsMinReps * gs_rep_seconds;  // a lower bound: the stop rule starts at three colourings
    }
    if (gs_pred) *gs_pred = gs;
    // GS entirely below the cone; a one-colouring bound never selects GS
    return (gs_reps_run >= 2 && gs < ns_lo) ? SGPM_SCHEME_GS : SGPM_SCHEME_NS;
}

namespace {

// relative standard deviation of one colouring's estimate c^(k-1) y_r from the
// pilot colourings (unbiased variance over the squared mean); +inf when their
// values are all zero or c^(k-1) y_r leaves 128 bits (then GS is not usable)
double gs_pilot_cv(const GsPrefix& pre, const Plan& p, uint32_t col) {
    unsigned __int128 scale = 1;
    for (int i = 0; i < p.k - 1; i++) {
        if (scale > ~(unsigned __int128)0 / col) return INFINITY;
        scale *= col;
    }
    Big S1(24), S2(24);
    for (int r = 0; r < pre.n; r++) {
        const unsigned __int128 x = pre.y[r] * scale;
        if (x / scale != pre.y[r]) return INFINITY;
        unsigned long long d1[4], d2[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int i = 0; i < 4; i++) d1[i] = (unsigned long long)(uint32_t)(x >> (32 * i));
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) {
                const unsigned long long pr = d1[a] * d1[b];
                d2[a + b] += pr & 0xFFFFFFFFull;
                if (a + b + 1 < 8) d2[a + b + 1] += pr >> 32;
            }
        big_add_digits(S1, d1, 4);
        big_add_digits(S2, d2, 8);
    }
    return std::sqrt((double)pre.n) * predicted_error_t(1.0, (uint64_t)pre.n, S1, S2);
}

}  // namespace

sgpm_status hybrid_estimate(sgpm_ctx* c, sgpm_graph* g, sgpm_pattern* pat, const sgpm_options& o, sgpm_result* res) {
    if (o.hybrid_selector == SGPM_HYBRID_COST_MODEL) {
        if (o.proposal) return fail(c, SGPM_EUNSUPPORTED, "the cost-model selector runs the uniform proposal");
        if (o.colours < 0 || o.colours > 256) return fail(c, SGPM_EINVAL, "colours must be 0 (choose) or in [1, 256]");
        return model_hybrid_estimate(c, g, pat, o, res);
    }
    if (o.hybrid_selector != SGPM_HYBRID_PILOTS) return fail(c, SGPM_EINVAL, "hybrid_selector");
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    const Plan& p = pat->plan;
    NsExtra ex{};
    if (o.proposal) {
        sgpm_status st = learn_args_for(c, g, pat, o.proposal, &ex.la);
        if (st != SGPM_OK) return st;
    }
    const uint64_t M = p.oriented ? (uint64_t)g->m : 2ull * (uint64_t)g->m;
    double ns_lo = INFINITY, ns_hi = INFINITY, gs_pred = INFINITY;
    int scheme = SGPM_SCHEME_NS;
    GsPrefix pre;
    uint32_t col = 0;
    {
        sgpm_status st = gs_resolve_colours(c, g, p, o, &col);
        if (st != SGPM_OK) return st;
    }
    if (M > 0) {
        // NS pilot: the estimation stream's first window, in two slices (its
        // first quarter and the rest); when NS is chosen the window is done
        sgpm_options po = o;
        po.checksum = o.checksum;
        po.trace_lo = po.trace_hi = 0;
        po.trace_buf = nullptr;
        const uint64_t first = next_window_end(0, o);
        const int slices = first >= 8 ? 2 : 1;
        const uint64_t ends[2] = {slices == 2 ? first / 4 : first, first};
        double sn[2], sec[2], eh[2], mu = 0.0;
        for (int i = 0; i < slices; i++) sn[i] = (double)(ends[i] - (i ? ends[i - 1] : 0));
        sgpm_status st = ns_pilot(c, g, p, po, ex.la, slices, ends, sec, eh, &mu, ex.prefix_sums);
        if (st != SGPM_OK) return st;
        ex.prefix_n = first;
        ex.prefix_launches = slices;
        for (int i = 0; i < slices; i++) ex.prefix_kernel_s += sec[i];
        ns_cone(slices, sn, sec, eh, o, &ns_lo, &ns_hi, nullptr, nullptr);
        // lower bound of the three colourings the GS stop rule needs at least
        double leaves = mu;
        for (int i = 0; i < p.k - 1; i++) leaves /= (double)col;
        const double sparse_deg = g->n > 0 ? 2.0 * (double)g->m / ((double)g->n * (double)col) : 0.0;
        // (the per-edge closed forms and the cliques' bitmaps count many leaves
        // per instruction: their search is charged its pass over the kept
        // edges, about m / c, at 2e9 edges per second instead)
        const double search = count_not_by_leaves(p) ? (double)g->m / (double)col / 2e9
                                                     : leaves / (sparse_deg < 16.0 ? 1e11 : 1e12);
        const double gs_floor = (double)kGsMinReps * (gs_sparsify_model_s(g->m) + search);
        // GS pilot: the GS engine's first colourings, timed end to end
        double rep_seconds = 0.0;
        for (int r = 0; r < 2 && gs_floor < ns_lo; r++) {
            const auto a = clk::now();
            double dev = 0.0;
            st = gs_rep(c, g, p, col, o.seed, (uint32_t)r, &pre.y[r], &dev);
            if (st != SGPM_OK) return st;
            pre.dev_seconds += dev;
            pre.n = r + 1;
            rep_seconds += std::chrono::duration<double>(clk::now() - a).count();
            if (r == 0 && (double)kGsMinReps * rep_seconds >= ns_lo) break;  // GS cannot lie below the cone
        }
        if (pre.n == 0) {
            gs_pred = gs_floor;  // a lower bound; GS was not run
        } else {
            rep_seconds /= pre.n;
            const double cv = pre.n >= 2 ? gs_pilot_cv(pre, p, col) : INFINITY;
            scheme = hybrid_choice(ns_lo, o.eps, o.confidence, pre.n, rep_seconds, cv, o.gs_reps_max, &gs_pred);
        }
    }
    const double pilot = std::chrono::duration<double>(clk::now() - t0).count();
    sgpm_status st;
    if (scheme == SGPM_SCHEME_GS) {
        sgpm_options go = o;
        go.colours = (int32_t)col;
        st = gs_estimate(c, g, p, go, res, &pre);
    } else {
        sgpm_options no = o;
        no.mode = SGPM_MODE_STRICT_NS;
        st = ns_estimate_solo(c, g, p, no, res, 0, &ex);
    }
    res->pred_ns_lo = ns_lo;
    res->pred_ns_hi = ns_hi;
    res->pred_gs = gs_pred;
    res->seconds_pilot = pilot;
    res->seconds_total += pilot;
    return st;
}

}  // namespace sgpm
