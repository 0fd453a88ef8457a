// GS engine host side: colour or Bernoulli edge sparsification into a new
// graph handle, the exact count, and the GS estimate over repetitions.
//
// Sec. 5.2: the estimate from one colouring with c colours is c^(k-1) * Y for a
// connected k-vertex pattern (all k vertices must share a colour), Y the exact
// count on the sparsified graph.  The paper gives GS no online confidence
// test; here independent colourings (rep = 0, 1, ...) are i.i.d. unbiased
// estimates X_r = c^(k-1) Y_r whose exact sums give the mean and a Student t
// interval: with few colourings the normal quantile and the 1/n variance of
// the NS rule would give far too narrow an interval, so the predicted error is
// t_{n-1} sqrt(D / (n - 1)) / S1 (unbiased variance, t quantile of n - 1
// degrees of freedom).  Stop at the first n >= 3 with that at most eps (two
// colourings of a small or skewed count often agree exactly, which would give
// an interval of width zero), capped at gs_reps_max colourings.
#include <cstdlib>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>

#include "sgpm_internal.h"

namespace sgpm {


// Slot i of the context's GS scratch, at least `bytes` long (grown by a
// quarter when it must grow, so colourings of slightly different sizes reuse it).
sgpm_status gs_scratch(sgpm_ctx* c, size_t i, size_t bytes, void** out) {
    if (c->gs_scratch.size() <= i) c->gs_scratch.resize(i + 1, {nullptr, 0});
    auto& b = c->gs_scratch[i];
    if (b.second < bytes) {
        if (b.first) HIP_TRY(c, hipFree(b.first));
        b = {nullptr, 0};
        const size_t want = bytes + bytes / 4;
        HIP_TRY(c, hipMalloc(&b.first, want));
        b.second = want;
    }
    *out = b.first;
    return SGPM_OK;
}

enum GsSlot : size_t {
    GS_COL, GS_RSTART, GS_RLOW, GS_TK, GS_TL, GS_TKO, GS_TLO, GS_SCAN, GS_EOFF, GS_PART, GS_CELL, GS_OVF,
    GS_SP_OFF, GS_SP_NBR, GS_SP_AROW, GS_SP_EPAIR  // a sparsified graph that lives only for one colouring
};

#define GS_SCRATCH(ctx, slot, bytes, ptr)                                        \
    do {                                                                         \
        void* _p = nullptr;                                                      \
        sgpm_status _s = gs_scratch((ctx), (slot), (bytes), &_p);               \
        if (_s != SGPM_OK) return _s;                                            \
        (ptr) = decltype(ptr)(_p);                                               \
    } while (0)

// colours: c of colour sparsification, or (bes) the inverse keep probability
sgpm_status sparsify(sgpm_ctx* c, sgpm_graph* g, uint32_t colours, uint64_t seed, uint32_t rep, sgpm_graph** out,
                     bool bes, bool scratch_graph) {
    if (colours < 1 || colours > 256) return fail(c, SGPM_EINVAL, "colours must be in [1, 256]");
    HIP_TRY(c, hipSetDevice(c->dev));
    const int64_t n = g->n;
    const int64_t nt = arc_tiles(2 * g->m);
    // temporaries from the context's scratch (no allocation once it has grown)
    const size_t nv = (size_t)std::max<int64_t>(n, 1), ntw = sizeof(int64_t) * (size_t)(nt + 1);
    uint8_t* col = nullptr;
    int64_t *rstart = nullptr, *rlow = nullptr, *tk = nullptr, *tl = nullptr, *tko = nullptr, *tlo = nullptr;
    int64_t *scan = nullptr, *d_eoff = nullptr;
    GS_SCRATCH(c, GS_COL, nv, col);
    GS_SCRATCH(c, GS_RSTART, sizeof(int64_t) * nv, rstart);
    GS_SCRATCH(c, GS_RLOW, sizeof(int64_t) * nv, rlow);
    GS_SCRATCH(c, GS_TK, ntw, tk);
    GS_SCRATCH(c, GS_TL, ntw, tl);
    GS_SCRATCH(c, GS_TKO, ntw, tko);
    GS_SCRATCH(c, GS_TLO, ntw, tlo);
    GS_SCRATCH(c, GS_SCAN, sizeof(int64_t) * (size_t)scan_scratch_words(nt), scan);
    GS_SCRATCH(c, GS_EOFF, sizeof(int64_t) * (size_t)(n + 1), d_eoff);
    auto h = std::make_unique<sgpm_graph>();
    h->ctx = c;
    h->n = n;
    if (!scratch_graph) h->perm = g->perm;  // ids map back only for graphs handed to the caller
    h->borrowed = scratch_graph;
    if (scratch_graph)
        GS_SCRATCH(c, GS_SP_OFF, sizeof(int64_t) * (size_t)(n + 1), h->d_off);
    else
        HIP_TRY(c, hipMalloc(&h->d_off, sizeof(int64_t) * (size_t)(n + 1)));
    const DGraph dg = g->view();
    const uint8_t* colp = bes ? nullptr : col;
    if (!bes) HIP_TRY(c, gs_colours(n, colours, seed, rep, col, c->st));
    // arcs surviving per tile, their exclusive scans, then the totals
    int64_t arcs = 0, edges = 0;
    if (nt > 0) {
        HIP_TRY(c, gs_arc_counts(dg, colp, colours, seed, rep, tk, tl, c->st));
        HIP_TRY(c, exclusive_scan_pair(tk, tl, nt, tko, tlo, scan, c->st));
        HIP_TRY(c, hipMemcpyAsync(&arcs, tko + nt, sizeof(int64_t), hipMemcpyDeviceToHost, c->st));
        HIP_TRY(c, hipMemcpyAsync(&edges, tlo + nt, sizeof(int64_t), hipMemcpyDeviceToHost, c->st));
        HIP_TRY(c, hipStreamSynchronize(c->st));
    } else {
        HIP_TRY(c, launch_fill_u64((unsigned long long*)tko, 1, 0ull, c->st));
        HIP_TRY(c, launch_fill_u64((unsigned long long*)tlo, 1, 0ull, c->st));
    }
    if (arcs != 2 * edges) return fail(c, SGPM_EHIP, "internal: sparsified graph is not symmetric");
    h->m = edges;
    const size_t arc_bytes = sizeof(int32_t) * (size_t)std::max<int64_t>(arcs, 1);
    const size_t edge_bytes = sizeof(int2) * (size_t)std::max<int64_t>(edges, 1);
    if (scratch_graph) {
        GS_SCRATCH(c, GS_SP_NBR, arc_bytes, h->d_nbr);
        GS_SCRATCH(c, GS_SP_AROW, arc_bytes, h->d_arow);
        GS_SCRATCH(c, GS_SP_EPAIR, edge_bytes, h->d_epair);
    } else {
        HIP_TRY(c, hipMalloc(&h->d_nbr, arc_bytes));
        HIP_TRY(c, hipMalloc(&h->d_arow, arc_bytes));
        HIP_TRY(c, hipMalloc(&h->d_epair, edge_bytes));
    }
    HIP_TRY(c, gs_arc_write(dg, colp, colours, seed, rep, tko, tlo, h->d_nbr, h->d_arow,
                            h->d_epair, rstart, rlow, h->d_off, d_eoff, c->st));
    if (scratch_graph) {  // not measured: an arc survives with about 1/c, so about the max degree / c
        h->maxdeg = g->maxdeg / (int64_t)colours;
        *out = h.release();
        return SGPM_OK;
    }
    unsigned long long* d_md = (unsigned long long*)rstart;  // reuse as the max-degree cell
    HIP_TRY(c, launch_fill_u64(d_md, 1, 0ull, c->st));
    HIP_TRY(c, max_degree(h->d_off, n, d_md, c->st));
    unsigned long long md = 0;
    HIP_TRY(c, hipMemcpyAsync(&md, d_md, sizeof(md), hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    h->maxdeg = (int64_t)md;
    *out = h.release();
    return SGPM_OK;
}

// Lanes per first edge of the exact count.  Narrow groups keep 64 / G first
// edges in flight per wave, which pays where every row the search reads is
// short; the whole wave pays where deeper levels scan long rows.  In the clique
// search every candidate row is a degree-ordered out-row, so on a sparse graph
// (mean degree below 16, as after colour sparsification) a triangle takes 8
// lanes and a 4-clique 16.  A 3-vertex pattern's search is one counted level
// per first edge, so the wedge is narrow too (16 lanes: 1.8 against 3.1 ms at
// c = 16).  Every other case, and any graph of mean degree 16 or more, takes
// the whole wave.  R-MAT 20 sparsified with c = 16, ms at 8 / 16 / 64
// lanes: triangle 0.51 / 0.86 / 3.07, 4-clique 1.65 / 1.25 / 3.20, 5-clique
// 17.0 / 8.0 / 6.7, diamond 384 / 182 / 25, 4-cycle 40 / 42 / 56.
// SGPM_EXACT_GROUP = 8, 16 or 64 fixes the width (tuning, and tests that run
// every width on one graph).
int exact_group(const sgpm_graph* g, const Plan& p) {
    if (const char* e = std::getenv("SGPM_EXACT_GROUP")) {
        const int v = std::atoi(e);
        if (v == 8 || v == 16 || v == 64) return v;
    }
    if (2.0 * (double)g->m >= 16.0 * (double)g->n) return 64;
    // hub rows (max degree 8,192 or more) take the next width up: triangle /
    // wedge ms at 8, 16, 64 lanes, R-MAT 20 at c = 4 (max degree 16K): 1.50 /
    // 8.29, 1.40 / 7.08, 2.90 / 6.51; R-MAT 24 at c = 4 (102K): 54.6 / 486,
    // 44.9 / 377, 41.1 / 275; R-MAT 20 at c = 16 (4K): 0.49 / 1.56, 0.82 /
    // 1.15, 2.88 / 2.89
    const bool hubs = g->maxdeg >= 8192;
    if (p.k == 3) return plan_is_clique(p) ? (hubs ? 16 : 8) : (hubs ? 64 : 16);  // one counted level per first edge
    return plan_is_clique(p) && p.k == 4 ? 16 : 64;
}

// exact count of the plan's tuples on g (the leaves of the pruned search tree).
// The 4-, 5- and 6-clique on oriented first edges take the bitmap count (one
// wave per first edge; first edges whose candidate set exceeds 64, then 128,
// go on through lists), unless SGPM_EXACT_GROUP fixes the general search's
// width or a list could outgrow its buffer.  Four 4-vertex patterns and the
// wedge have closed forms over edges (edge_shape), counted by one pass of
// per-edge terms, under the same SGPM_EXACT_GROUP exception.  The rest take
// the general search.  The buffers come from the caller: block partials (two
// words per slot, part_blocks slots), kCountCells counter and sum words
// (cleared here), and the list of ovf_cap first-edge ids.

// The patterns counted from per-edge terms (t the edge's common neighbours,
// du and dw its endpoints' degrees, K4 the 4-cliques), by identities the
// oracle's counts are pinned against:
//   wedge          sum (du + dw - 2) / 2;  vertex-induced: sum (du + dw - 2 - 2t) / 2
//   3-star         sum (C(du - 1, 2) + C(dw - 1, 2)) / 3;  induced: that - tt + 2 dia - 4 K4
//   4-path         sum ((du - 1)(dw - 1) - t);  (induced: needs the 4-cycles, not here)
//   tailed triangle tt = sum t (du + dw - 4) / 2;  induced: tt - 4 dia + 12 K4
//   diamond        dia = sum C(t, 2);  induced: dia - 6 K4
// With the 4-cycles C4 from the general search, also
//   induced 4-path   sum ((du - 1)(dw - 1) - t) - 2 tt - 4 C4 + 6 dia - 12 K4
//   induced 4-cycle  C4 - dia + 3 K4
int edge_shape(const Plan& p) {
    if (p.k != 3 && p.k != 4) return SHAPE_NONE;
    int deg[4] = {0, 0, 0, 0}, edges = 0;
    for (int j = 1; j < p.k; j++)
        for (int i = 0; i < j; i++)
            if (p.connect[j] >> i & 1) {
                deg[i]++;
                deg[j]++;
                edges++;
            }
    std::sort(deg, deg + p.k);
    if (p.k == 3) return edges == 2 ? SHAPE_WEDGE : SHAPE_NONE;
    if (edges == 3 && deg[3] == 3) return SHAPE_STAR3;
    if (edges == 3 && deg[3] == 2) return p.induced ? SHAPE_IPATH4 : SHAPE_PATH4;
    if (edges == 4 && deg[3] == 3) return SHAPE_TAILED;
    if (edges == 4 && deg[3] == 2) return p.induced ? SHAPE_ICYCLE4 : SHAPE_NONE;
    if (edges == 5) return SHAPE_DIAMOND;
    return SHAPE_NONE;
}

bool count_not_by_leaves(const Plan& p) {
    const int sh = edge_shape(p);  // the induced 4-path and 4-cycle search the 4-cycles
    return (sh != SHAPE_NONE && sh != SHAPE_IPATH4 && sh != SHAPE_ICYCLE4) ||
           (plan_is_clique(p) && p.oriented && p.k >= 4 && p.k <= 6);
}

namespace {

struct CountBuffers {
    unsigned long long* part;
    size_t part_blocks;
    unsigned long long* cells;
    uint32_t* ovf;
    uint64_t ovf_cap;
};

const Plan& clique4_plan() {
    static const Plan plan = [] {
        const int32_t e[12] = {0, 1, 0, 2, 0, 3, 1, 2, 1, 3, 2, 3};
        Plan q{};
        std::string err;
        (void)compile_pattern(4, 6, e, 0, q, err);
        return q;
    }();
    return plan;
}

const Plan& cycle4_plan() {
    static const Plan plan = [] {
        const int32_t e[8] = {0, 1, 1, 2, 2, 3, 3, 0};
        Plan q{};
        std::string err;
        (void)compile_pattern(4, 4, e, 0, q, err);
        return q;
    }();
    return plan;
}

bool bitmap_count_applies(const Plan& p, uint64_t nfirst) {
    return plan_is_clique(p) && p.oriented && p.k >= 4 && p.k <= 6 && nfirst <= (1ull << 28) &&
           !std::getenv("SGPM_EXACT_GROUP");
}

sgpm_status exact_count_with(sgpm_ctx* c, sgpm_graph* g, const Plan& p, const CountBuffers& b, unsigned __int128* out,
                             double* seconds) {
    const uint64_t nfirst = p.oriented ? (uint64_t)g->m : 2ull * (uint64_t)g->m;
    *out = 0;
    if (seconds) *seconds = 0.0;
    if (nfirst == 0) return SGPM_OK;
    const bool bitmap = bitmap_count_applies(p, nfirst) && nfirst <= b.ovf_cap;
    const int shape = std::getenv("SGPM_EXACT_GROUP") ? (int)SHAPE_NONE : edge_shape(p);
    int group = exact_group(g, p);
    // cells, three passes of ticket, count or spare, 2 sums: the 64-member
    // bitmaps (0-3), the 128-member bitmaps (4-7), the general search (8-11);
    // words 16 on are the 4-clique count's of an induced pattern with a closed form,
    // words 32 on the 4-cycle count's
    unsigned long long* d = b.cells;
    HIP_TRY(c, launch_fill_u64(d, 12, 0ull, c->st));
    ScopedEvents<2> ev;
    if (seconds) {
        HIP_TRY(c, ev.create());
        HIP_TRY(c, hipEventRecord(ev.e[0], c->st));
    }
    // Ticket plans.  Every ticket is one atomic on one counter, and those
    // serialise at about 12 ns per wave-wide atomic on this device, so a
    // kernel of T tickets takes at least 12 T ns.  The general search: about
    // 32 tickets per wave (over the wave's groups), starting at one edge (four
    // for narrow groups) and growing linearly, since the search below a first
    // edge costs the most on the high-degree rows at the front of the edge
    // order.  The bitmap count (even, short work per edge): about 8 tickets
    // per wave of at least 32 edges each.
    auto general_plan = [&](int grp, int blocks, uint64_t nf) {
        const uint64_t T = (uint64_t)blocks * 4 * 32, base = grp == 64 ? 1 : 4;
        if (nf <= base * T || nf >= (1ull << 32)) return TicketPlan{std::max<uint64_t>(base, nf / T), 0};
        return TicketPlan{base, std::max<uint64_t>(1, T * T / (2 * (nf - base * T)))};
    };
    auto bitmap_plan = [&](int blocks, uint64_t nf) {
        return TicketPlan{std::max<uint64_t>(32, nf / ((uint64_t)blocks * 4 * 8)), 0};
    };
    if (shape != SHAPE_NONE) {
        // terms: ET 0 diamond, 1 tailed, 2 4-path, 3 3-star, 4 wedge, 5 induced wedge
        int sel[3] = {-1, -1, -1};
        const bool ind = p.induced != 0;
        switch (shape) {
            case SHAPE_WEDGE: sel[0] = ind ? 5 : 4; break;
            case SHAPE_STAR3: sel[0] = 3; if (ind) { sel[1] = 1; sel[2] = 0; } break;
            case SHAPE_PATH4: sel[0] = 2; break;
            case SHAPE_TAILED: sel[0] = 1; if (ind) sel[1] = 0; break;
            case SHAPE_IPATH4: sel[0] = 2; sel[1] = 1; sel[2] = 0; break;
            default: sel[0] = 0; break;  // diamond, induced 4-cycle
        }
        const bool need_t = !((shape == SHAPE_WEDGE || shape == SHAPE_STAR3) && !ind);
        const bool need_k4 = ind && shape != SHAPE_WEDGE;
        const bool need_c4 = shape == SHAPE_IPATH4 || shape == SHAPE_ICYCLE4;
        // 8 lanes per edge unless some rows are long (hubs), where 64 pay:
        // diamond, R-MAT 20 at c = 16 (max degree 3,983) 1.2 ms at 8 lanes, 3.3
        // at 64; R-MAT 20 at c = 4 (about 16K) 15.7 and 5.2; R-MAT 24 at c = 16
        // (about 25K) 51 and 15.7.  Six partial words per block: at most a
        // third of the partials slots.
        const int grp = (2.0 * (double)g->m >= 16.0 * (double)g->n || g->maxdeg >= 8192) ? 64 : 8;
        const int blocks =
            (int)std::min<size_t>((size_t)c->cus * (size_t)edge_terms_blocks_per_cu(grp, need_t), b.part_blocks / 3);
        if (blocks < 1) return fail(c, SGPM_EINVAL, "the count's launch exceeds its partials buffer");
        HIP_TRY(c, launch_edge_terms(g->view(), grp, need_t, blocks, general_plan(grp, blocks, (uint64_t)g->m), sel,
                                     d, b.part, d + 4, c->st));
        unsigned __int128 k4 = 0, c4 = 0;
        if (need_k4) {
            CountBuffers bk = b;
            bk.cells = b.cells + 16;
            sgpm_status st = exact_count_with(c, g, clique4_plan(), bk, &k4, nullptr);
            if (st != SGPM_OK) return st;
        }
        if (need_c4) {  // the 4-cycles by the general search (cells 32 on)
            CountBuffers bc = b;
            bc.cells = b.cells + 32;
            sgpm_status st = exact_count_with(c, g, cycle4_plan(), bc, &c4, nullptr);
            if (st != SGPM_OK) return st;
        }
        if (seconds) HIP_TRY(c, hipEventRecord(ev.e[1], c->st));
        unsigned long long six[6];
        HIP_TRY(c, hipMemcpyAsync(six, d + 4, sizeof(six), hipMemcpyDeviceToHost, c->st));
        HIP_TRY(c, hipStreamSynchronize(c->st));
        if (seconds) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, ev.e[0], ev.e[1]);
            *seconds = ms * 1e-3;
        }
        __int128 S[3];
        for (int q = 0; q < 3; q++) S[q] = (__int128)six[2 * q] + ((__int128)six[2 * q + 1] << 32);
        const __int128 K4 = (__int128)k4, C4 = (__int128)c4;
        __int128 v = -1;
        bool exact = true;  // the divisions are exact by the identities
        auto div = [&](__int128 x, int q) {
            if (x % q != 0) exact = false;
            return x / q;
        };
        switch (shape) {
            case SHAPE_WEDGE: v = div(S[0], 2); break;
            case SHAPE_STAR3: v = ind ? div(S[0], 3) - div(S[1], 2) + 2 * S[2] - 4 * K4 : div(S[0], 3); break;
            case SHAPE_PATH4: v = S[0]; break;
            case SHAPE_TAILED: v = ind ? div(S[0], 2) - 4 * S[1] + 12 * K4 : div(S[0], 2); break;
            case SHAPE_IPATH4: v = S[0] - S[1] - 4 * C4 + 6 * S[2] - 12 * K4; break;  // S[1] = 2 tt
            case SHAPE_ICYCLE4: v = C4 - S[0] + 3 * K4; break;
            default: v = ind ? S[0] - 6 * K4 : S[0]; break;
        }
        if (!exact || v < 0) return fail(c, SGPM_EHIP, "internal: per-edge terms do not give a count");
        *out = (unsigned __int128)v;
        return SGPM_OK;
    }
    // Bitmap passes: candidate sets of up to 64 members, then the first pass's
    // list of larger sets at up to 128 members when the second list fits after
    // the first; what is left goes to the general search.
    uint64_t rest = 0;  // first edges left to the general search (bitmap count)
    const uint32_t* rest_list = nullptr;
    if (bitmap) {
        const int blocks = c->cus * clique_bitmap_blocks_per_cu(p.k);
        if ((size_t)blocks > b.part_blocks) return fail(c, SGPM_EINVAL, "the count's launch exceeds its partials buffer");
        HIP_TRY(c, launch_clique_bitmap(g->view(), p.k, nfirst, blocks, bitmap_plan(blocks, nfirst), d, b.part,
                                        d + 2, b.ovf, d + 1, c->st));
        unsigned long long nov = 0;
        HIP_TRY(c, hipMemcpyAsync(&nov, d + 1, sizeof(nov), hipMemcpyDeviceToHost, c->st));
        HIP_TRY(c, hipStreamSynchronize(c->st));
        rest = nov;
        rest_list = b.ovf;
        if (nov > 0 && 2 * nov <= b.ovf_cap) {
            const int blocks2 = c->cus * clique_bitmap128_blocks_per_cu(p.k);
            if ((size_t)blocks2 > b.part_blocks)
                return fail(c, SGPM_EINVAL, "the count's launch exceeds its partials buffer");
            HIP_TRY(c, launch_clique_bitmap128(g->view(), p.k, b.ovf, nov, blocks2, general_plan(64, blocks2, nov),
                                               d + 4, b.part, d + 6, b.ovf + nov, d + 5, c->st));
            unsigned long long nov2 = 0;
            HIP_TRY(c, hipMemcpyAsync(&nov2, d + 5, sizeof(nov2), hipMemcpyDeviceToHost, c->st));
            HIP_TRY(c, hipStreamSynchronize(c->st));
            rest = nov2;
            rest_list = b.ovf + nov;
        }
        group = 64;
    }
    if (!bitmap || rest > 0) {
        const uint64_t nf = bitmap ? rest : nfirst;
        const int blocks = c->cus * exact_blocks_per_cu(group);
        if ((size_t)blocks > b.part_blocks) return fail(c, SGPM_EINVAL, "the count's launch exceeds its partials buffer");
        HIP_TRY(c, launch_exact_count(g->view(), p, nf, group, blocks, general_plan(group, blocks, nf), d + 8, b.part,
                                      d + 10, bitmap ? rest_list : nullptr, c->st));
    }
    if (seconds) HIP_TRY(c, hipEventRecord(ev.e[1], c->st));
    unsigned long long sums[12];
    HIP_TRY(c, hipMemcpyAsync(sums, d, sizeof(sums), hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    if (seconds) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ev.e[0], ev.e[1]);
        *seconds = ms * 1e-3;
    }
    // low and high 32-bit halves of the three passes' sums
    unsigned __int128 total = 0;
    for (int q = 2; q < 12; q += 4) total += (unsigned __int128)sums[q] + ((unsigned __int128)sums[q + 1] << 32);
    *out = total;
    return SGPM_OK;
}

}  // namespace

sgpm_status exact_count(sgpm_ctx* c, sgpm_graph* g, const Plan& p, unsigned __int128* out, double* seconds) {
    HIP_TRY(c, hipSetDevice(c->dev));
    const uint64_t nfirst = p.oriented ? (uint64_t)g->m : 2ull * (uint64_t)g->m;
    *out = 0;
    if (seconds) *seconds = 0.0;
    if (nfirst == 0) return SGPM_OK;
    const bool bitmap = bitmap_count_applies(p, nfirst);
    const int shape = edge_shape(p);
    const bool closed = shape != SHAPE_NONE;  // a closed form over edges (its 4-cliques when induced)
    const int maxblocks = c->cus * std::max({exact_blocks_per_cu(64), exact_blocks_per_cu(exact_group(g, p)),
                                             bitmap || closed ? clique_bitmap_blocks_per_cu(4) : 1,
                                             bitmap ? std::max(clique_bitmap_blocks_per_cu(p.k), clique_bitmap128_blocks_per_cu(p.k)) : 1,
                                             closed ? clique_bitmap128_blocks_per_cu(4) : 1,
                                             closed ? exact_blocks_per_cu(16) : 1,
                                             1});
    // the per-edge terms take three slots per block
    const int term_blocks = closed ? c->cus * std::max({edge_terms_blocks_per_cu(8, true),
                                                         edge_terms_blocks_per_cu(64, true),
                                                         edge_terms_blocks_per_cu(64, false)})
                                    : 0;
    CountBuffers b{};
    b.part_blocks = std::max((size_t)maxblocks, 3 * (size_t)term_blocks);
    GS_SCRATCH(c, GS_PART, sizeof(unsigned long long) * 2 * b.part_blocks, b.part);
    GS_SCRATCH(c, GS_CELL, sizeof(unsigned long long) * kCountCells, b.cells);
    if (bitmap || (closed && p.induced)) {  // an induced closed form counts 4-cliques over the m oriented edges
        // room for the first bitmap pass's list and, after it, the second's
        const uint64_t cap = 2 * std::max<uint64_t>(nfirst, (uint64_t)g->m);
        GS_SCRATCH(c, GS_OVF, sizeof(uint32_t) * (size_t)std::max<uint64_t>(cap, 1), b.ovf);
        b.ovf_cap = cap;
    }
    return exact_count_with(c, g, p, b, out, seconds);
}

sgpm_status gs_rep(sgpm_ctx* c, sgpm_graph* g, const Plan& p, uint32_t colours, uint64_t seed, uint32_t rep,
                   unsigned __int128* y, double* dev_seconds, bool bes) {
    sgpm_graph* sp = nullptr;
    sgpm_status st = sparsify(c, g, colours, seed, rep, &sp, bes, true);
    if (st != SGPM_OK) return st;
    st = exact_count(c, sp, p, y, dev_seconds);
    sgpm_graph_free(sp);
    return st;
}

// colours = 0: choose c in 4..16 (Sec. 4.4, the colour-count figure, and
// Sec. 5.2).  A colouring's time is sparsification (one pass over the arcs,
// nearly independent of c) plus the exact search, whose leaves shrink as
// c^-(k-1) (a match survives when its k vertices share a colour).  Past some c
// the sparsification dominates and the time stops falling (the paper's
// stabilisation window), so the fewest colours -- the largest keep probability,
// hence the lowest variance -- inside that window are the best choice.  One
// probe colouring at c = 16 (repetition id kColourProbeRep, outside the ids the
// estimate uses) counts its leaves Y16; with the device rates of the two parts
// (sparsification 1e11 arcs/s plus 0.3 ms of launches per colouring; the
// search 3e9 leaves/s, measured 1.4e9 to 3.7e9 on a sparsified power-law
// graph) a colouring at c is predicted to take 2m / 1e11 + 3e-4 +
// Y16 (16 / c)^(k-1) / 3e9 seconds, and c is the smallest of 4, 5, 6, 8, 10,
// 12, 16 predicted within 25 % of the time at 16.  The choice depends only on
// the graph, the pattern and the seed, so runs repeat exactly.
constexpr uint32_t kColourProbeRep = 0x3FFFFFFFu;

double gs_sparsify_model_s(int64_t m) { return 2.0 * (double)m / 1e11 + 3e-4; }

uint32_t colours_from_probe(int64_t m, int k, double leaves16) {
    static const uint32_t cands[] = {4, 5, 6, 8, 10, 12, 16};
    const double t_sp = gs_sparsify_model_s(m);
    const double at16 = t_sp + leaves16 / 3e9;
    for (uint32_t cc : cands)
        if (t_sp + leaves16 * std::pow(16.0 / (double)cc, (double)(k - 1)) / 3e9 <= 1.25 * at16) return cc;
    return 16;
}

sgpm_status gs_choose_colours(sgpm_ctx* c, sgpm_graph* g, const Plan& p, uint64_t seed, uint32_t* out) {
    sgpm_graph* sp = nullptr;
    sgpm_status st = sparsify(c, g, 16, seed, kColourProbeRep, &sp, false, true);
    if (st != SGPM_OK) return st;
    unsigned __int128 y = 0;
    st = exact_count(c, sp, p, &y, nullptr);
    sgpm_graph_free(sp);
    if (st != SGPM_OK) return st;
    *out = colours_from_probe(g->m, p.k, (double)y);
    return SGPM_OK;
}

sgpm_status gs_resolve_colours(sgpm_ctx* c, sgpm_graph* g, const Plan& p, const sgpm_options& o, uint32_t* col) {
    if (o.colours < 0 || o.colours > 256) return fail(c, SGPM_EINVAL, "colours must be 0 (choose) or in [1, 256]");
    if (o.colours > 0) {
        *col = (uint32_t)o.colours;
        return SGPM_OK;
    }
    if (o.gs_scheme == SGPM_GS_BERNOULLI) {
        *col = 8;  // the choice follows the colour scheme's survival law; Bernoulli takes c = 8
        return SGPM_OK;
    }
    return gs_choose_colours(c, g, p, o.seed, col);
}

sgpm_status gs_estimate(sgpm_ctx* c, sgpm_graph* g, const Plan& p, const sgpm_options& o, sgpm_result* res,
                        const GsPrefix* pre) {
    auto t0 = std::chrono::steady_clock::now();
    std::memset(res, 0, sizeof(*res));
    res->scheme = SGPM_SCHEME_GS;
    uint32_t col = 0;
    if (pre) {
        col = (uint32_t)o.colours;  // the hybrid resolved it before its pilot colourings
    } else {
        sgpm_status st = gs_resolve_colours(c, g, p, o, &col);
        if (st != SGPM_OK) return st;
    }
    if (col < 1 || col > 256) return fail(c, SGPM_EINVAL, "colours must be 0 (choose) or in [1, 256]");
    const int reps = o.gs_reps_max > 0 ? o.gs_reps_max : 64;
    double z = student_t_quantile(o.confidence, 1);
    // Bernoulli edge sparsification keeps every edge with probability 1/c, so
    // a match survives with c^-l (l pattern edges); it does not preserve
    // non-edges, so vertex-induced constraints are refused
    const bool bes = o.gs_scheme == SGPM_GS_BERNOULLI;
    int expo = p.k - 1;
    if (bes) {
        expo = 0;
        for (int j = 1; j < p.k; j++) {
            if (p.disconnect[j]) return fail(c, SGPM_EUNSUPPORTED, "Bernoulli edge sparsification is edge-induced");
            expo += __builtin_popcount((unsigned)p.connect[j]);
        }
    }
    // c^(k-1) (colours) or c^l (Bernoulli) as an exact integer
    unsigned __int128 scale = 1;
    for (int i = 0; i < expo; i++) {
        if (scale > ~(unsigned __int128)0 / col) return fail(c, SGPM_EOVERFLOW, "GS scale exceeds 128 bits");
        scale *= col;
    }
    Big S1(24), S2(24);
    uint64_t n = 0, nonzero = 0;
    double dev = pre ? pre->dev_seconds : 0.0;
    bool converged = false;
    for (int r = 0; r < reps; r++) {
        unsigned __int128 y = 0;
        if (pre && r < pre->n) {
            y = pre->y[r];
        } else {
            double secs = 0;
            sgpm_status st = gs_rep(c, g, p, col, o.seed, (uint32_t)r, &y, &secs, bes);
            if (st != SGPM_OK) return st;
            dev += secs;
        }
        const unsigned __int128 x = y * scale;
        if (scale && x / scale != y) return fail(c, SGPM_EOVERFLOW, "GS estimate exceeds 128 bits");
        unsigned long long d1[4], d2[8];
        for (int i = 0; i < 4; i++) d1[i] = (unsigned long long)(uint32_t)(x >> (32 * i));
        // x^2 as 32-bit digit columns (each < 2^35: low and high halves of the digit products)
        for (int i = 0; i < 8; i++) d2[i] = 0;
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++) {
                const unsigned long long pr = d1[a] * d1[b];
                d2[a + b] += pr & 0xFFFFFFFFull;
                if (a + b + 1 < 8) d2[a + b + 1] += pr >> 32;
            }
        big_add_digits(S1, d1, 4);
        big_add_digits(S2, d2, 8);
        n++;
        if (y) nonzero++;
        if (n >= 2) z = student_t_quantile(o.confidence, (int)(n - 1));
        const double eh = predicted_error_t(z, n, S1, S2);
        if (n >= kGsMinReps && eh <= o.eps) {
            converged = true;
            break;
        }
    }
    res->n_samples = n;
    res->n_hits = nonzero;
    for (int i = 0; i < 8; i++) res->sum_digits[i] = S1.d[(size_t)i];
    for (int i = 0; i < 12; i++) res->sumsq_digits[i] = S2.d[(size_t)i];
    res->estimate = big_to_double(S1) / (double)n;
    res->eps_hat = predicted_error_t(z, n, S1, S2);
    res->z = z;
    const double sigma = std::isfinite(res->eps_hat) ? res->estimate * res->eps_hat / z : INFINITY;
    res->ci_lo = res->estimate - z * sigma;
    res->ci_hi = res->estimate + z * sigma;
    res->colours = (int32_t)col;
    res->converged = converged ? 1 : 0;
    res->windows = (int32_t)n;
    res->seconds_kernel = dev;
    res->seconds_sampling = dev;
    res->seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (!converged) return fail(c, SGPM_NOT_CONVERGED, "gs_reps_max colourings reached");
    return SGPM_OK;
}

}  // namespace sgpm

using namespace sgpm;

extern "C" {

sgpm_status sgpm_gs_sparsify(sgpm_ctx_t c, sgpm_graph_t g, uint32_t colours, uint64_t seed, uint32_t rep,
                             sgpm_graph_t* out) {
    if (!c || !g || !out) return fail(c, SGPM_EINVAL, "null argument");
    return sparsify(c, g, colours, seed, rep, out);
}

sgpm_status sgpm_bes_sparsify(sgpm_ctx_t c, sgpm_graph_t g, uint32_t inv_p, uint64_t seed, uint32_t rep,
                              sgpm_graph_t* out) {
    if (!c || !g || !out) return fail(c, SGPM_EINVAL, "null argument");
    return sparsify(c, g, inv_p, seed, rep, out, true);
}

sgpm_status sgpm_exact_count(sgpm_ctx_t c, sgpm_graph_t g, sgpm_pattern_t p, uint64_t* count_lo, uint64_t* count_hi) {
    if (!c || !g || !p || !count_lo) return fail(c, SGPM_EINVAL, "null argument");
    unsigned __int128 v = 0;
    sgpm_status st = exact_count(c, g, p->plan, &v, nullptr);
    if (st != SGPM_OK) return st;
    *count_lo = (uint64_t)v;
    if (count_hi) *count_hi = (uint64_t)(v >> 64);
    return SGPM_OK;
}

// sgpm_exact_count with its scratch in the device's file-scope array (no
// allocation): the same kernels and ticket plans, so the same count.  A graph
// whose first edges outnumber the array's list takes the general search for
// cliques too, which counts the same tuples.
sgpm_status sgpm_exact_count_noalloc(sgpm_ctx_t c, sgpm_graph_t g, sgpm_pattern_t p, uint64_t* count_lo,
                                     uint64_t* count_hi) {
    if (!c || !g || !p || !count_lo) return fail(c, SGPM_EINVAL, "null argument");
    HIP_TRY(c, hipSetDevice(c->dev));
    unsigned long long* base = nullptr;
    HIP_TRY(c, count_scratch_address(c->dev, &base));
    CountBuffers b{};
    b.part = base;
    b.part_blocks = kCountScratchBlocks;
    b.cells = base + 2 * kCountScratchBlocks;
    b.ovf = (uint32_t*)(base + 2 * kCountScratchBlocks + kCountCells);
    b.ovf_cap = kCountScratchOvf;
    unsigned __int128 v = 0;
    sgpm_status st = exact_count_with(c, g, p->plan, b, &v, nullptr);
    if (st != SGPM_OK) return st;
    *count_lo = (uint64_t)v;
    if (count_hi) *count_hi = (uint64_t)(v >> 64);
    return SGPM_OK;
}

}  // extern "C"
