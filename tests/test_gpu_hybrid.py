"""Loose mode (hybrid NS/GS selection, Sec. 5.1) on the GPU.

Whatever engine the pilots select, the hybrid result equals that engine's
own result with the same options bit for bit (the NS pilot draws from its own
Philox stream; the GS pilot colourings are the GS run's first two).  Two
clear-cut cases check the choice itself: a common pattern on a power-law
graph (NS), and a handful of planted 5-cliques in a large sparse graph, where
NS pilots see almost no hits while one exact count is cheap (GS)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2405_03488_amd import sgpm
    return sgpm


@pytest.fixture(scope="module")
def ctx(S):
    c = S.sgpm_create(0)
    yield c
    S.sgpm_destroy(c)


def same(a, b):
    assert a.scheme == b.scheme and a.n_samples == b.n_samples
    assert a.S1 == b.S1 and a.S2 == b.S2 and a.n_hits == b.n_hits
    assert a.checksum == b.checksum and a.converged == b.converged and a.windows == b.windows
    assert a.estimate == b.estimate and a.eps_hat == b.eps_hat


def run_pair(S, ctx, g, p, **kw):
    oh = S.sgpm_options_default(mode=S.MODE_HYBRID, **kw)
    rh, _ = S.sgpm_estimate(ctx, g, p, oh)
    mode = S.MODE_GS if rh.scheme == S.SCHEME_GS else S.MODE_STRICT_NS
    ro, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=mode, **kw))
    same(rh, ro)
    print("hybrid:", "GS" if rh.scheme == S.SCHEME_GS else "NS", "ns cone", rh.pred_ns_lo, rh.pred_ns_hi, "gs",
          rh.pred_gs, "pilot s", rh.seconds_pilot, flush=True)
    assert rh.pred_ns_lo <= rh.pred_ns_hi and rh.seconds_pilot > 0
    return rh


def test_hybrid_picks_ns_for_a_common_pattern(S, synth, ctx):
    n = 20000
    off, nbr = synth.pairs_to_csr(n, synth.chung_lu_pairs(n, 16, 2.1, 4))
    g = S.sgpm_graph_from_csr(ctx, n, off, nbr)
    p = S.sgpm_pattern_create(ctx, *synth.pattern("triangle"))
    rh = run_pair(S, ctx, g, p, eps=0.02, seed=5, checksum=1, colours=2)
    assert rh.scheme == S.SCHEME_NS and np.isfinite(rh.pred_ns_lo)
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)


@pytest.mark.parametrize("case", ["stops_in_pilot", "max_samples_first", "tiny_first", "many_windows"])
def test_pilot_window_ends(S, O, synth, ctx, case):
    """The NS pilot is the estimate's first window: when NS is chosen the
    estimate applies that window's stop test before any launch of its own.
    Whether the run stops there (eps reached, max_samples reached) or goes on
    (tiny first windows, many windows), the hybrid result equals strict NS and
    the oracle's run bit for bit."""
    n = 20000
    off, nbr = synth.pairs_to_csr(n, synth.chung_lu_pairs(n, 16, 2.1, 4))
    g = S.sgpm_graph_from_csr(ctx, n, off, nbr)
    og = O.OGraph.from_raw_csr(n, off, nbr)
    k, e = synth.pattern("triangle")
    p = S.sgpm_pattern_create(ctx, k, e)
    kw = {"stops_in_pilot": dict(eps=0.2, n_min=1 << 16, w_min=1 << 14, quantum=1),
          "max_samples_first": dict(eps=1e-4, n_min=1 << 15, w_min=1 << 14, quantum=1, max_samples=1 << 15),
          "tiny_first": dict(eps=0.03, n_min=5, w_min=1 << 12, quantum=1),
          "many_windows": dict(eps=0.01, n_min=1 << 12, w_min=1 << 12, quantum=1 << 8)}[case]
    kw.update(seed=21, checksum=1, colours=2)
    rh = run_pair(S, ctx, g, p, **kw)
    if case in ("stops_in_pilot", "max_samples_first"):
        assert rh.scheme == S.SCHEME_NS  # one window of NS against two colourings
    elif rh.scheme == S.SCHEME_GS:
        # the pilots chose GS (equal to the GS mode's run, checked above)
        S.sgpm_pattern_free(p)
        S.sgpm_graph_free(g)
        return
    oo = O.make_opts(eps=kw["eps"], confidence=0.95, seed=21, tag=0, n_min=kw["n_min"], w_min=kw["w_min"],
                     quantum=kw["quantum"], max_samples=kw.get("max_samples", 1 << 40))
    orr = O.run(og, O.compile_plan(k, e), oo)
    assert rh.n_samples == orr.n and rh.windows == orr.windows and rh.converged == orr.converged
    assert rh.S1 == orr.S1 and rh.S2 == orr.S2 and rh.checksum == orr.checksum
    if case == "stops_in_pilot":
        assert rh.windows == 1 and rh.converged == 1
    if case == "max_samples_first":
        assert rh.windows == 1 and rh.converged == 0 and rh.n_samples == 1 << 15
    if case == "many_windows":
        assert rh.windows > 3
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)


def planted(synth, n, m, cliques, k, seed):
    rng = np.random.default_rng(seed)
    pairs = [synth.er_pairs(n, m, seed)]
    for _ in range(cliques):
        vs = rng.choice(n, size=k, replace=False)
        pairs.append(np.array([(a, b) for i, a in enumerate(vs) for b in vs[i + 1:]], dtype=np.int32))
    return np.concatenate(pairs).astype(np.int32)


def test_hybrid_picks_gs_for_rare_matches(S, O, synth, ctx):
    n = 200000
    pairs = planted(synth, n, 200000, 8, 5, 11)
    off, nbr = synth.pairs_to_csr(n, pairs)
    g = S.sgpm_graph_from_csr(ctx, n, off, nbr)
    og = O.OGraph.from_raw_csr(n, off, nbr)
    k, e = synth.pattern("5-clique")
    p = S.sgpm_pattern_create(ctx, k, e)
    exact = O.plan_count(og, O.compile_plan(k, e))
    assert exact >= 8
    # one colour: GS is the exact count, so three identical colourings converge (the rule starts at three)
    rh = run_pair(S, ctx, g, p, eps=0.02, seed=9, checksum=1, colours=1)
    assert rh.scheme == S.SCHEME_GS and rh.converged == 1
    assert rh.estimate == exact and rh.n_samples == 3
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)


@pytest.mark.parametrize("name,colours", [("4-cycle", 2), ("diamond", 4), ("4-clique", 8)])
def test_hybrid_equals_selected_engine(S, synth, ctx, name, colours):
    n = 3000
    off, nbr = synth.pairs_to_csr(n, synth.chung_lu_pairs(n, 12, 2.1, 8))
    g = S.sgpm_graph_from_csr(ctx, n, off, nbr)
    p = S.sgpm_pattern_create(ctx, *synth.pattern(name))
    run_pair(S, ctx, g, p, eps=0.05, seed=17, checksum=1, colours=colours, gs_reps_max=200, n_min=1 << 16,
             w_min=1 << 15, quantum=1 << 12)
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)


def test_hybrid_on_an_edgeless_graph(S, synth, ctx):
    off, nbr = synth.pairs_to_csr(9, np.zeros((0, 2), dtype=np.int32))
    g = S.sgpm_graph_from_csr(ctx, 9, off, nbr)
    p = S.sgpm_pattern_create(ctx, *synth.pattern("triangle"))
    r, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_HYBRID))
    assert r.scheme == S.SCHEME_NS and r.estimate == 0.0 and r.converged == 1
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)


def windows_for(S, pred_samples, quantum):
    q = quantum or 1
    return max(q, math.ceil(0.1 * pred_samples / q) * q)


@pytest.mark.parametrize("name", ["triangle", "4-clique", "diamond"])
def test_cost_model_selector_runs_the_chosen_engine(S, O, synth, ctx, name):
    """Loose mode with the paper's profiler and cost models: the result equals
    the chosen engine run on its own -- NS with windows of 10 % of the
    predicted samples (and the oracle's run with those windows), or GS at the
    chosen colour count."""
    n = 3000
    off, nbr = synth.pairs_to_csr(n, synth.chung_lu_pairs(n, 12, 2.1, 8))
    g = S.sgpm_graph_from_csr(ctx, n, off, nbr)
    og = O.OGraph.from_raw_csr(n, off, nbr)
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    kw = dict(eps=0.05, seed=17, checksum=1, quantum=1 << 10)
    rh, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_HYBRID,
                                                              hybrid_selector=S.HYBRID_COST_MODEL, **kw))
    assert rh.seconds_pilot > 0 and rh.pred_ns_lo <= rh.pred_ns_hi
    if rh.scheme == S.SCHEME_NS:
        w = windows_for(S, rh.pred_samples, kw["quantum"])
        ro, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(n_min=w, w_min=w, window_growth=0.0, **kw))
        same(rh, ro)
        orr = O.run(og, O.compile_plan(k, e), O.make_opts(eps=0.05, seed=17, n_min=w, w_min=w, growth=0.0,
                                                           quantum=kw["quantum"]))
        assert (rh.n_samples, rh.S1, rh.S2, rh.checksum) == (orr.n, orr.S1, orr.S2, orr.checksum)
    else:
        ro, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_GS, colours=rh.colours, **kw))
        same(rh, ro)
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)


def test_cost_model_selector_picks_gs_for_rare_matches(S, O, synth, ctx):
    """A few planted 5-cliques in a large sparse graph: NS pilots find no hit,
    so NS cannot be predicted and GS runs; one colour makes it exact."""
    n = 200000
    pairs = planted(synth, n, 200000, 8, 5, 11)
    off, nbr = synth.pairs_to_csr(n, pairs)
    g = S.sgpm_graph_from_csr(ctx, n, off, nbr)
    og = O.OGraph.from_raw_csr(n, off, nbr)
    k, e = synth.pattern("5-clique")
    p = S.sgpm_pattern_create(ctx, k, e)
    exact = O.plan_count(og, O.compile_plan(k, e))
    rh, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_HYBRID, hybrid_selector=S.HYBRID_COST_MODEL,
                                                              eps=0.02, seed=9, colours=1))
    assert rh.scheme == S.SCHEME_GS and rh.estimate == exact and rh.converged == 1
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)
