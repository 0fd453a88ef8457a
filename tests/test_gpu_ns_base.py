"""NS-base (lazy verification) on the GPU against the CPU oracle, through the
C-ABI: the sampler the paper measures NS-prune against (Sec. 4.2).

Bar: walks, statuses (including failed closure checks), weights, exact
integer sums, hit counts and checksums are bit-identical to the oracle's.
Cases: every pattern edge- and vertex-induced with a ragged sample count and a
traced id range; hubs whose unions exceed the kernel's LDS list (the rescan
path); the strict stop rule; the degenerate graphs; options NS-base rejects.
"""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NAMES = ["edge", "triangle", "wedge", "4-clique", "4-cycle", "4-path", "3-star", "tailed-triangle", "diamond",
         "house", "5-clique"]


@pytest.fixture(scope="module")
def S():
    from paper_2405_03488_amd import sgpm
    return sgpm


@pytest.fixture(scope="module")
def ctx(S):
    c = S.sgpm_create(0)
    yield c
    S.sgpm_destroy(c)


def addr(buf):
    return C.cast(buf, C.c_void_p).value


def load(S, O, synth, ctx, n, pairs):
    off, nbr = synth.pairs_to_csr(n, pairs)
    return S.sgpm_graph_from_csr(ctx, n, off, nbr), O.OGraph.from_raw_csr(n, off, nbr)


def check_run(r, orr):
    assert (r.n_samples, r.S1, r.S2, r.n_hits, r.checksum) == (orr.n, orr.S1, orr.S2, orr.hits, orr.checksum)
    assert r.estimate == orr.estimate
    assert r.eps_hat == orr.eps_hat or (np.isinf(r.eps_hat) and np.isinf(orr.eps_hat))


def check_trace(buf, recs):
    assert len(buf) == len(recs)
    for a, b in zip(buf, recs):
        st = 0xFF if b.hit else b.fail_step
        assert (a.s, a.status, list(a.v), a.alpha) == (b.s, st, list(b.v), b.alpha), (a.s, b.s)


@pytest.fixture(scope="module")
def cl_graph(S, O, synth, ctx):
    print("building Chung-Lu(3000, 12, 2.1)", flush=True)
    g, og = load(S, O, synth, ctx, 3000, synth.chung_lu_pairs(3000, 12, 2.1, 4))
    yield g, og
    S.sgpm_graph_free(g)


@pytest.fixture(scope="module")
def hub_graph(S, O, synth, ctx):
    """Two hubs of 2,500 leaves each, joined, plus a sparse random layer: the
    union of a hub's row with another row exceeds the kernel's 896-entry list."""
    rng = np.random.default_rng(7)
    n = 6000
    pairs = [(0, 1)] + [(0, i) for i in range(2, 2502)] + [(1, i) for i in range(2002, 4502)]
    pairs += [tuple(x) for x in rng.integers(2, n, size=(6000, 2)).tolist() if x[0] != x[1]]
    print("building two-hub graph", flush=True)
    g, og = load(S, O, synth, ctx, n, np.array(pairs, dtype=np.int32))
    yield g, og
    S.sgpm_graph_free(g)


@pytest.mark.parametrize("induced", [False, True])
@pytest.mark.parametrize("name", NAMES)
def test_fixed_n_matches_oracle(S, O, synth, ctx, cl_graph, name, induced):
    print(f"NS-base {name} induced={induced}", flush=True)
    g, og = cl_graph
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e, induced)
    op = O.compile_plan(k, e, induced)
    N = 60000 + 77
    orr = O.run(og, op, O.make_opts(fixed_n=N, seed=13, tag=3, sampler=1))
    buf = S.trace_buffer(600)
    opts = S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=13, query_tag=3, checksum=1,
                                  sampler=S.SAMPLER_BASE, trace_lo=N - 400, trace_hi=N + 200, trace_buf=addr(buf))
    r, _ = S.sgpm_estimate(ctx, g, p, opts)
    check_run(r, orr)
    check_trace(buf[:400], O.trace_base(og, op, 13, 3, N - 400, 400))
    assert all(x.s == 0 and x.k == 0 for x in buf[400:])
    assert r.lanes_per_sample == 64
    S.sgpm_pattern_free(p)


@pytest.mark.parametrize("name", ["triangle", "4-clique", "diamond"])
def test_unions_beyond_the_list(S, O, synth, ctx, hub_graph, name):
    g, og = hub_graph
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    op = O.compile_plan(k, e)
    N = 20000 + 5
    recs = O.trace_base(og, op, 21, 1, 0, N)
    big = sum(1 for x in recs if any(int(x.size[j]) > 896 for j in range(2, k)))
    assert big > 100  # the rescan path is exercised
    orr = O.run(og, op, O.make_opts(fixed_n=N, seed=21, tag=1, sampler=1))
    buf = S.trace_buffer(N)
    opts = S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=21, query_tag=1, checksum=1,
                                  sampler=S.SAMPLER_BASE, trace_lo=0, trace_hi=N, trace_buf=addr(buf))
    r, _ = S.sgpm_estimate(ctx, g, p, opts)
    check_run(r, orr)
    check_trace(buf, recs)
    S.sgpm_pattern_free(p)


def test_strict_mode_matches_oracle(S, O, synth, ctx, cl_graph):
    g, og = cl_graph
    k, e = synth.pattern("triangle")
    p = S.sgpm_pattern_create(ctx, k, e)
    kw = dict(n_min=20000, w_min=20000, quantum=1000)
    opts = S.sgpm_options_default(eps=0.05, seed=4, checksum=1, sampler=S.SAMPLER_BASE, window_growth=0.1, **kw)
    r, rc = S.sgpm_estimate(ctx, g, p, opts)
    orr = O.run(og, O.compile_plan(k, e), O.make_opts(eps=0.05, seed=4, growth=0.1, sampler=1, **kw))
    check_run(r, orr)
    assert r.windows == orr.windows and r.converged == orr.converged == 1 and rc == S.SGPM_OK
    # NS-prune on the same graph stops with fewer samples (a higher hit rate, smaller weights)
    rp, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(eps=0.05, seed=4, window_growth=0.1, **kw))
    assert rp.n_samples <= r.n_samples and rp.n_hits / rp.n_samples > r.n_hits / r.n_samples
    S.sgpm_pattern_free(p)


def test_degenerate_graphs_and_rejected_options(S, O, synth, ctx):
    g, og = load(S, O, synth, ctx, 5, np.zeros((0, 2), dtype=np.int32))
    k, e = synth.pattern("triangle")
    p = S.sgpm_pattern_create(ctx, k, e)
    r, rc = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(sampler=S.SAMPLER_BASE))
    assert rc == S.SGPM_OK and r.estimate == 0.0 and r.n_samples == 0
    S.sgpm_graph_free(g)
    g, og = load(S, O, synth, ctx, 40, synth.er_pairs(40, 100, 2))
    for kw in (dict(mode=S.MODE_GS), dict(mode=S.MODE_HYBRID), dict(sampler=2)):
        with pytest.raises(S.SgpmError):
            S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(sampler=kw.pop("sampler", S.SAMPLER_BASE), **kw))
    with pytest.raises(S.SgpmError):
        S.sgpm_estimate_batch(ctx, [g], [p], [S.sgpm_options_default(sampler=S.SAMPLER_BASE)])
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)
