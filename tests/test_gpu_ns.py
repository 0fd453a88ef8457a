"""NS-prune on the GPU against the CPU oracle, through the C-ABI.

Bar: walks, hit flags, weights, exact integer sums, hit counts and checksums
are bit-identical; FP64 estimates and predicted errors are identical because
both sides derive them from the same exact integers in the same order.
"""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ALL = ["edge", "triangle", "wedge", "4-clique", "5-clique", "4-cycle", "5-cycle", "4-path", "5-path", "3-star",
       "tailed-triangle", "diamond", "house", "dumbbell", "6-clique"]


@pytest.fixture(scope="module")
def S():
    from paper_2405_03488_amd import sgpm
    return sgpm


@pytest.fixture(scope="module")
def ctx(S):
    c = S.sgpm_create(0)
    yield c
    S.sgpm_destroy(c)


TRACE_DTYPE = np.dtype([("s", "<u8"), ("v", "<i4", 8), ("status", "<u4"), ("k", "<u4"), ("alo", "<u8"),
                        ("ahi", "<u8")])


def addr(buf):
    return C.cast(buf, C.c_void_p).value


def load(S, O, synth, ctx, n, pairs):
    off, nbr = synth.pairs_to_csr(n, pairs)
    g = S.sgpm_graph_from_csr(ctx, n, off, nbr)
    og = O.OGraph.from_raw_csr(n, off, nbr)
    return g, og


def check_run(S, O, r, orr):
    assert r.n_samples == orr.n
    assert r.S1 == orr.S1
    assert r.S2 == orr.S2
    assert r.n_hits == orr.hits
    assert r.checksum == orr.checksum
    assert r.estimate == orr.estimate
    assert r.eps_hat == orr.eps_hat or (np.isinf(r.eps_hat) and np.isinf(orr.eps_hat))


def check_trace(buf, recs):
    assert len(buf) == len(recs)
    for a, b in zip(buf, recs):
        st = 0xFF if b.hit else b.fail_step
        assert (a.s, a.status, list(a.v), a.alpha) == (b.s, st, list(b.v), b.alpha), (a.s, b.s)


@pytest.fixture(scope="module")
def c1(S, O, synth, ctx):
    """ER G(n=10,000, M=80,000) (average degree 16), generator seed 1."""
    print("building C1 ER(10000, 80000)", flush=True)
    g, og = load(S, O, synth, ctx, 10000, synth.er_pairs(10000, 80000, 1))
    yield g, og
    S.sgpm_graph_free(g)


def test_torch_shares_the_hip_runtime(S, ctx):
    import torch
    assert torch.cuda.is_available()
    x = torch.ones(1 << 20, device="cuda")
    torch.cuda.synchronize()
    assert float(x.sum()) == float(1 << 20)


def test_graph_upload_matches_oracle(S, c1, ctx):
    g, og = c1
    off, nbr = S.sgpm_graph_export(ctx, g)
    n, m, maxdeg, perm = S.sgpm_graph_stats(g)
    assert (n, m) == (og.n, og.m)
    assert np.array_equal(off, og.off) and np.array_equal(nbr, og.nbr) and np.array_equal(perm, og.perm)
    assert maxdeg == int(np.diff(og.off).max())


@pytest.mark.parametrize("off_dtype", ["int32", "int64"])
def test_graph_from_device_tensors(S, O, synth, ctx, c1, off_dtype):
    """The raw (unsymmetrised, duplicated) C1 CSR handed over as torch device
    tensors builds the same canonical graph as the host path and the oracle."""
    import torch
    _, og = c1
    off, nbr = synth.pairs_to_csr(10000, synth.er_pairs(10000, 80000, 1))
    d_off = torch.from_numpy(np.asarray(off).astype(off_dtype)).cuda()
    d_nbr = torch.from_numpy(np.asarray(nbr, dtype=np.int32)).cuda()
    g = S.sgpm_graph_from_csr(ctx, 10000, d_off, d_nbr)
    goff, gnbr = S.sgpm_graph_export(ctx, g)
    n, m, _, perm = S.sgpm_graph_stats(g)
    assert (n, m) == (og.n, og.m)
    assert np.array_equal(goff, og.off) and np.array_equal(gnbr, og.nbr) and np.array_equal(perm, og.perm)
    S.sgpm_graph_free(g)


def test_empty_graph_from_device_tensors(S, ctx):
    """Device input with no edges (and with no vertices): nothing to copy for
    the neighbours, and the graph is empty."""
    import torch
    for n in (5, 0):
        d_off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        d_nbr = torch.zeros(0, dtype=torch.int32, device="cuda")
        g = S.sgpm_graph_from_csr(ctx, n, d_off, d_nbr)
        assert S.sgpm_graph_stats(g)[:3] == (n, 0, 0)
        S.sgpm_graph_free(g)


@pytest.mark.parametrize("lanes", [1, 4, 16, 64])
def test_c1_triangle_full_run(S, O, synth, ctx, c1, lanes):
    """Triangles on the ER graph, 1e6 samples, Philox seed 1: sums, hits and
    the full-run checksum equal the oracle's; the first 4096 walks match."""
    print(f"C1 triangle lanes={lanes}", flush=True)
    g, og = c1
    k, e = synth.pattern("triangle")
    p = S.sgpm_pattern_create(ctx, k, e)
    op = O.compile_plan(k, e)
    ntr = 4096
    buf = S.trace_buffer(ntr)
    opts = S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=1000000, seed=1, checksum=1, lanes_per_sample=lanes,
                                  trace_lo=0, trace_hi=ntr, trace_buf=addr(buf))
    r, rc = S.sgpm_estimate(ctx, g, p, opts)
    orr = O.run(og, op, O.make_opts(fixed_n=1000000, seed=1))
    check_run(S, O, r, orr)
    check_trace(buf, O.trace(og, op, 1, 0, 0, ntr))
    S.sgpm_pattern_free(p)


def test_c1_bytes_counted(S, O, synth, ctx, c1):
    g, og = c1
    k, e = synth.pattern("triangle")
    p = S.sgpm_pattern_create(ctx, k, e)
    opts = S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=300000, seed=3, lanes_per_sample=1)
    r, _ = S.sgpm_estimate(ctx, g, p, opts, counted=True)
    orr = O.run(og, O.compile_plan(k, e), O.make_opts(fixed_n=300000, seed=3))
    assert r.bytes == orr.bytes
    S.sgpm_pattern_free(p)


@pytest.fixture(scope="module")
def cl_graph(S, O, synth, ctx):
    print("building Chung-Lu(3000, 12, 2.1)", flush=True)
    g, og = load(S, O, synth, ctx, 3000, synth.chung_lu_pairs(3000, 12, 2.1, 4))
    yield g, og
    S.sgpm_graph_free(g)


@pytest.mark.parametrize("induced", [False, True])
@pytest.mark.parametrize("name", ALL)
def test_patterns_fixed_n(S, O, synth, ctx, cl_graph, name, induced):
    """Every pattern, edge- and vertex-induced, a ragged sample count: lanes
    1, 16 and 64 with a trace (64: the generic one-sample-per-wave kernel) and
    64 without one (the kernel strict runs launch: the clique specialisation
    for cliques of 3 to 6 vertices) must give the oracle's sums and checksum."""
    print(f"pattern {name} induced={induced}", flush=True)
    g, og = cl_graph
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e, induced)
    op = O.compile_plan(k, e, induced)
    N = 200000 + 123
    orr = O.run(og, op, O.make_opts(fixed_n=N, seed=11, tag=5))
    recs = O.trace(og, op, 11, 5, N - 500, 500)
    for lanes in (1, 16, 64):
        buf = S.trace_buffer(700)
        opts = S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=11, query_tag=5, checksum=1,
                                      lanes_per_sample=lanes, trace_lo=N - 500, trace_hi=N + 200,
                                      trace_buf=addr(buf))
        r, _ = S.sgpm_estimate(ctx, g, p, opts)
        assert r.lanes_per_sample == lanes
        check_run(S, O, r, orr)
        check_trace(buf[:500], recs)
        assert all(x.s == 0 and x.k == 0 for x in buf[500:])  # ids beyond the run are never written
    opts = S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=11, query_tag=5, checksum=1,
                                  lanes_per_sample=64)
    r, _ = S.sgpm_estimate(ctx, g, p, opts)
    assert r.lanes_per_sample == 64
    check_run(S, O, r, orr)
    S.sgpm_pattern_free(p)


@pytest.fixture(scope="module")
def dense_small(S, O, synth, ctx):
    print("building ER(300, 25000)", flush=True)
    g, og = load(S, O, synth, ctx, 300, synth.er_pairs(300, 25000, 3))
    yield g, og
    S.sgpm_graph_free(g)


@pytest.mark.parametrize("induced", [False, True])
@pytest.mark.parametrize("name", ["7-clique", "8-clique", "7-cycle", "8-path", "wheel-7"])
def test_seven_and_eight_vertex_patterns(S, O, synth, ctx, dense_small, name, induced):
    """Patterns of 7 and 8 vertices (the largest the library accepts) on a
    dense graph where they have hits: every lane width, traced and not, equals
    the oracle's sums, hits and checksum, and the traced walks match."""
    print(f"pattern {name} induced={induced}", flush=True)
    g, og = dense_small
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e, induced)
    op = O.compile_plan(k, e, induced)
    N = 60000 + 7
    orr = O.run(og, op, O.make_opts(fixed_n=N, seed=5, tag=2))
    assert orr.hits > 10
    recs = O.trace(og, op, 5, 2, 0, 400)
    for lanes in (1, 4, 16, 64):
        buf = S.trace_buffer(400)
        opts = S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=5, query_tag=2, checksum=1,
                                      lanes_per_sample=lanes, trace_lo=0, trace_hi=400, trace_buf=addr(buf))
        r, _ = S.sgpm_estimate(ctx, g, p, opts)
        check_run(S, O, r, orr)
        check_trace(buf, recs)
        r, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=5,
                                                                 query_tag=2, checksum=1, lanes_per_sample=lanes))
        check_run(S, O, r, orr)
    S.sgpm_pattern_free(p)


@pytest.fixture(scope="module")
def dense_big(S, O, synth, ctx):
    """ER(2000, 1.6M): 80 % of all pairs, so an edge's common neighbours number
    about 1,280 and a step's candidate set often exceeds the 896 entries the
    one-sample-per-wave kernels keep in LDS."""
    print("building ER(2000, 1600000)", flush=True)
    g, og = load(S, O, synth, ctx, 2000, synth.er_pairs(2000, 1600000, 7))
    yield g, og
    S.sgpm_graph_free(g)


@pytest.mark.parametrize("name", ["triangle", "4-clique", "diamond", "4-cycle"])
def test_candidate_list_overflow(S, O, synth, ctx, dense_big, name):
    """Candidate sets larger than the LDS list: the kernels count them fully
    and select the drawn member by rescanning the rows.  The oracle shows the
    case occurs in many samples; every width, traced and not, matches it."""
    print(f"overflow {name}", flush=True)
    g, og = dense_big
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    op = O.compile_plan(k, e)
    N = 20000 + 3
    recs = O.trace(og, op, 9, 1, 0, N)
    big = sum(1 for r in recs if max(r.size[2:k]) > 896)
    assert big >= N // 20, big
    orr = O.run(og, op, O.make_opts(fixed_n=N, seed=9, tag=1))
    for lanes in (1, 16, 64):
        buf = S.trace_buffer(N)
        opts = S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=9, query_tag=1, checksum=1,
                                      lanes_per_sample=lanes, trace_lo=0, trace_hi=N, trace_buf=addr(buf))
        r, _ = S.sgpm_estimate(ctx, g, p, opts)
        check_run(S, O, r, orr)
        check_trace(buf, recs)
    r, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=9, query_tag=1,
                                                             checksum=1, lanes_per_sample=64))
    check_run(S, O, r, orr)
    S.sgpm_pattern_free(p)


@pytest.mark.parametrize("name", ["triangle", "4-clique", "4-cycle"])
def test_strict_mode_matches_oracle(S, O, synth, ctx, cl_graph, name):
    g, og = cl_graph
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    kw = dict(n_min=50000, w_min=20000, quantum=1000)
    opts = S.sgpm_options_default(eps=0.02, confidence=0.95, seed=9, checksum=1, lanes_per_sample=0,
                                  window_growth=0.1, **kw)
    r, rc = S.sgpm_estimate(ctx, g, p, opts)
    orr = O.run(og, O.compile_plan(k, e), O.make_opts(eps=0.02, confidence=0.95, seed=9, growth=0.1, **kw))
    check_run(S, O, r, orr)
    assert r.windows == orr.windows and r.converged == orr.converged == 1 and rc == S.SGPM_OK
    assert r.eps_hat <= 0.02
    S.sgpm_pattern_free(p)


@pytest.mark.parametrize("name,seed", [("triangle", 3), ("4-cycle", 4), ("diamond", 5)])
def test_windows_queued_ahead_keep_the_stop_rule(S, O, synth, ctx, cl_graph, name, seed):
    """Many short windows: after each window whose error predicts two more, the
    library queues the window after next on a second stream.  The stop point,
    window count and exact sums must still be the oracle's (a window queued
    past the stop is dropped)."""
    g, og = cl_graph
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    kw = dict(n_min=2000, w_min=2000, quantum=100)
    opts = S.sgpm_options_default(eps=0.01, confidence=0.95, seed=seed, checksum=1, lanes_per_sample=64,
                                  window_growth=0.0, **kw)
    r, rc = S.sgpm_estimate(ctx, g, p, opts)
    orr = O.run(og, O.compile_plan(k, e), O.make_opts(eps=0.01, confidence=0.95, seed=seed, growth=0.0, **kw))
    check_run(S, O, r, orr)
    assert r.windows == orr.windows and r.windows >= 4 and r.converged == orr.converged
    S.sgpm_pattern_free(p)


def test_not_converged_is_reported(S, O, synth, ctx, cl_graph):
    g, og = cl_graph
    k, e = synth.pattern("5-clique")
    p = S.sgpm_pattern_create(ctx, k, e)
    opts = S.sgpm_options_default(eps=1e-6, seed=2, n_min=10000, w_min=10000, quantum=100, max_samples=35000,
                                  checksum=1)
    r, rc = S.sgpm_estimate(ctx, g, p, opts)
    assert rc == S.SGPM_NOT_CONVERGED and r.converged == 0
    orr = O.run(og, O.compile_plan(k, e), O.make_opts(eps=1e-6, seed=2, n_min=10000, w_min=10000, quantum=100,
                                                       max_samples=35000))
    check_run(S, O, r, orr)
    S.sgpm_pattern_free(p)


def test_empty_graph_and_edge_pattern(S, O, synth, ctx):
    g, og = load(S, O, synth, ctx, 5, np.zeros((0, 2), dtype=np.int32))
    k, e = synth.pattern("triangle")
    p = S.sgpm_pattern_create(ctx, k, e)
    r, rc = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default())
    assert rc == S.SGPM_OK and r.estimate == 0.0 and r.converged == 1 and r.n_samples == 0
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)
    g, og = load(S, O, synth, ctx, 40, synth.er_pairs(40, 100, 2))
    k, e = synth.pattern("edge")
    p = S.sgpm_pattern_create(ctx, k, e)
    r, rc = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(n_min=1000, quantum=1))
    assert rc == S.SGPM_OK and r.estimate == 100.0 and r.eps_hat == 0.0 and r.windows == 1
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)


def test_errors(S, ctx, synth):
    with pytest.raises(S.SgpmError) as ei:
        S.sgpm_pattern_create(ctx, 4, [(0, 1), (2, 3)])
    assert ei.value.status == S.SGPM_EUNSUPPORTED
    off, nbr = synth.pairs_to_csr(10, synth.ring_pairs(10))
    nbr = nbr.copy()
    nbr[0] = 99
    with pytest.raises(S.SgpmError) as ei:
        S.sgpm_graph_from_csr(ctx, 10, off, nbr)
    assert ei.value.status == S.SGPM_EBADGRAPH


@pytest.fixture(scope="module")
def c2(S, O, synth, ctx):
    """R-MAT scale 20, edge factor 16, (a, b, c) = (0.57, 0.19, 0.19), seed 1."""
    print("building C2 R-MAT scale 20", flush=True)
    pairs = synth.rmat_pairs(20, 16, seed=1)
    g, og = load(S, O, synth, ctx, 1 << 20, pairs)
    yield g, og
    S.sgpm_graph_free(g)


@pytest.mark.parametrize("name,seed", [("4-clique", 3), ("5-clique", 4)])
def test_c2_strict_run_matches_oracle(S, O, synth, ctx, c2, name, seed):
    """Full-size R-MAT-20 at the benchmark's options (strict, eps 1 %, 95 %,
    default windows, autotuned lanes: the clique kernel the benchmark times,
    which has no trace path): stop point, windows, exact sums, hits and the
    checksum over every sample equal the oracle's run."""
    print(f"C2 strict {name}", flush=True)
    g, og = c2
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    so = S.sgpm_options_default(eps=0.01, confidence=0.95, seed=seed, checksum=1)
    r, rc = S.sgpm_estimate(ctx, g, p, so)
    orr = O.run(og, O.compile_plan(k, e), O.make_opts(eps=so.eps, confidence=so.confidence, seed=so.seed,
                                                       tag=so.query_tag, n_min=so.n_min, w_min=so.w_min,
                                                       quantum=so.quantum, max_samples=so.max_samples,
                                                       growth=so.window_growth))
    check_run(S, O, r, orr)
    assert r.windows == orr.windows and r.converged == orr.converged == 1 and rc == S.SGPM_OK
    S.sgpm_pattern_free(p)


@pytest.mark.parametrize("name", ["4-clique", "5-clique"])
def test_c2_sampled_walks(S, O, synth, ctx, c2, name):
    """Full-size R-MAT-20 in the benchmark's launch configuration (autotuned
    lanes): walks of sampled id ranges equal the oracle's, one by one."""
    print(f"C2 {name}", flush=True)
    g, og = c2
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    op = O.compile_plan(k, e)
    N = 1 << 21
    buf = S.trace_buffer(N)
    opts = S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=1, lanes_per_sample=0,
                                  trace_lo=0, trace_hi=N, trace_buf=addr(buf))
    r, _ = S.sgpm_estimate(ctx, g, p, opts)
    rng = np.random.default_rng(0)
    picks = np.unique(np.concatenate([np.arange(2048), rng.integers(0, N, 4000), np.arange(N - 2048, N)]))
    hits = 0
    for s in picks.tolist():
        b = O.sample(og, op, 1, 0, s)
        a = buf[s]
        st = 0xFF if b.hit else b.fail_step
        assert (a.s, a.status, list(a.v), a.alpha) == (b.s, st, list(b.v), b.alpha), s
        hits += b.hit
    # the traced records reproduce the run's exact sums
    rec = np.frombuffer(buf, dtype=TRACE_DTYPE)
    assert np.array_equal(rec["s"], np.arange(N, dtype=np.uint64))
    def exact_sum(x):
        return int((x & 0xFFFFFFFF).sum(dtype=np.uint64)) + (int((x >> 32).sum(dtype=np.uint64)) << 32)

    S1 = exact_sum(rec["alo"]) + (exact_sum(rec["ahi"]) << 64)
    assert S1 == r.S1 and int((rec["status"] == 0xFF).sum()) == r.n_hits
    assert hits > 0
    S.sgpm_pattern_free(p)
