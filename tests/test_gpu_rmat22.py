"""The large-graph sampling path (the 5-clique on a power-law R-MAT graph held
in HBM, uniform and learned proposal) against the oracle at R-MAT scale 22
(4.2M vertices, edge factor 16): sampled walks one by one, and the exact sums
and checksum of runs in the launch configuration the estimates use."""
import ctypes as C

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


@pytest.fixture(scope="module")
def rmat22(S, O, synth, ctx):
    print("building R-MAT scale 22", flush=True)
    n = 1 << 22
    off, nbr = synth.pairs_to_csr(n, synth.rmat_pairs(22, 16, seed=1))
    g = S.sgpm_graph_from_csr(ctx, n, off, nbr)
    print("oracle graph", flush=True)
    og = O.OGraph.from_raw_csr(n, off, nbr)
    yield g, og
    S.sgpm_graph_free(g)


def addr(buf):
    return C.cast(buf, C.c_void_p).value


def picks(N, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.arange(1024), rng.integers(0, N, 3000), np.arange(N - 1024, N)])).tolist()


@pytest.mark.parametrize("name", ["5-clique", "4-clique"])
def test_rmat22_uniform(S, O, synth, ctx, rmat22, name):
    g, og = rmat22
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    op = O.compile_plan(k, e)
    N = 1 << 20
    buf = S.trace_buffer(N)
    r, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=3, query_tag=1,
                                                             trace_lo=0, trace_hi=N, trace_buf=addr(buf)))
    hits = 0
    for s in picks(N, 1):
        b = O.sample(og, op, 3, 1, s)
        a = buf[s]
        st = 0xFF if b.hit else b.fail_step
        assert (a.s, a.status, list(a.v), a.alpha) == (b.s, st, list(b.v), b.alpha), s
        hits += b.hit
    assert hits > 100
    # the untraced run (clique kernel, autotuned lanes) over every sample
    print(f"oracle run {name}", flush=True)
    orr = O.run(og, op, O.make_opts(fixed_n=N, seed=3, tag=1))
    r, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=3, query_tag=1,
                                                             checksum=1))
    assert (r.S1, r.S2, r.n_hits, r.checksum) == (orr.S1, orr.S2, orr.hits, orr.checksum)
    assert r.estimate == orr.estimate
    S.sgpm_pattern_free(p)


def test_rmat22_learned(S, O, synth, ctx, rmat22):
    g, og = rmat22
    k, e = synth.pattern("5-clique")
    p = S.sgpm_pattern_create(ctx, k, e)
    op = O.compile_plan(k, e)
    table = np.random.default_rng(11).integers(1, 65536, size=(8, 32, 32, 32)).astype(np.uint16)
    model = S.sgpm_model_from_tables(ctx, [p], table)
    N = 1 << 18
    buf = S.trace_buffer(N)
    S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=5, proposal=model.value,
                                                      trace_lo=0, trace_hi=N, trace_buf=addr(buf)))
    hits = 0
    for s in picks(N, 2):
        b, _ = O.sample_learned(og, op, table, 5, 0, s)
        a = buf[s]
        st = 0xFF if b.hit else b.fail_step
        assert (a.s, a.status, list(a.v), a.alpha) == (b.s, st, list(b.v), b.alpha), s
        hits += b.hit
    assert hits > 100
    # untraced (the learned clique kernel) over every sample of a shorter run
    M = 1 << 13
    print("oracle learned sums", flush=True)
    S1 = S2 = nh = cs = 0
    for s in range(M):
        b, _ = O.sample_learned(og, op, table, 5, 0, s)
        S1 += b.alpha
        S2 += b.alpha * b.alpha
        nh += b.hit
        cs = (cs + O.rec_hash(b)) % (1 << 64)
    r, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=M, seed=5, checksum=1,
                                                             proposal=model.value))
    assert (r.S1, r.S2, r.n_hits, r.checksum) == (S1, S2, nh, cs)
    S.sgpm_model_free(model)
    S.sgpm_pattern_free(p)
