"""Persistent batched estimation: every query's result equals the oracle's run
and its solo run bit for bit (samples drawn, exact sums, hits, checksum,
windows, stop point), the device's stop test agrees with the host arithmetic,
and replays of the captured hipGraph with new seeds stay equal to solo runs."""
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


def graph_inputs(synth):
    for n, pairs in [(3000, synth.chung_lu_pairs(3000, 12, 2.1, 1)), (1 << 14, synth.rmat_pairs(14, 16, seed=3)),
                     (5000, synth.er_pairs(5000, 40000, 2))]:
        yield n, synth.pairs_to_csr(n, pairs)


@pytest.fixture(scope="module")
def graphs(S, synth, ctx):
    print("building batch graphs", flush=True)
    out = [S.sgpm_graph_from_csr(ctx, n, off, nbr) for n, (off, nbr) in graph_inputs(synth)]
    yield out
    for g in out:
        S.sgpm_graph_free(g)


@pytest.fixture(scope="module")
def ographs(O, synth):
    return [O.OGraph.from_raw_csr(n, off, nbr) for n, (off, nbr) in graph_inputs(synth)]


def same(a, b):
    assert a.n_samples == b.n_samples
    assert a.S1 == b.S1 and a.S2 == b.S2
    assert a.n_hits == b.n_hits and a.checksum == b.checksum
    assert a.windows == b.windows and a.converged == b.converged
    assert a.estimate == b.estimate and a.eps_hat == b.eps_hat


MOTIFS = [("3-star", True), ("4-path", True), ("tailed-triangle", True), ("4-cycle", True), ("diamond", True),
          ("4-clique", True), ("wedge", True), ("triangle", False)]


def make_queries(S, synth, ctx, graphs, seed0):
    qs = []
    for gi, g in enumerate(graphs):
        for pi, (name, induced) in enumerate(MOTIFS):
            k, e = synth.pattern(name)
            p = S.sgpm_pattern_create(ctx, k, e, induced)
            i = len(qs)
            if i % 5 == 4:
                o = S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=123457 + i, seed=seed0 + i, checksum=1)
            else:
                o = S.sgpm_options_default(eps=0.03, seed=seed0 + i, query_tag=i, n_min=1 << 16, w_min=1 << 15,
                                           quantum=1 << 12, checksum=1, max_samples=1 << 24)
            qs.append((g, p, o))
    return qs


def test_batch_equals_solo(S, synth, ctx, graphs):
    qs = make_queries(S, synth, ctx, graphs, 100)
    res = S.sgpm_estimate_batch(ctx, [q[0] for q in qs], [q[1] for q in qs], [q[2] for q in qs])
    assert len(res) == 24
    for (g, p, o), rb in zip(qs, res):
        rs, _ = S.sgpm_estimate(ctx, g, p, o)
        same(rb, rs)
        assert rb.tile >= 16 and rb.tile & (rb.tile - 1) == 0
    for q in qs:
        S.sgpm_pattern_free(q[1])


def check_against_oracle(S, O, synth, ographs, qs, res):
    i = 0
    for og in ographs:
        for name, induced in MOTIFS:
            g, p, o = qs[i]
            rb = res[i]
            op = O.compile_plan(*synth.pattern(name), induced)
            if o.mode == S.MODE_FIXED_N:
                oo = O.make_opts(fixed_n=o.fixed_n, seed=o.seed, tag=o.query_tag)
            else:
                oo = O.make_opts(eps=o.eps, confidence=o.confidence, seed=o.seed, tag=o.query_tag, n_min=o.n_min,
                                 w_min=o.w_min, quantum=o.quantum, max_samples=o.max_samples,
                                 growth=o.window_growth)
            orr = O.run(og, op, oo)
            print(f"query {i} {name} lanes={rb.lanes_per_sample} tile={rb.tile} n={orr.n}", flush=True)
            assert rb.n_samples == orr.n and rb.windows == orr.windows and rb.converged == orr.converged
            assert rb.S1 == orr.S1 and rb.S2 == orr.S2 and rb.n_hits == orr.hits and rb.checksum == orr.checksum
            assert rb.estimate == orr.estimate
            assert rb.eps_hat == orr.eps_hat or (rb.eps_hat == float("inf") and orr.eps_hat == float("inf"))
            i += 1


def test_batch_equals_oracle(S, O, synth, ctx, graphs, ographs):
    """Every query of the persistent batch (strict queries with their own
    windows and device-side stop test, fixed-n queries) against the oracle's
    run at the same options: stop point, windows, exact sums, hits, checksum,
    estimate and predicted error."""
    qs = make_queries(S, synth, ctx, graphs, 100)
    res = S.sgpm_estimate_batch(ctx, [q[0] for q in qs], [q[1] for q in qs], [q[2] for q in qs])
    check_against_oracle(S, O, synth, ographs, qs, res)
    for q in qs:
        S.sgpm_pattern_free(q[1])


@pytest.mark.parametrize("lanes", [(1, 4, 16, 64), (16, 4), (1,)])
def test_batch_lane_groups_equal_oracle(S, O, synth, ctx, graphs, ographs, lanes):
    """Queries pinned to 1, 4, 16 or 64 lanes per sample (the build with the
    lane-group samplers; strict and fixed-n, ragged last tiles) against the
    oracle, and each query reports the lane count it ran."""
    qs = make_queries(S, synth, ctx, graphs, 700)
    for i, (_, _, o) in enumerate(qs):
        o.lanes_per_sample = lanes[i % len(lanes)]
    res = S.sgpm_estimate_batch(ctx, [q[0] for q in qs], [q[1] for q in qs], [q[2] for q in qs])
    for (_, _, o), rb in zip(qs, res):
        assert rb.lanes_per_sample == o.lanes_per_sample
        assert rb.tile % (64 // rb.lanes_per_sample) == 0
    check_against_oracle(S, O, synth, ographs, qs, res)
    for q in qs:
        S.sgpm_pattern_free(q[1])


def test_batch_autotuned_lanes(S, synth, ctx, graphs):
    """lanes_per_sample = 0: the autotuner picks each query's lane count from
    timed pilots (a count the solo estimate chose is reused); every result
    still equals its solo run at the lane count the solo run picks."""
    qs = make_queries(S, synth, ctx, graphs, 1300)
    res = S.sgpm_estimate_batch(ctx, [q[0] for q in qs], [q[1] for q in qs], [q[2] for q in qs])
    picked = [rb.lanes_per_sample for rb in res]
    print("batch lanes picked:", picked, flush=True)
    assert all(l in (1, 4, 16, 64) for l in picked)
    for (g, p, o), rb in zip(qs, res):
        rs, _ = S.sgpm_estimate(ctx, g, p, o)
        same(rb, rs)
    for q in qs:
        S.sgpm_pattern_free(q[1])


def test_batch_rejects_bad_lanes(S, synth, ctx, graphs):
    k, e = synth.pattern("triangle")
    p = S.sgpm_pattern_create(ctx, k, e)
    o = S.sgpm_options_default(eps=0.05, lanes_per_sample=8)
    with pytest.raises(S.SgpmError) as ei:
        S.sgpm_estimate_batch(ctx, [graphs[0]], [p], [o])
    assert ei.value.status == S.SGPM_EINVAL
    S.sgpm_pattern_free(p)


def test_batch_replay_new_seeds(S, synth, ctx, graphs):
    """The second and third calls with the same shape replay the captured graph."""
    for seed0 in (500, 900):
        qs = make_queries(S, synth, ctx, graphs, seed0)
        res = S.sgpm_estimate_batch(ctx, [q[0] for q in qs], [q[1] for q in qs], [q[2] for q in qs])
        for (g, p, o), rb in zip(qs, res):
            rs, _ = S.sgpm_estimate(ctx, g, p, o)
            same(rb, rs)
        for q in qs:
            S.sgpm_pattern_free(q[1])


def test_batch_single_and_empty(S, O, synth, ctx, graphs):
    off, nbr = synth.pairs_to_csr(7, synth.ring_pairs(7)[:0])
    empty = S.sgpm_graph_from_csr(ctx, 7, off, nbr)
    k, e = synth.pattern("triangle")
    p = S.sgpm_pattern_create(ctx, k, e)
    o = S.sgpm_options_default(eps=0.05, seed=3, n_min=1 << 14, w_min=1 << 14, quantum=1, checksum=1)
    res = S.sgpm_estimate_batch(ctx, [empty, graphs[0]], [p, p], [o, o])
    assert res[0].estimate == 0.0 and res[0].n_samples == 0 and res[0].converged == 1
    rs, _ = S.sgpm_estimate(ctx, graphs[0], p, o)
    same(res[1], rs)
    res = S.sgpm_estimate_batch(ctx, [graphs[2]], [p], [o])
    rs, _ = S.sgpm_estimate(ctx, graphs[2], p, o)
    same(res[0], rs)
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(empty)


def test_batch_rejects_unsupported(S, synth, ctx, graphs):
    k, e = synth.pattern("triangle")
    p = S.sgpm_pattern_create(ctx, k, e)
    o = S.sgpm_options_default(mode=S.MODE_GS)
    with pytest.raises(S.SgpmError) as ei:
        S.sgpm_estimate_batch(ctx, [graphs[0]], [p], [o])
    assert ei.value.status == S.SGPM_EUNSUPPORTED
    S.sgpm_pattern_free(p)


def test_batch_motifs_on_power_law_graph(S, synth, ctx):
    """The batched motif set at the scale of the smallest motif-batch graph
    (Chung-Lu, 2^18 vertices, average degree 32, gamma 2.1): hubs of ~1e5
    neighbours, vertex-induced patterns; every query equals its solo run."""
    n = 1 << 18
    print("building Chung-Lu 2^18", flush=True)
    off, nbr = synth.pairs_to_csr(n, synth.chung_lu_pairs(n, 32, 2.1, 18))
    g = S.sgpm_graph_from_csr(ctx, n, off, nbr)
    qs = []
    for i, (name, induced) in enumerate(MOTIFS):
        k, e = synth.pattern(name)
        p = S.sgpm_pattern_create(ctx, k, e, induced)
        o = S.sgpm_options_default(eps=0.05, seed=40 + i, query_tag=i, checksum=1, max_samples=1 << 24)
        qs.append((g, p, o))
    res = S.sgpm_estimate_batch(ctx, [q[0] for q in qs], [q[1] for q in qs], [q[2] for q in qs])
    for (g_, p, o), rb in zip(qs, res):
        rs, _ = S.sgpm_estimate(ctx, g_, p, o)
        same(rb, rs)
    for q in qs:
        S.sgpm_pattern_free(q[1])
    S.sgpm_graph_free(g)
