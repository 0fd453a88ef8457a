"""GS engine on the GPU against the oracle: colour and Bernoulli edge sparsification (bit-exact
sparsified CSR), the plan-driven exact count (bit-exact counts) and the GS
estimate over repeated colourings (identical per-colouring counts and sums)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NAMES = ["edge", "triangle", "wedge", "4-clique", "5-clique", "4-cycle", "5-cycle", "4-path", "3-star",
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


def load(S, O, synth, ctx, n, pairs):
    off, nbr = synth.pairs_to_csr(n, pairs)
    return S.sgpm_graph_from_csr(ctx, n, off, nbr), O.OGraph.from_raw_csr(n, off, nbr)


@pytest.fixture(scope="module")
def cl(S, O, synth, ctx):
    print("building Chung-Lu(4000, 14, 2.1)", flush=True)
    g, og = load(S, O, synth, ctx, 4000, synth.chung_lu_pairs(4000, 14, 2.1, 6))
    yield g, og
    S.sgpm_graph_free(g)


@pytest.mark.parametrize("c,seed,rep", [(1, 3, 0), (2, 3, 0), (4, 3, 1), (8, 99, 7), (256, 5, 2)])
def test_sparsify_matches_oracle(S, O, ctx, cl, c, seed, rep):
    g, og = cl
    sp = S.sgpm_gs_sparsify(ctx, g, c, seed, rep)
    off, nbr = S.sgpm_graph_export(ctx, sp)
    n, m, maxdeg, _ = S.sgpm_graph_stats(sp)
    col = np.array([O.gs_colour(seed, rep, c, v) for v in range(og.n)], dtype=np.int32)
    osp = O.gs_sparsify(og, col)
    assert m == osp.m and np.array_equal(off, osp.off) and np.array_equal(nbr, osp.nbr)
    assert maxdeg == (int(np.diff(osp.off).max()) if osp.n else 0)
    S.sgpm_graph_free(sp)


@pytest.fixture(scope="module")
def cl_small(S, O, synth, ctx):
    g, og = load(S, O, synth, ctx, 1500, synth.chung_lu_pairs(1500, 10, 2.1, 6))
    yield g, og
    S.sgpm_graph_free(g)


@pytest.fixture(scope="module")
def er_small(S, O, synth, ctx):
    g, og = load(S, O, synth, ctx, 400, synth.er_pairs(400, 3000, 6))
    yield g, og
    S.sgpm_graph_free(g)


@pytest.mark.parametrize("induced", [False, True])
@pytest.mark.parametrize("name", NAMES)
def test_exact_count_matches_oracle(S, O, synth, ctx, cl_small, er_small, name, induced):
    """Every pattern on a small power-law graph (the 6-vertex dumbbell, whose
    edge-induced count is large there, on a small ER graph)."""
    print(f"exact {name} induced={induced}", flush=True)
    g, og = er_small if name == "dumbbell" else cl_small
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e, induced)
    want = O.plan_count(og, O.compile_plan(k, e, induced))
    assert S.sgpm_exact_count(ctx, g, p) == want
    S.sgpm_pattern_free(p)


def test_exact_count_closed_forms(S, O, synth, ctx):
    import math
    g, _ = load(S, O, synth, ctx, 12, synth.complete_pairs(12))
    for kk, name in [(3, "triangle"), (4, "4-clique"), (5, "5-clique"), (6, "6-clique")]:
        p = S.sgpm_pattern_create(ctx, *synth.pattern(name))
        assert S.sgpm_exact_count(ctx, g, p) == math.comb(12, kk)
        S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)
    g, _ = load(S, O, synth, ctx, 1 << 6, synth.hypercube_pairs(6))
    p = S.sgpm_pattern_create(ctx, *synth.pattern("4-cycle"))
    assert S.sgpm_exact_count(ctx, g, p) == math.comb(6, 2) * 2 ** 4
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)
    g, _ = load(S, O, synth, ctx, 5, np.zeros((0, 2), dtype=np.int32))
    p = S.sgpm_pattern_create(ctx, *synth.pattern("triangle"))
    assert S.sgpm_exact_count(ctx, g, p) == 0
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)


@pytest.mark.parametrize("kk", [4, 5, 6])
def test_exact_clique_dense_neighbourhoods(S, O, synth, ctx, kk):
    """Cliques where the common lower neighbourhood of an edge passes 64 (the
    first bitmap pass's list, counted by 128-member bitmaps) or 128 (the second
    pass's list, counted by the general search), next to edges where it does
    not: K_90, and K_140 (K_132 for the 6-clique, whose general search grows
    fast), against C(n, k); a dense core (100 vertices, edge probability 0.7)
    inside a power-law graph against the oracle."""
    import math
    print(f"dense clique k={kk}", flush=True)
    k, e = synth.pattern(f"{kk}-clique")
    p = S.sgpm_pattern_create(ctx, k, e)
    for n in (90, 132 if kk == 6 else 140):
        g, _ = load(S, O, synth, ctx, n, synth.complete_pairs(n))
        assert S.sgpm_exact_count(ctx, g, p) == math.comb(n, kk)
        S.sgpm_graph_free(g)
    rng = np.random.default_rng(31)
    core = synth.complete_pairs(100)
    core = core[rng.random(len(core)) < 0.7]
    n = 3000
    pairs = np.concatenate([core, synth.chung_lu_pairs(n, 8, 2.1, 7)])
    g, og = load(S, O, synth, ctx, n, pairs)
    assert S.sgpm_exact_count(ctx, g, p) == O.plan_count(og, O.compile_plan(k, e))
    S.sgpm_graph_free(g)
    S.sgpm_pattern_free(p)


@pytest.mark.parametrize("induced", [False, True])
def test_exact_diamond_by_edge_pairs(S, O, synth, ctx, induced):
    """The diamond counted as pairs of common neighbours per edge (less 6 per
    4-clique when vertex-induced): K_90 against 6 C(90, 4) and 0, and a dense
    core inside a power-law graph (4-cliques through the overflow list)
    against the oracle's search."""
    import math
    print(f"diamond induced={induced}", flush=True)
    k, e = synth.pattern("diamond")
    p = S.sgpm_pattern_create(ctx, k, e, induced)
    g, _ = load(S, O, synth, ctx, 90, synth.complete_pairs(90))
    assert S.sgpm_exact_count(ctx, g, p) == (0 if induced else 6 * math.comb(90, 4))
    S.sgpm_graph_free(g)
    rng = np.random.default_rng(31)
    core = synth.complete_pairs(100)
    core = core[rng.random(len(core)) < 0.7]
    pairs = np.concatenate([core, synth.chung_lu_pairs(3000, 8, 2.1, 7)])
    g, og = load(S, O, synth, ctx, 3000, pairs)
    assert S.sgpm_exact_count(ctx, g, p) == O.plan_count(og, O.compile_plan(k, e, induced))
    S.sgpm_graph_free(g)
    S.sgpm_pattern_free(p)


@pytest.mark.parametrize("induced", [False, True])
def test_closed_forms_at_wave_width(S, O, synth, ctx, induced):
    """The per-edge closed forms at 64 lanes per edge (a graph of mean degree
    16 or more: ER(400, 4000)) against the oracle's search, for the wedge,
    3-star, 4-path, tailed triangle and diamond, and the vertex-induced 4-path
    and 4-cycle through the 4-cycles' search."""
    print(f"closed forms 64 lanes induced={induced}", flush=True)
    g, og = load(S, O, synth, ctx, 400, synth.er_pairs(400, 4000, 9))
    assert 2 * S.sgpm_graph_stats(g)[1] >= 16 * 400
    for name in ["wedge", "3-star", "4-path", "tailed-triangle", "diamond", "4-cycle"]:
        k, e = synth.pattern(name)
        p = S.sgpm_pattern_create(ctx, k, e, induced)
        assert S.sgpm_exact_count(ctx, g, p) == O.plan_count(og, O.compile_plan(k, e, induced)), name
        S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)


def test_closed_forms_degenerate_graphs(S, O, synth, ctx):
    """Degree-1 endpoints, edges without common neighbours and graphs without
    edges: a star K_{1,50} (C(50, 3) 3-stars and C(50, 2) wedges, edge- and
    vertex-induced, and nothing else), one edge, and 20 isolated vertices; the
    clique bitmaps on the same graphs (no cliques)."""
    import math
    star = np.array([(0, i) for i in range(1, 51)], dtype=np.int32)
    want_star = {"wedge": math.comb(50, 2), "3-star": math.comb(50, 3), "4-path": 0, "tailed-triangle": 0,
                 "diamond": 0, "4-cycle": 0, "4-clique": 0, "5-clique": 0, "6-clique": 0}
    for n, pairs, want in [(51, star, want_star), (2, np.array([(0, 1)], dtype=np.int32), None),
                           (20, np.zeros((0, 2), dtype=np.int32), None)]:
        g, _ = load(S, O, synth, ctx, n, pairs)
        for name in want_star:
            for induced in (False, True):
                p = S.sgpm_pattern_create(ctx, *synth.pattern(name), induced)
                got = S.sgpm_exact_count(ctx, g, p)
                assert got == (want[name] if want else 0), (n, name, induced, got)
                S.sgpm_pattern_free(p)
        S.sgpm_graph_free(g)


@pytest.mark.parametrize("name,c", [("triangle", 4), ("4-cycle", 3), ("diamond", 2)])
def test_gs_estimate_matches_oracle(S, O, synth, ctx, cl, name, c):
    g, og = cl
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    opts = S.sgpm_options_default(mode=S.MODE_GS, colours=c, seed=17, eps=0.05, gs_reps_max=40)
    r, rc = S.sgpm_estimate(ctx, g, p, opts)
    orr, ys = O.gs_run(og, O.compile_plan(k, e), c, 17, eps=0.05, confidence=0.95, reps_max=40)
    assert r.scheme == S.SCHEME_GS and r.colours == c
    assert r.n_samples == orr.reps and r.S1 == orr.S1 and r.S2 == orr.S2
    assert r.estimate == orr.estimate
    # the t quantile is computed by different methods on the two sides and may
    # round one unit in the last place apart
    assert r.eps_hat == pytest.approx(orr.eps_hat, rel=1e-15, abs=0) and r.z == pytest.approx(orr.z, rel=1e-15)
    assert r.converged == orr.converged
    assert (rc == S.SGPM_OK) == bool(orr.converged)
    S.sgpm_pattern_free(p)


@pytest.fixture(scope="module")
def rmat13(S, O, synth, ctx):
    print("building R-MAT scale 13", flush=True)
    g, og = load(S, O, synth, ctx, 1 << 13, synth.rmat_pairs(13, 16, seed=2))
    yield g, og
    S.sgpm_graph_free(g)


@pytest.mark.parametrize("name", ["triangle", "4-clique", "5-clique", "diamond", "4-cycle"])
def test_exact_count_rmat13(S, O, synth, ctx, rmat13, name):
    """Skewed R-MAT degrees (hub rows spanning many 64-entry chunks)."""
    g, og = rmat13
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    want = O.plan_count(og, O.compile_plan(k, e))
    assert S.sgpm_exact_count(ctx, g, p) == want
    S.sgpm_pattern_free(p)


@pytest.mark.parametrize("name,c", [("triangle", 1), ("4-clique", 1), ("4-cycle", 2)])
def test_gs_estimate_rmat13_matches_oracle(S, O, synth, ctx, rmat13, name, c):
    """GS on R-MAT (hub rows) against the oracle: per-colouring counts of a
    sparse triangle and 4-clique search take 8 and 16 lanes per first edge,
    the 4-cycle the whole wave."""
    g, og = rmat13
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    opts = S.sgpm_options_default(mode=S.MODE_GS, colours=c, seed=23, eps=0.02, gs_reps_max=4)
    r, rc = S.sgpm_estimate(ctx, g, p, opts)
    orr, ys = O.gs_run(og, O.compile_plan(k, e), c, 23, eps=0.02, confidence=0.95, reps_max=4)
    assert r.n_samples == orr.reps and r.S1 == orr.S1 and r.S2 == orr.S2
    assert r.estimate == orr.estimate and r.converged == orr.converged
    S.sgpm_pattern_free(p)


_want = {}


@pytest.mark.parametrize("group", ["8", "16", "64"])
@pytest.mark.parametrize("name", ["triangle", "4-clique", "5-clique", "diamond", "4-cycle"])
def test_exact_count_every_group_width(S, O, synth, ctx, cl_small, rmat13, monkeypatch, name, group):
    """Each lane-group width of the count (8, 16 or 64 lanes per first edge,
    forced) gives the oracle's count, on a power-law graph and on R-MAT (hub
    rows spanning many group-wide windows)."""
    monkeypatch.setenv("SGPM_EXACT_GROUP", group)
    print(f"exact {name} group={group}", flush=True)
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    for gname, (g, og) in (("cl", cl_small), ("rmat13", rmat13)):
        if (gname, name) not in _want:
            _want[(gname, name)] = O.plan_count(og, O.compile_plan(k, e))
        assert S.sgpm_exact_count(ctx, g, p) == _want[(gname, name)]
    S.sgpm_pattern_free(p)


def test_sparsified_graph_supports_ns(S, O, synth, ctx, cl):
    """NS on a sparsified handle equals the oracle's NS on its sparsified graph."""
    g, og = cl
    sp = S.sgpm_gs_sparsify(ctx, g, 2, 11, 0)
    col = np.array([O.gs_colour(11, 0, 2, v) for v in range(og.n)], dtype=np.int32)
    osp = O.gs_sparsify(og, col)
    k, e = synth.pattern("triangle")
    p = S.sgpm_pattern_create(ctx, k, e)
    r, _ = S.sgpm_estimate(ctx, sp, p, S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=100000, seed=4,
                                                               checksum=1))
    orr = O.run(osp, O.compile_plan(k, e), O.make_opts(fixed_n=100000, seed=4))
    assert r.S1 == orr.S1 and r.checksum == orr.checksum
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(sp)


# ------------------------------------------------------------------ Bernoulli edge sparsification
@pytest.mark.parametrize("c,seed,rep", [(1, 3, 0), (2, 3, 0), (3, 8, 1), (16, 99, 7), (256, 5, 2)])
def test_bes_sparsify_matches_oracle(S, O, ctx, cl, c, seed, rep):
    g, og = cl
    sp = S.sgpm_bes_sparsify(ctx, g, c, seed, rep)
    off, nbr = S.sgpm_graph_export(ctx, sp)
    n, m, maxdeg, _ = S.sgpm_graph_stats(sp)
    osp = O.bes_sparsify(og, c, seed, rep)
    assert m == osp.m and np.array_equal(off, osp.off) and np.array_equal(nbr, osp.nbr)
    assert maxdeg == (int(np.diff(osp.off).max()) if osp.m else 0)
    S.sgpm_graph_free(sp)


@pytest.mark.parametrize("name,c", [("triangle", 2), ("4-cycle", 2), ("diamond", 2), ("tailed-triangle", 3)])
def test_bes_estimate_matches_oracle(S, O, synth, ctx, cl, name, c):
    g, og = cl
    k, e = synth.pattern(name)
    p = S.sgpm_pattern_create(ctx, k, e)
    opts = S.sgpm_options_default(mode=S.MODE_GS, gs_scheme=S.GS_BERNOULLI, colours=c, seed=23, eps=0.05,
                                  gs_reps_max=30)
    r, rc = S.sgpm_estimate(ctx, g, p, opts)
    orr, ys = O.bes_run(og, O.compile_plan(k, e), c, 23, eps=0.05, confidence=0.95, reps_max=30)
    assert r.scheme == S.SCHEME_GS and r.colours == c
    assert r.n_samples == orr.reps and r.S1 == orr.S1 and r.S2 == orr.S2
    assert r.estimate == orr.estimate and r.converged == orr.converged
    assert r.eps_hat == pytest.approx(orr.eps_hat, rel=1e-15, abs=0)
    S.sgpm_pattern_free(p)


def test_bes_refuses_what_it_cannot_estimate(S, O, synth, ctx, cl):
    g, og = cl
    k, e = synth.pattern("4-cycle")
    p = S.sgpm_pattern_create(ctx, k, e, True)  # vertex-induced: non-edges are not preserved
    with pytest.raises(S.SgpmError):
        S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_GS, gs_scheme=S.GS_BERNOULLI, colours=2))
    S.sgpm_pattern_free(p)
    k, e = synth.pattern("triangle")
    p = S.sgpm_pattern_create(ctx, k, e)
    for kw in (dict(mode=S.MODE_STRICT_NS), dict(mode=S.MODE_HYBRID), dict(gs_scheme=5)):
        with pytest.raises(S.SgpmError):
            S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(**{"gs_scheme": S.GS_BERNOULLI, **kw}))
    S.sgpm_pattern_free(p)


def test_colour_choice(S, O, synth, ctx, cl):
    """colours = 0: the library probes one colouring at 16 colours (repetition
    0x3FFFFFFF), chooses c from its leaves by the rule sgpm_host_colours_choice
    states, and the estimate equals the GS run at that c."""
    g, og = cl
    for name in ["triangle", "4-clique", "diamond"]:
        k, e = synth.pattern(name)
        p = S.sgpm_pattern_create(ctx, k, e)
        sp = S.sgpm_gs_sparsify(ctx, g, 16, 23, 0x3FFFFFFF)
        y16 = S.sgpm_exact_count(ctx, sp, p)
        S.sgpm_graph_free(sp)
        assert y16 == O.gs_count(og, O.compile_plan(k, e), 16, 23, 0x3FFFFFFF)
        want = S.sgpm_host_colours_choice(og.m, k, float(y16))
        assert 4 <= want <= 16
        r, rc = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_GS, colours=0, seed=23, eps=0.05,
                                                                   gs_reps_max=20))
        assert r.colours == want
        r2, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_GS, colours=want, seed=23, eps=0.05,
                                                                    gs_reps_max=20))
        assert (r.n_samples, r.S1, r.S2, r.estimate) == (r2.n_samples, r2.S1, r2.S2, r2.estimate)
        S.sgpm_pattern_free(p)
    p = S.sgpm_pattern_create(ctx, *synth.pattern("triangle"))
    for bad in (-1, 257):
        for mode in (S.MODE_GS, S.MODE_HYBRID):
            with pytest.raises(S.SgpmError) as ei:
                S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=mode, colours=bad))
            assert ei.value.status == S.SGPM_EINVAL
    S.sgpm_pattern_free(p)
