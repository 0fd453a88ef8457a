"""The allocation-free exact count (sgpm_exact_count_noalloc, scratch in the
library's fixed device array) against sgpm_exact_count through the C ABI: the
same count on every path the count takes (clique bitmaps with and without the
overflow list, the general search at each width, and cliques on a graph whose
first edges outnumber the array's list, which the allocation-free call counts
by the general search), over consecutive calls whose inputs shrink."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PATTERNS = ["triangle", "4-clique", "5-clique", "6-clique", "diamond", "4-cycle"]


@pytest.fixture(scope="module")
def S():
    from paper_2405_03488_amd import sgpm
    return sgpm


@pytest.fixture(scope="module")
def ctx(S):
    c = S.sgpm_create(0)
    yield c
    S.sgpm_destroy(c)


def load(S, synth, ctx, n, pairs):
    off, nbr = synth.pairs_to_csr(n, pairs)
    return S.sgpm_graph_from_csr(ctx, n, off, nbr)


def dense_core(synth, n, core, prob, seed):
    rng = np.random.default_rng(seed)
    cp = synth.complete_pairs(core)
    cp = cp[rng.random(len(cp)) < prob]
    return np.concatenate([cp, synth.chung_lu_pairs(n, 8, 2.1, seed)])


def both(S, synth, ctx, g, name):
    p = S.sgpm_pattern_create(ctx, *synth.pattern(name))
    a = S.sgpm_exact_count_noalloc(ctx, g, p)
    b = S.sgpm_exact_count(ctx, g, p)
    S.sgpm_pattern_free(p)
    return a, b


def test_noalloc_equals_exact_count_shrinking_inputs(S, synth, ctx):
    # first call: a dense core (first edges past 64 candidates go to the list)
    # in a power-law graph; second: K_90 (smaller); third: a small ER graph
    graphs = [("core", 3000, dense_core(synth, 3000, 110, 0.75, 5)),
              ("K90", 90, synth.complete_pairs(90)),
              ("er", 400, synth.er_pairs(400, 3000, 6))]
    for label, n, pairs in graphs:
        g = load(S, synth, ctx, n, pairs)
        for name in PATTERNS:
            print(f"noalloc {label} {name}", flush=True)
            a, b = both(S, synth, ctx, g, name)
            assert a == b, (label, name, a, b)
            if label == "K90" and name.endswith("clique"):
                assert a == math.comb(90, int(name[0]))
        S.sgpm_graph_free(g)


def test_noalloc_past_the_overflow_list(S, synth, ctx):
    """R-MAT 18 (about 4M first edges, more than the array's 2^21-entry list):
    the allocation-free call counts cliques by the general search, the other
    by bitmaps (the diamond by edge pairs on both); then a smaller graph on the
    same array."""
    n = 1 << 18
    print("noalloc rmat18", flush=True)
    g = load(S, synth, ctx, n, synth.rmat_pairs(18, 16, seed=3))
    assert S.sgpm_graph_stats(g)[1] > (1 << 21)
    for name in ["4-clique", "triangle", "diamond"]:
        print(f"noalloc rmat18 {name}", flush=True)
        a, b = both(S, synth, ctx, g, name)
        assert a == b, (name, a, b)
    S.sgpm_graph_free(g)
    g = load(S, synth, ctx, 1500, synth.chung_lu_pairs(1500, 10, 2.1, 6))
    for name in ["4-clique", "diamond"]:
        a, b = both(S, synth, ctx, g, name)
        assert a == b, (name, a, b)
    S.sgpm_graph_free(g)


def test_noalloc_rejects_null_arguments(S, synth, ctx):
    import ctypes as C
    g = load(S, synth, ctx, 90, synth.complete_pairs(90))
    p = S.sgpm_pattern_create(ctx, *synth.pattern("4-clique"))
    lo = C.c_uint64()
    assert S.lib().sgpm_exact_count_noalloc(ctx, g, p, None, None) == S.SGPM_EINVAL
    assert S.lib().sgpm_exact_count_noalloc(ctx, None, p, C.byref(lo), None) == S.SGPM_EINVAL
    assert S.lib().sgpm_exact_count_noalloc(ctx, g, p, C.byref(lo), None) == S.SGPM_OK
    assert lo.value == math.comb(90, 4)
    S.sgpm_pattern_free(p)
    S.sgpm_graph_free(g)
