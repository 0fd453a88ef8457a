"""Pins for the oracle's colour-sparsification path (Sec. 2.2 subgraph
sampling, Sec. 5.2): over every colouring of a tiny graph the mean of
c^(k-1) * Y equals the exact count, and the variance equals
C (c^(k-1) - 1) + sum_z t_z (c^(z-1) - 1) with t_z the ordered pairs of distinct
matches sharing z vertices; c = 1 is exact."""
import itertools
from fractions import Fraction

import numpy as np
import pytest


def _matches(n, A, k, edges):
    """Occurrences as (vertex frozenset, edge frozenset), edge-induced."""
    occ = set()
    for phi in itertools.permutations(range(n), k):
        if all(A[phi[a]][phi[b]] for a, b in edges):
            es = frozenset(frozenset((phi[a], phi[b])) for a, b in edges)
            occ.add((frozenset(phi), es))
    return list(occ)


@pytest.mark.parametrize("name,c", [("triangle", 2), ("triangle", 3), ("4-cycle", 2), ("wedge", 3),
                                    ("diamond", 2), ("4-clique", 2)])
def test_exhaustive_colourings(O, synth, name, c):
    n = 7 if c == 2 else 6
    pairs = synth.er_pairs(n, 12, 31)
    g = O.OGraph.from_pairs(n, pairs)
    off, nbr = g.off, g.nbr
    A = [[False] * n for _ in range(n)]
    for u in range(n):
        for w in nbr[off[u]:off[u + 1]]:
            A[u][w] = True
    k, e = synth.pattern(name)
    p = O.compile_plan(k, e)
    C = O.plan_count(g, p)
    occ = _matches(n, A, k, e.tolist())
    assert len(occ) == C
    vals = []
    for col in itertools.product(range(c), repeat=n):
        sp = O.gs_sparsify(g, np.array(col, dtype=np.int32))
        vals.append(c ** (k - 1) * O.plan_count(sp, p, 1))
    mean = Fraction(sum(vals), len(vals))
    assert mean == C
    var = Fraction(sum(v * v for v in vals), len(vals)) - mean * mean
    tz = {}
    for a in range(len(occ)):
        for b in range(len(occ)):
            if a != b:
                z = len(occ[a][0] & occ[b][0])
                tz[z] = tz.get(z, 0) + 1
    want = C * (c ** (k - 1) - 1) + sum(t * (Fraction(c) ** (z - 1) - 1) for z, t in tz.items() if z >= 1)
    assert var == want


def test_single_colour_is_exact(O, synth):
    g = O.OGraph.from_pairs(200, synth.er_pairs(200, 1500, 2))
    for name in ["triangle", "4-cycle", "diamond"]:
        k, e = synth.pattern(name)
        p = O.compile_plan(k, e)
        assert O.gs_count(g, p, 1, 9, 0) == O.plan_count(g, p)


def test_sparsified_graph_keeps_monochromatic_edges(O, synth):
    n = 300
    g = O.OGraph.from_pairs(n, synth.er_pairs(n, 2000, 3))
    col = np.array([O.gs_colour(77, 2, 5, v) for v in range(n)], dtype=np.int32)
    assert col.min() >= 0 and col.max() < 5
    sp = O.gs_sparsify(g, col)
    off, nbr, so, sn = g.off, g.nbr, sp.off, sp.nbr
    for u in range(n):
        want = [w for w in nbr[off[u]:off[u + 1]].tolist() if col[w] == col[u]]
        assert sn[so[u]:so[u + 1]].tolist() == want


def test_colour_uniformity(O):
    c = 8
    cnt = np.bincount([O.gs_colour(5, 0, c, v) for v in range(40000)], minlength=c)
    chi2 = float(((cnt - 5000) ** 2 / 5000).sum())
    assert chi2 < 30.0
