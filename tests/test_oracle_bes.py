"""Pins for the oracle's Bernoulli edge sparsification (BES), the second GS
scheme (Sec. 2.2, the edge-sparsification algorithm; the GS trade-off section).

- Exact expectation over every edge subset of a small graph, in exact
  rationals: sum over subsets of Pr(subset) * count(subset) * c^l equals the
  count, with l the number of pattern EDGES (colour sparsification scales by
  c^(k-1) instead; the two agree only for trees, and the test checks that the
  other exponent fails for every pattern with a cycle).
- The keep decision is per undirected edge (the same from both ends), the
  sparsified graph is a subgraph of G, and the kept fraction concentrates at 1/c.
- c = 1 keeps every edge: each repetition is the exact count, zero variance.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest


@pytest.mark.parametrize("name", ["triangle", "4-cycle", "diamond", "wedge"])
def test_exact_expectation_over_edge_subsets(O, synth, name):
    k, e = synth.pattern(name)
    p = O.compile_plan(k, e)
    l = O.plan_edges(p)
    assert l == len(e)
    n = 6
    pairs = synth.er_pairs(n, 9, 5)
    want = O.plan_count(O.OGraph.from_pairs(n, pairs), p)
    assert want > 0
    m = len(pairs)
    counts = {}
    for keep in itertools.product((0, 1), repeat=m):
        sub = [pairs[i] for i in range(m) if keep[i]]
        counts[keep] = O.plan_count(O.OGraph.from_pairs(n, np.array(sub, dtype=np.int32).reshape(-1, 2)), p, 1) \
            if sub else 0
    for c in (2, 3):
        q = Fraction(1, c)
        total = sum((q ** sum(kp) * (1 - q) ** (m - sum(kp)) * cnt for kp, cnt in counts.items() if cnt),
                    Fraction(0))
        assert total * c ** l == want
        if l != k - 1:
            assert total * c ** (k - 1) != want


def test_keep_is_per_edge_and_sparsified_graph_is_a_subgraph(O, synth):
    n = 2000
    g = O.OGraph.from_pairs(n, synth.er_pairs(n, 20000, 3))
    off, nbr = g.off, g.nbr
    for c in (2, 5):
        sp = O.bes_sparsify(g, c, 17, 4)
        soff, snbr = sp.off, sp.nbr
        kept = 0
        for u in range(0, n, 7):
            row = set(nbr[off[u]:off[u + 1]].tolist())
            srow = snbr[soff[u]:soff[u + 1]].tolist()
            assert set(srow) <= row
            for w in row:
                assert O.bes_keep(17, 4, c, u, w) == O.bes_keep(17, 4, c, w, u) == (w in srow)
        assert sp.m * 2 == len(snbr)
        frac = sp.m / g.m
        sd = np.sqrt((1 / c) * (1 - 1 / c) / g.m)
        assert abs(frac - 1 / c) < 6 * sd


def test_c1_is_exact(O, synth):
    g = O.OGraph.from_pairs(200, synth.er_pairs(200, 1500, 8))
    k, e = synth.pattern("diamond")
    p = O.compile_plan(k, e)
    want = O.plan_count(g, p)
    r, ys = O.bes_run(g, p, 1, 3, eps=0.01, reps_max=5)
    # c = 1 keeps every edge: each repetition is exact and the rule stops at its third
    assert ys == [want] * 3 and r.reps == 3 and r.converged == 1 and r.estimate == want
