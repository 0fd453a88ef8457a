"""Pins for the oracle's NS-prune sampler.

- Unbiasedness lemma (Sec. 4.2): the exact expectation over every random walk,
  in exact rationals, equals the brute-force count, for edge- and
  vertex-induced patterns.
- The paper's 4-cycle algorithm (Sec. 4.2) retraced by hand with Python sets.
- k = 2: every sample is M, so the estimator has zero variance.
- Misses carry X = 0 and a fail step; random draws average to the count.
"""
from fractions import Fraction

import numpy as np
import pytest

NAMES = ["triangle", "wedge", "4-clique", "4-cycle", "4-path", "3-star", "tailed-triangle", "diamond",
         "5-cycle", "house", "5-clique"]


@pytest.mark.parametrize("induced", [False, True])
@pytest.mark.parametrize("name", NAMES)
def test_exact_expectation_equals_count(O, synth, name, induced):
    k, e = synth.pattern(name)
    p = O.compile_plan(k, e, induced)
    for seed in (21, 22):
        n = 7
        g = O.OGraph.from_pairs(n, synth.er_pairs(n, 13, seed))
        want = O.brute_count(g, k, e, induced)[1]
        assert O.exact_expectation(g, p) == Fraction(want)


def test_exact_expectation_complete_graph(O, synth):
    import math
    g = O.OGraph.from_pairs(6, synth.complete_pairs(6))
    for name in ["4-clique", "4-cycle", "diamond", "5-clique"]:
        k, e = synth.pattern(name)
        assert O.exact_expectation(g, O.compile_plan(k, e)) == Fraction(O.plan_count(g, O.compile_plan(k, e)))
    k, e = synth.pattern("4-clique")
    assert O.exact_expectation(g, O.compile_plan(k, e)) == math.comb(6, 4)


def _r_for(i, N):
    return -((-i << 64) // N)


def test_paper_four_cycle_hand_trace(O, synth):
    """Retrace the paper's NS-prune 4-cycle algorithm with Python sets:
    (v0, v1) an edge with v1 < v0; A = N(v1) - {v0, v1}, members < v0;
    B = N(v0) & N(v2), members < v1; X = m |A| |B|."""
    pairs = np.array([[0, 1], [1, 2], [2, 3], [3, 0], [0, 2], [3, 4], [4, 1], [4, 2]], dtype=np.int32)
    g = O.OGraph.from_pairs(5, pairs)
    off, nbr = g.off, g.nbr
    N = {u: set(nbr[off[u]:off[u + 1]].tolist()) for u in range(5)}
    edges = list(zip(g.esrc.tolist(), g.edst.tolist()))
    m = g.m
    k, e = synth.pattern("4-cycle")
    p = O.compile_plan(k, e)
    checked = 0
    for ei, (v0, v1) in enumerate(edges):
        A = sorted(x for x in N[v1] - {v0, v1} if x < v0)
        rec = O.sample(g, p, 0, 0, 0, [_r_for(ei, m), 0, 0, 0])
        assert (rec.v[0], rec.v[1]) == (v0, v1)
        if not A:
            assert not rec.hit and rec.fail_step == 2 and rec.alpha == 0
            continue
        for ai, v2 in enumerate(A):
            B = sorted(x for x in (N[v0] & N[v2]) - {v0, v1, v2} if x < v1)
            if not B:
                rec = O.sample(g, p, 0, 0, 0, [_r_for(ei, m), 0, _r_for(ai, len(A)), 0])
                assert not rec.hit and rec.fail_step == 3 and rec.v[2] == v2
                continue
            for bi, v3 in enumerate(B):
                rec = O.sample(g, p, 0, 0, 0, [_r_for(ei, m), 0, _r_for(ai, len(A)), _r_for(bi, len(B))])
                assert rec.hit
                assert list(rec.v)[:4] == [v0, v1, v2, v3]
                assert rec.alpha == m * len(A) * len(B)
                checked += 1
    assert checked > 0


def test_k2_zero_variance(O, synth):
    g = O.OGraph.from_pairs(50, synth.er_pairs(50, 200, 1))
    k, e = synth.pattern("edge")
    p = O.compile_plan(k, e)
    opts = O.make_opts(eps=0.01, n_min=1000, w_min=1000, quantum=1)
    r = O.run(g, p, opts)
    assert r.converged == 1 and r.windows == 1 and r.eps_hat == 0.0
    assert r.estimate == g.m
    assert r.S1 == r.n * g.m and r.S2 == r.n * g.m * g.m


def test_miss_records(O, synth):
    g = O.OGraph.from_pairs(40, synth.er_pairs(40, 60, 3))
    k, e = synth.pattern("5-clique")
    p = O.compile_plan(k, e)
    recs = O.trace(g, p, 7, 0, 0, 500, 1)
    misses = [r for r in recs if not r.hit]
    assert misses
    for r in misses:
        assert r.alpha == 0 and 2 <= r.fail_step < k and r.size[r.fail_step] == 0
        assert all(r.v[i] >= 0 for i in range(r.fail_step))
    for r in recs:
        assert r.s == recs[0].s + (r.s - recs[0].s)


def test_sampler_mean_matches_count(O, synth):
    n = 300
    g = O.OGraph.from_pairs(n, synth.er_pairs(n, 3000, 4))
    for name in ["triangle", "4-cycle", "wedge"]:
        k, e = synth.pattern(name)
        p = O.compile_plan(k, e)
        C = O.plan_count(g, p)
        r = O.run(g, p, O.make_opts(fixed_n=400000, seed=5))
        # 6 sigma from the run's own standard error
        sigma = r.estimate * r.eps_hat / r.z
        assert abs(r.estimate - C) < 6 * sigma, (name, r.estimate, C)


def test_trace_equals_sample(O, synth):
    g = O.OGraph.from_pairs(100, synth.er_pairs(100, 600, 8))
    k, e = synth.pattern("diamond")
    p = O.compile_plan(k, e)
    recs = O.trace(g, p, 11, 3, 1000, 64, 3)
    for i, r in enumerate(recs):
        one = O.sample(g, p, 11, 3, 1000 + i)
        assert bytes(r) == bytes(one)
