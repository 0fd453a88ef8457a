"""Pins for the oracle's NS-base sampler (lazy verification), the sampler the
paper measures NS-prune against (Sec. 4.2 and the evaluation's hit-rate and
convergence comparisons).

- The candidate set of a step is the UNION of the neighbourhoods of the earlier
  positions joined to it by a pattern edge: its members, as a set, equal the
  union computed with Python sets, each once.
- Unbiasedness: the exact expectation over every random walk, in exact
  rationals, equals the brute-force count, for edge- and vertex-induced
  patterns (a dropped closure test or a wrong alpha breaks it).
- Complete graph K_n: every union is the whole vertex set, so a triangle is hit
  with probability C(n,3) / (m n) = (n-2)/(3n) and a 4-clique with
  C(n,4) / (m n^2); NS-prune's hit probabilities differ (1 - 2/n for the
  triangle), which separates the two samplers.
- Misses: an empty union ends the walk at its position, a failed closure check
  reports position k with every vertex drawn; X = 0 on a miss.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

NAMES = ["triangle", "wedge", "4-clique", "4-cycle", "4-path", "3-star", "tailed-triangle", "diamond", "house"]


def nbrs(off, nbr, u):
    return set(int(x) for x in nbr[off[u]:off[u + 1]])


@pytest.mark.parametrize("name", ["diamond", "4-clique", "4-cycle", "house"])
def test_candidates_are_the_union_of_joined_rows(O, synth, name):
    k, e = synth.pattern(name)
    p = O.compile_plan(k, e)
    g = O.OGraph.from_pairs(60, synth.er_pairs(60, 400, 3))
    off, nbr = g.off, g.nbr
    checked = 0
    for s in range(200):
        r = O.sample_base(g, p, 5, 0, s)
        reached = r.k if (r.hit or r.fail_step == r.k) else r.fail_step
        for j in range(2, reached):
            rows = [i for i in range(j) if p.connect[j] >> i & 1]
            want = set()
            for i in rows:
                want |= nbrs(off, nbr, r.v[i])
            got = O.union_candidates(g, p, j, [r.v[i] for i in range(j)])
            assert len(got) == len(set(got.tolist())) == len(want) == r.size[j]
            assert set(got.tolist()) == want
            checked += 1
    assert checked > 100


@pytest.mark.parametrize("induced", [False, True])
@pytest.mark.parametrize("name", NAMES)
def test_exact_expectation_equals_count(O, synth, name, induced):
    k, e = synth.pattern(name)
    p = O.compile_plan(k, e, induced)
    for seed in (31, 32):
        n = 7
        g = O.OGraph.from_pairs(n, synth.er_pairs(n, 12, seed))
        want = O.brute_count(g, k, e, induced)[1]
        assert O.exact_expectation(g, p, base=True) == Fraction(want)


@pytest.mark.parametrize("n", [4, 5, 6])
def test_hit_probability_on_complete_graph(O, synth, n):
    g = O.OGraph.from_pairs(n, synth.complete_pairs(n))
    m = n * (n - 1) // 2
    k, e = synth.pattern("triangle")
    p = O.compile_plan(k, e)
    ex, hit = O.exact_expectation(g, p, base=True, with_hit_prob=True)
    assert ex == math.comb(n, 3)
    assert hit == Fraction(n - 2, 3 * n) == Fraction(math.comb(n, 3), m * n)
    _, hit_prune = O.exact_expectation(g, p, with_hit_prob=True)
    assert hit_prune == 1 - Fraction(2, n) != hit
    k, e = synth.pattern("4-clique")
    p = O.compile_plan(k, e)
    ex, hit = O.exact_expectation(g, p, base=True, with_hit_prob=True)
    assert ex == math.comb(n, 4)
    assert hit == Fraction(math.comb(n, 4), m * n * n)


def test_miss_records(O, synth):
    g = O.OGraph.from_pairs(24, synth.er_pairs(24, 180, 9))
    k, e = synth.pattern("4-clique")
    p = O.compile_plan(k, e)
    kinds = set()
    for s in range(2000):
        r = O.sample_base(g, p, 3, 0, s)
        if r.hit:
            assert r.alpha == int(r.size[0]) * int(r.size[2]) * int(r.size[3])
            kinds.add("hit")
        else:
            assert r.alpha == 0 and 2 <= r.fail_step <= r.k
            if r.fail_step == r.k:
                assert all(r.v[i] >= 0 for i in range(r.k))
                kinds.add("closure")
            else:
                assert r.size[r.fail_step] == 0 and r.v[r.fail_step] == -1
    assert {"hit", "closure"} <= kinds


def test_trace_and_run_agree_with_samples(O, synth):
    g = O.OGraph.from_pairs(300, synth.er_pairs(300, 3000, 4))
    k, e = synth.pattern("diamond")
    p = O.compile_plan(k, e)
    recs = O.trace_base(g, p, 11, 2, 1000, 400, threads=3)
    S1 = S2 = 0
    csum = 0
    for i, r in enumerate(recs):
        one = O.sample_base(g, p, 11, 2, 1000 + i)
        assert (r.hit, r.fail_step, r.alpha, list(r.v)) == (one.hit, one.fail_step, one.alpha, list(one.v))
    opts = O.make_opts(fixed_n=5000, seed=11, tag=2, sampler=1, threads=3)
    res = O.run(g, p, opts)
    for r in O.trace_base(g, p, 11, 2, 0, 5000, threads=2):
        S1 += r.alpha
        S2 += r.alpha * r.alpha
        csum = (csum + O.rec_hash(r)) % (1 << 64)
    assert (res.S1, res.S2, res.checksum, res.n) == (S1, S2, csum, 5000)
    # lazy verification hits less often than NS-prune on the same walks' graph
    pr = O.run(g, p, O.make_opts(fixed_n=5000, seed=11, tag=2, threads=3))
    assert res.hits < pr.hits
