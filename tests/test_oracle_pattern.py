"""Pins for the oracle's pattern compiler: automorphism group sizes from
closed forms, the paper's 4-cycle plan (Sec. 4.2), and the bijection
"restricted tuples x |Aut| = injective homomorphisms" against brute force."""
import itertools
import math

import numpy as np
import pytest

AUT = {"edge": 2, "triangle": 6, "wedge": 2, "4-clique": 24, "5-clique": 120, "6-clique": 720, "4-cycle": 8,
       "5-cycle": 10, "4-path": 2, "5-path": 2, "3-star": 6, "tailed-triangle": 2, "diamond": 4, "house": 2,
       "dumbbell": 8}


@pytest.mark.parametrize("name", sorted(AUT))
def test_aut_sizes(O, synth, name):
    k, e = synth.pattern(name)
    assert O.automorphisms(k, e) == AUT[name]
    assert O.compile_plan(k, e).aut == AUT[name]


def test_paper_four_cycle_plan(O, synth):
    """Sec. 4.2: v0 is the maximum of the four and v3 < v1; A = N(v1) bounded by v0,
    B = N(v0) & N(v2) bounded by v1; first edge from the m edges."""
    k, e = synth.pattern("4-cycle")
    p = O.plan_dict(O.compile_plan(k, e))
    assert p["oriented"] == 1                       # v0 > v1, alpha starts at m
    assert p["connect"][2] == 0b010                 # v2 in N(v1)
    assert p["connect"][3] == 0b101                 # v3 in N(v0) & N(v2)
    assert p["upper"][2] == 0b001                   # v2 < v0
    assert p["upper"][3] == 0b011                   # v3 < v0 and v3 < v1
    assert all(x == 0 for x in p["lower"])


@pytest.mark.parametrize("name", sorted(AUT))
def test_plan_is_a_valid_order(O, synth, name):
    k, e = synth.pattern(name)
    p = O.plan_dict(O.compile_plan(k, e))
    assert sorted(p["order"]) == list(range(k))
    adj = {(a, b) for a, b in e.tolist()} | {(b, a) for a, b in e.tolist()}
    assert (p["order"][0], p["order"][1]) in adj
    for j in range(1, k):
        assert p["connect"][j] != 0
        for i in range(j):
            assert bool(p["connect"][j] >> i & 1) == ((p["order"][i], p["order"][j]) in adj)


def test_compile_rejects(O):
    with pytest.raises(ValueError):
        O.compile_plan(4, [(0, 1), (2, 3)])         # disconnected
    with pytest.raises(ValueError):
        O.compile_plan(9, [(i, i + 1) for i in range(8)])
    with pytest.raises(ValueError):
        O.compile_plan(1, [])


def _inj_homs(adjG, n, k, edges, induced):
    """Independent brute force in Python: injective maps preserving edges (and non-edges)."""
    pe = {(a, b) for a, b in edges} | {(b, a) for a, b in edges}
    cnt = 0
    for phi in itertools.permutations(range(n), k):
        ok = True
        for a in range(k):
            for b in range(a + 1, k):
                e = adjG[phi[a]][phi[b]]
                if (a, b) in pe and not e:
                    ok = False
                    break
                if induced and (a, b) not in pe and e:
                    ok = False
                    break
            if not ok:
                break
        cnt += ok
    return cnt


@pytest.mark.parametrize("induced", [False, True])
@pytest.mark.parametrize("name", ["triangle", "wedge", "4-clique", "4-cycle", "4-path", "3-star",
                                  "tailed-triangle", "diamond", "5-cycle", "house"])
def test_restricted_times_aut_equals_injective(O, synth, name, induced):
    k, e = synth.pattern(name)
    p = O.compile_plan(k, e, induced)
    for seed in range(3):
        n = 8
        pairs = synth.er_pairs(n, 14, seed + 10)
        g = O.OGraph.from_pairs(n, pairs)
        off, nbr = g.off, g.nbr
        adjG = [[False] * n for _ in range(n)]
        for u in range(n):
            for w in nbr[off[u]:off[u + 1]]:
                adjG[u][w] = True
        inj = _inj_homs(adjG, n, k, e.tolist(), induced)
        assert O.plan_count(g, p) * p.aut == inj
        assert O.brute_count(g, k, e, induced) == (inj, inj // p.aut)
