"""Pins for the oracle's exact counters: closed forms on structured graphs and
degree / common-neighbour identities computed with independent numpy algebra."""
import itertools
import math

import numpy as np
import pytest


def count(O, synth, n, pairs, name, induced=False):
    k, e = synth.pattern(name)
    g = O.OGraph.from_pairs(n, pairs)
    return O.plan_count(g, O.compile_plan(k, e, induced))


def kn_count(n, k, aut):
    return math.factorial(n) // math.factorial(n - k) // aut


@pytest.mark.parametrize("n", [5, 7, 9])
def test_complete_graph(O, synth, n):
    pairs = synth.complete_pairs(n)
    for kk, name in [(3, "triangle"), (4, "4-clique"), (5, "5-clique")]:
        assert count(O, synth, n, pairs, name) == math.comb(n, kk)
    assert count(O, synth, n, pairs, "4-cycle") == 3 * math.comb(n, 4)
    assert count(O, synth, n, pairs, "diamond") == 6 * math.comb(n, 4)
    assert count(O, synth, n, pairs, "5-cycle") == 12 * math.comb(n, 5)
    assert count(O, synth, n, pairs, "house") == kn_count(n, 5, 2)
    assert count(O, synth, n, pairs, "tailed-triangle") == kn_count(n, 4, 2)
    assert count(O, synth, n, pairs, "3-star") == kn_count(n, 4, 6)
    # induced non-cliques never occur in K_n
    for name in ["4-cycle", "diamond", "4-path", "3-star", "tailed-triangle", "wedge"]:
        assert count(O, synth, n, pairs, name, induced=True) == 0
    assert count(O, synth, n, pairs, "4-clique", induced=True) == math.comb(n, 4)


def test_complete_graph_six_clique(O, synth):
    assert count(O, synth, 9, synth.complete_pairs(9), "6-clique") == math.comb(9, 6)


@pytest.mark.parametrize("n", [4, 5, 6, 9])
def test_ring(O, synth, n):
    pairs = synth.ring_pairs(n)
    assert count(O, synth, n, pairs, "triangle") == 0
    assert count(O, synth, n, pairs, "4-cycle") == (1 if n == 4 else 0)
    assert count(O, synth, n, pairs, "5-cycle") == (1 if n == 5 else 0)
    assert count(O, synth, n, pairs, "wedge") == n
    # a k-vertex path in C_n (k <= n) is C_n minus a run of n - k + 1 edges: n of them
    assert count(O, synth, n, pairs, "4-path") == (n if n >= 4 else 0)
    assert count(O, synth, n, pairs, "5-path") == (n if n >= 5 else 0)


@pytest.mark.parametrize("a,b", [(2, 2), (3, 4), (5, 6)])
def test_grid(O, synth, a, b):
    pairs = synth.grid_pairs(a, b)
    assert count(O, synth, a * b, pairs, "4-cycle") == (a - 1) * (b - 1)
    assert count(O, synth, a * b, pairs, "triangle") == 0


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_hypercube(O, synth, d):
    assert count(O, synth, 1 << d, synth.hypercube_pairs(d), "4-cycle") == math.comb(d, 2) * 2 ** (d - 2)


@pytest.mark.parametrize("a,b", [(2, 3), (3, 4), (4, 6)])
def test_complete_bipartite(O, synth, a, b):
    assert count(O, synth, a + b, synth.complete_bipartite_pairs(a, b), "4-cycle") == math.comb(a, 2) * math.comb(b, 2)
    assert count(O, synth, a + b, synth.complete_bipartite_pairs(a, b), "triangle") == 0


def test_petersen(O, synth):
    p = synth.petersen_pairs()
    assert count(O, synth, 10, p, "triangle") == 0
    assert count(O, synth, 10, p, "4-cycle") == 0
    assert count(O, synth, 10, p, "5-cycle") == 12


@pytest.mark.parametrize("t", [3, 5, 8])
def test_star(O, synth, t):
    p = synth.star_pairs(t)
    assert count(O, synth, t + 1, p, "wedge") == math.comb(t, 2)
    assert count(O, synth, t + 1, p, "3-star") == math.comb(t, 3)
    assert count(O, synth, t + 1, p, "triangle") == 0


def _adj(n, pairs):
    A = np.zeros((n, n), dtype=np.int64)
    for u, v in np.asarray(pairs).reshape(-1, 2):
        if u != v:
            A[u, v] = A[v, u] = 1
    return A


@pytest.mark.parametrize("seed", [1, 2])
def test_degree_identities(O, synth, seed):
    n = 60
    pairs = synth.chung_lu_pairs(n, 10, 2.3, seed)
    A = _adj(n, pairs)
    d = A.sum(1)
    A2 = A @ A
    A3 = A2 @ A
    T = int(np.trace(A3)) // 6
    tv = np.diag(A3) // 2
    E = [(u, v) for u in range(n) for v in range(u + 1, n) if A[u, v]]
    wedges = int(sum(math.comb(int(x), 2) for x in d))
    stars = int(sum(math.comb(int(x), 3) for x in d))
    p4 = int(sum((d[u] - 1) * (d[v] - 1) for u, v in E)) - 3 * T
    tt = int(sum(int(tv[v]) * (int(d[v]) - 2) for v in range(n)))
    dia = int(sum(math.comb(int(A2[u, v]), 2) for u, v in E))
    c4 = sum(math.comb(int(A2[u, w]), 2) for u in range(n) for w in range(u + 1, n)) // 2
    assert count(O, synth, n, pairs, "triangle") == T
    assert count(O, synth, n, pairs, "wedge") == wedges
    assert count(O, synth, n, pairs, "3-star") == stars
    assert count(O, synth, n, pairs, "4-path") == p4
    assert count(O, synth, n, pairs, "tailed-triangle") == tt
    assert count(O, synth, n, pairs, "diamond") == dia
    assert count(O, synth, n, pairs, "4-cycle") == c4
    # induced <-> non-induced relations among the six connected 4-vertex graphs
    I = {nm: count(O, synth, n, pairs, nm, induced=True)
         for nm in ["3-star", "4-path", "tailed-triangle", "4-cycle", "diamond", "4-clique"]}
    K4 = I["4-clique"]
    assert count(O, synth, n, pairs, "4-clique") == K4
    assert dia == I["diamond"] + 6 * K4
    assert c4 == I["4-cycle"] + I["diamond"] + 3 * K4
    assert tt == I["tailed-triangle"] + 4 * I["diamond"] + 12 * K4
    assert p4 == I["4-path"] + 2 * I["tailed-triangle"] + 4 * I["4-cycle"] + 6 * I["diamond"] + 12 * K4
    assert stars == I["3-star"] + I["tailed-triangle"] + 2 * I["diamond"] + 4 * K4


def test_all_graphs_on_five_vertices(O, synth):
    """Every labelled graph on 5 vertices: plan counter equals brute force."""
    n = 5
    slots = list(itertools.combinations(range(n), 2))
    names = ["triangle", "wedge", "4-clique", "4-cycle", "4-path", "3-star", "tailed-triangle", "diamond",
             "5-cycle", "house"]
    plans = {}
    for nm in names:
        k, e = synth.pattern(nm)
        plans[nm] = (k, e, O.compile_plan(k, e, False), O.compile_plan(k, e, True))
    for mask in range(1 << len(slots)):
        pairs = np.array([slots[i] for i in range(len(slots)) if mask >> i & 1], dtype=np.int32).reshape(-1, 2)
        g = O.OGraph.from_pairs(n, pairs)
        for nm, (k, e, pe, pi) in plans.items():
            assert O.plan_count(g, pe, 1) == O.brute_count(g, k, e, False)[1]
            assert O.plan_count(g, pi, 1) == O.brute_count(g, k, e, True)[1]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_graphs_vs_brute_force(O, synth, seed):
    n = 12
    g = O.OGraph.from_pairs(n, synth.er_pairs(n, 30, seed))
    for nm in ["5-clique", "5-cycle", "house", "5-path", "4-clique", "diamond"]:
        k, e = synth.pattern(nm)
        for induced in (False, True):
            assert O.plan_count(g, O.compile_plan(k, e, induced), 2) == O.brute_count(g, k, e, induced)[1]
