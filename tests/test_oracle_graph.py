"""Pins for the oracle's canonical graph: invariants that any correct
symmetrise / dedupe / degree-descending relabel must satisfy, checked with
independent numpy code."""
import numpy as np
import pytest


def _expected_edges(n, pairs):
    """Set of undirected edges (original ids) after symmetrising and dropping loops/dups."""
    p = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    p = p[p[:, 0] != p[:, 1]]
    lo = np.minimum(p[:, 0], p[:, 1])
    hi = np.maximum(p[:, 0], p[:, 1])
    return set(zip(lo.tolist(), hi.tolist()))


def _check(O, n, pairs):
    g = O.OGraph.from_pairs(n, pairs)
    off, nbr, perm = g.off, g.nbr, g.perm
    assert g.n == n
    assert off[0] == 0 and off[-1] == 2 * g.m
    assert np.all(np.diff(off) >= 0)
    # permutation
    assert sorted(perm.tolist()) == list(range(n))
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    # rows strictly ascending, no loops, symmetric
    arcs = set()
    for u in range(n):
        row = nbr[off[u]:off[u + 1]]
        assert np.all(np.diff(row) > 0)
        assert not np.any(row == u)
        for w in row.tolist():
            arcs.add((u, w))
    for (u, w) in arcs:
        assert (w, u) in arcs
    # same edge set up to the relabel
    want = _expected_edges(n, pairs)
    got = set()
    for (u, w) in arcs:
        a, b = int(inv[u]), int(inv[w])
        got.add((min(a, b), max(a, b)))
    assert got == want
    # degree descending, ties by original id ascending
    deg = np.diff(off)
    for r in range(n - 1):
        assert deg[r] > deg[r + 1] or (deg[r] == deg[r + 1] and inv[r] < inv[r + 1])
    # oriented edges: all arcs (u, w) with w < u in (u, w) order
    lower = [(u, w) for u in range(n) for w in nbr[off[u]:off[u + 1]].tolist() if w < u]
    assert list(zip(g.esrc.tolist(), g.edst.tolist())) == lower
    # arc rows
    assert np.array_equal(g.arow, np.repeat(np.arange(n), deg))
    return g


def test_canon_er(O, synth):
    _check(O, 300, synth.er_pairs(300, 1500, 5))


def test_canon_rmat_with_dups_and_loops(O, synth):
    pairs = synth.rmat_pairs(9, 8, seed=3)
    assert np.any(pairs[:, 0] == pairs[:, 1])  # the generator does produce loops
    _check(O, 512, pairs)


def test_canon_chung_lu(O, synth):
    _check(O, 400, synth.chung_lu_pairs(400, 8, 2.1, 4))


def test_canon_isolated_and_empty(O):
    g = _check(O, 6, np.array([[1, 4], [4, 1], [2, 2]], dtype=np.int32))
    assert g.m == 1
    g0 = O.OGraph.from_pairs(4, np.zeros((0, 2), dtype=np.int32))
    assert g0.m == 0 and g0.off.tolist() == [0, 0, 0, 0, 0]


def test_canon_rejects_bad_ids(O):
    with pytest.raises(ValueError):
        O.OGraph.from_raw_csr(3, np.array([0, 1, 1, 1]), np.array([7], dtype=np.int32))
    with pytest.raises(ValueError):
        O.OGraph.from_raw_csr(3, np.array([0, 2, 1, 2]), np.array([1, 2], dtype=np.int32))
