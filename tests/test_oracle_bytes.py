"""Pins for the oracle's measurement definitions.

- Algorithmic bytes of an NS sample: 8 for the first edge, 16 per earlier
  vertex whose row a step reads, and 4 per entry of every row a step merges
  inside the step's symmetry-breaking bounds, up to the first empty step
  (the merge work of the sampler, Sec. 4.3: each sample is a sequence of set
  operations whose cost follows the sizes of the sets).  Recomputed here from
  the trace records with plain Python lists, and against a closed form on K_n.
- The degree bucket floor(log2(1 + deg)) clipped to 31 of the learned proposal.
"""
import math

import numpy as np
import pytest

NAMES = ["triangle", "wedge", "4-clique", "4-cycle", "4-path", "3-star", "tailed-triangle", "diamond",
         "5-cycle", "house", "5-clique", "dumbbell"]


def _bits(mask):
    return [i for i in range(8) if mask >> i & 1]


def _python_bytes(off, nbr, plan, rec):
    """(every-row bytes, smallest-connected-row bytes) of one trace record."""
    k = plan.k
    last = k - 1 if rec.hit else rec.fail_step
    v = list(rec.v)
    total = small_total = 8
    opened = set()
    for j in range(2, last + 1):
        lo, hi = -1, math.inf
        for i in _bits(plan.upper[j]):
            hi = min(hi, v[i])
        for i in _bits(plan.lower[j]):
            lo = max(lo, v[i])
        rows = sorted(set(_bits(plan.connect[j])) | set(_bits(plan.disconnect[j])))
        head = 0
        inside = {}
        for i in rows:
            if i not in opened:
                head += 16
                opened.add(i)
            row = nbr[off[v[i]]:off[v[i] + 1]].tolist()
            inside[i] = 4 * sum(1 for x in row if lo < x < hi)
        total += head + sum(inside.values())
        conn = _bits(plan.connect[j])
        best = min(conn, key=lambda i: (off[v[i] + 1] - off[v[i]], i))
        small_total += head + inside[best]
    return total, small_total


@pytest.mark.parametrize("induced", [False, True])
@pytest.mark.parametrize("name", NAMES)
def test_bytes_recomputed_from_records(O, synth, name, induced):
    n = 400
    g = O.OGraph.from_raw_csr(n, *synth.pairs_to_csr(n, synth.chung_lu_pairs(n, 10, 2.1, 5)))
    k, e = synth.pattern(name)
    p = O.compile_plan(k, e, induced)
    recs = O.trace(g, p, 3, 0, 0, 1500)
    off, nbr = g.off, g.nbr
    ends = set()
    for r in recs:
        want, want_min = _python_bytes(off, nbr, p, r)
        assert (r.bytes, r.bytes_min) == (want, want_min), (r.s, r.hit, r.fail_step)
        assert r.bytes_min <= r.bytes
        ends.add(-1 if r.hit else r.fail_step)
    # hits and misses at some step both occur, so the early-exit rule is exercised
    assert -1 in ends and len(ends) >= 2
    # the run total is the sum of the records
    res = O.run(g, p, O.make_opts(fixed_n=1500, seed=3))
    assert res.bytes == sum(r.bytes for r in recs)


def test_bytes_closed_form_complete_graph(O, synth):
    """Triangle on K_n: the plan orders v0 > v1 > v2, so the one step merges the
    rows of v0 and v1 below v1; each holds exactly v1 such entries (ids 0..v1-1),
    giving 8 + 2 * 16 + 2 * 4 * v1 bytes; the smallest-row figure counts one row."""
    n = 30
    g = O.OGraph.from_pairs(n, synth.complete_pairs(n))
    k, e = synth.pattern("triangle")
    p = O.compile_plan(k, e)
    for r in O.trace(g, p, 11, 0, 0, 300):
        assert r.v[0] > r.v[1]
        # v1 = 0 leaves no candidate below it: a miss at step 2 after the same merge
        assert (r.hit == 1 and r.v[1] > r.v[2]) if r.v[1] > 0 else (r.hit == 0 and r.fail_step == 2)
        assert r.bytes == 40 + 8 * r.v[1]
        assert r.bytes_min == 40 + 4 * r.v[1]


def test_bytes_edge_pattern_is_first_edge_only(O, synth):
    g = O.OGraph.from_pairs(50, synth.er_pairs(50, 200, 4))
    k, e = synth.pattern("edge")
    for r in O.trace(g, O.compile_plan(k, e), 1, 0, 0, 100):
        assert r.bytes == 8 and r.bytes_min == 8


def test_bucket_is_floor_log2_one_plus_degree(O, synth):
    n = 3000
    g = O.OGraph.from_raw_csr(n, *synth.pairs_to_csr(n, synth.chung_lu_pairs(n, 20, 2.1, 9)))
    deg = np.diff(g.off)
    assert deg.max() > 300  # several buckets are populated
    for v in range(n):
        want = min(31, int(deg[v] + 1).bit_length() - 1)
        assert O.bucket(g, v) == want
    # buckets never increase along the degree-descending relabel
    b = [O.bucket(g, v) for v in range(n)]
    assert all(b[i] >= b[i + 1] for i in range(n - 1))


def _python_tree_bytes(g, plan):
    """Algorithmic bytes of the exact search, from the definition: every node
    of the nested loops (a partial match v_0..v_{j-1} at level j) reads 16 per
    row first merged at level j along its path and 4 per entry of each merged
    row inside the level's bounds; 8 per first edge.  Candidates by Python sets."""
    off, nbr = g.off, g.nbr
    rows = {u: set(nbr[off[u]:off[u + 1]].tolist()) for u in range(len(off) - 1)}
    k = plan.k
    first_merge = {}
    for j in range(2, k):
        for i in _bits(plan.connect[j]) + _bits(plan.disconnect[j]):
            first_merge.setdefault(i, j)
            first_merge[i] = min(first_merge[i], j)

    def node(j, v):
        lo, hi = -1, math.inf
        for i in _bits(plan.upper[j]):
            hi = min(hi, v[i])
        for i in _bits(plan.lower[j]):
            lo = max(lo, v[i])
        merged = sorted(set(_bits(plan.connect[j])) | set(_bits(plan.disconnect[j])))
        b = sum(16 for i in merged if first_merge[i] == j)
        b += sum(4 * sum(1 for x in rows[v[i]] if lo < x < hi) for i in merged)
        cand = None
        for i in _bits(plan.connect[j]):
            cand = set(rows[v[i]]) if cand is None else cand & rows[v[i]]
        for i in _bits(plan.disconnect[j]):
            cand -= rows[v[i]]
        cand = sorted(x for x in cand if lo < x < hi and x not in v[:j])
        if j == k - 1:
            return b
        return b + sum(node(j + 1, v[:j] + [x]) for x in cand)

    total = 0
    n = len(off) - 1
    for u in range(n):
        for w in sorted(rows[u]):
            if plan.oriented and not w < u:
                continue
            total += 8
            if k > 2:
                total += node(2, [u, w])
    return total


@pytest.mark.parametrize("induced", [False, True])
@pytest.mark.parametrize("name", ["triangle", "wedge", "4-clique", "4-cycle", "3-star", "diamond", "5-cycle",
                                  "house", "5-clique"])
def test_exact_search_bytes_recomputed(O, synth, name, induced):
    """The exact count's algorithmic bytes (every node of the search tree)
    against the definition recomputed with Python sets."""
    n = 120
    g = O.OGraph.from_raw_csr(n, *synth.pairs_to_csr(n, synth.chung_lu_pairs(n, 8, 2.1, 7)))
    k, e = synth.pattern(name)
    p = O.compile_plan(k, e, induced)
    assert O.plan_count_bytes(g, p, threads=3) == _python_tree_bytes(g, p)


def test_exact_search_bytes_closed_form_complete_graph(O, synth):
    """Triangle on K_n: the first edges are the pairs v0 > v1, each node reads
    both rows below v1 (v1 entries each) after opening them: sum over v1 of
    (n - 1 - v1) * (8 + 32 + 8 v1)."""
    n = 25
    g = O.OGraph.from_pairs(n, synth.complete_pairs(n))
    k, e = synth.pattern("triangle")
    p = O.compile_plan(k, e)
    want = sum((n - 1 - v1) * (8 + 32 + 8 * v1) for v1 in range(n))
    assert O.plan_count_bytes(g, p) == want
