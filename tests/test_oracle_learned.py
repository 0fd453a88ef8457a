"""Pins for the oracle's learned-proposal sampler and MLP reference.

- Importance sampling with any positive weight table is unbiased: the exact
  expectation over all walks (rational walk probabilities, the sampler's FP64
  weights) equals the brute-force count to FP64 accuracy.
- A constant table reduces to uniform selection: every member has probability
  1/|S_j| and alpha' is the uniform NS weight.
- One step retraced by hand on a graph with two candidate buckets.
- BF16 rounding matches torch's bfloat16 conversion; the FP64 backward pass
  matches central finite differences.
"""
from fractions import Fraction

import numpy as np
import pytest


def table(seed, lo=1, hi=65535):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(8, 32, 32, 32), dtype=np.int64).astype(np.uint16)


@pytest.mark.parametrize("name", ["triangle", "4-clique", "4-cycle", "diamond", "tailed-triangle", "5-cycle"])
def test_learned_exact_expectation(O, synth, name):
    k, e = synth.pattern(name)
    p = O.compile_plan(k, e)
    for seed in (1, 2):
        g = O.OGraph.from_pairs(9, synth.chung_lu_pairs(9, 5, 2.1, seed + 40))
        C = O.brute_count(g, k, e)[1]
        ex = O.exact_expectation_learned(g, p, table(seed))
        assert abs(float(ex) - C) <= 1e-12 * max(1, C), (name, float(ex), C)


def test_constant_table_is_uniform(O, synth):
    g = O.OGraph.from_pairs(60, synth.chung_lu_pairs(60, 8, 2.1, 3))
    k, e = synth.pattern("4-clique")
    p = O.compile_plan(k, e)
    t = np.ones((8, 32, 32, 32), dtype=np.uint16) * 7
    for s in range(400):
        r, af = O.sample_learned(g, p, t, 5, 0, s)
        u = O.sample(g, p, 5, 0, s)
        # same first edge; weight = uniform NS weight for the walk actually taken
        assert (r.v[0], r.v[1]) == (u.v[0], u.v[1])
        if r.hit:
            sizes = [int(r.size[j]) for j in range(2, k)]
            want = (g.m if p.oriented else 2 * g.m) * int(np.prod(sizes))
            assert af == float(want) and r.alpha == want << 52


def test_hand_trace_two_buckets(O, synth):
    # v0 = 0 adjacent to a hub (high bucket) and to low-degree vertices
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3)] + [(1, 10 + i) for i in range(20)]
    g = O.OGraph.from_pairs(30, np.array(pairs, dtype=np.int32))
    k, e = synth.pattern("wedge")  # arcs; S_2 = N(v0) minus v1 (wedge centre first)
    p = O.compile_plan(k, e)
    t = np.ones((8, 32, 32, 32), dtype=np.uint16)
    for s in range(300):
        r, af = O.sample_learned(g, p, t, 9, 0, s)
        if not r.hit:
            continue
        cands = O.candidates(g, p, 2, list(r.v)[:2])
        b0, bp = O.bucket(g, r.v[0]), O.bucket(g, r.v[1])
        assert r.v[2] in cands
        assert af == float(2 * g.m * len(cands))
    # the wedge's only step is its last: uniform whatever the table says
    t2 = np.ones((8, 32, 32, 32), dtype=np.uint16)
    t2[:, :, :, 4:] = 1000
    for s in range(300):
        r, af = O.sample_learned(g, p, t2, 9, 0, s)
        if r.hit:
            assert af == float(2 * g.m * len(O.candidates(g, p, 2, list(r.v)[:2])))
    # a 3-star's step 2 is weighted: the low buckets 1000x, factor Sigma / w_b
    # (centre 0: S_2 holds the hub and a low-degree vertex); its last step is
    # uniform, factor |S_3|
    t3 = np.ones((8, 32, 32, 32), dtype=np.uint16)
    t3[:, :, :, :4] = 1000
    k, e = synth.pattern("3-star")
    p = O.compile_plan(k, e)
    M = g.m if p.oriented else 2 * g.m
    seen = 0
    for s in range(4000):
        r, af = O.sample_learned(g, p, t3, 9, 0, s)
        if not r.hit:
            continue
        cands = O.candidates(g, p, 2, list(r.v)[:2])
        ws = [1 if O.bucket(g, x) >= 4 else 1000 for x in cands]
        sigma = sum(ws)
        wb = 1 if O.bucket(g, r.v[2]) >= 4 else 1000
        last = len(O.candidates(g, p, 3, list(r.v)[:3]))
        assert af == float(M) * (sigma / wb) * last
        seen += 1 if len(set(ws)) > 1 else 0
    assert seen > 0


def test_bf16_matches_torch(O):
    import torch
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-5, 5, 2000),
                         [0.0, 1.0, -1.0, 1.00390625, 1.005859375, 3.4e38]]).astype(np.float32)
    want = torch.tensor(xs).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([O.bf16(float(x)) for x in xs])
    assert np.array_equal(got, want)


def test_mlp_backward_finite_differences(O):
    rng = np.random.default_rng(1)
    n = O.mlp_nparams()
    params = (rng.standard_normal(n) * 0.3).astype(np.float32)
    X = rng.standard_normal((16, 16)).astype(np.float32)
    y = rng.standard_normal(16).astype(np.float32)
    loss, _, g = O.mlp(params, X, y, bf16=False, grads=True)
    idx = rng.choice(n, 60, replace=False)
    for i in idx:
        h = 1e-4 * max(1.0, abs(float(params[i])))  # small enough not to cross a ReLU kink
        pp = params.astype(np.float64).copy()
        pm = pp.copy()
        pp[i] += h
        pm[i] -= h
        # evaluate in float64 through float32 params: use a step exactly representable
        fp = O.mlp(pp.astype(np.float32), X, y, bf16=False)[0]
        fm = O.mlp(pm.astype(np.float32), X, y, bf16=False)[0]
        hh = (float(np.float32(pp[i])) - float(np.float32(pm[i]))) / 2
        fd = (fp - fm) / (2 * hh)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_mlp_forward_matches_numpy(O):
    rng = np.random.default_rng(2)
    n = O.mlp_nparams()
    params = (rng.standard_normal(n) * 0.3).astype(np.float32)
    X = rng.standard_normal((32, 16)).astype(np.float32)
    W1 = params[:1024].reshape(16, 64).astype(np.float64)
    b1 = params[1024:1088].astype(np.float64)
    W2 = params[1088:1088 + 4096].reshape(64, 64).astype(np.float64)
    b2 = params[5184:5248].astype(np.float64)
    w3 = params[5248:5312].astype(np.float64)
    b3 = float(params[5312])
    h1 = np.maximum(X.astype(np.float64) @ W1 + b1, 0)
    h2 = np.maximum(h1 @ W2 + b2, 0)
    s = h2 @ w3 + b3
    _, got, _ = O.mlp(params, X, bf16=False)
    assert np.allclose(got, s, rtol=1e-12, atol=1e-12)


# --- the learned table from the network (oracle's orc_learned_table) ---------
# Networks that read chosen features through one hidden unit:
# s = 16 * relu(sum_i w_i x_i + bias), every weight exact in BF16, so each
# cell's score is a small integer and every table entry is a known power of two.

def _reader(O, weights, bias=0.0):
    nh, nin = 64, 16
    P = np.zeros(O.mlp_nparams(), dtype=np.float32)
    W1, b1 = 0, nin * nh
    W2 = b1 + nh
    w3 = W2 + nh * nh + nh
    for i, w in weights.items():
        P[W1 + i * nh + 0] = w
    P[b1 + 0] = bias
    P[W2 + 0 * nh + 0] = 1.0
    P[w3 + 0] = 16.0
    return P


def _quant(scores):
    mx = max(scores)
    return [max(1, min(65535, int(round(2.0 ** (s - mx + 15))))) for s in scores]


def _check_rows(tab, k, score):
    """score(j, b0, bp, bc) -> expected score; rows of steps 2..k-2 only."""
    for j in range(8):
        for b0 in (0, 5, 31):
            for bp in (0, 7, 31):
                row = tab[j, b0, bp]
                if j < 2 or j > k - 2:
                    assert (row == 1).all(), (j, b0, bp)
                    continue
                want = _quant([score(j, b0, bp, bc) for bc in range(32)])
                assert list(row) == want, (j, b0, bp, list(row), want)


def test_table_constant_network(O):
    P = np.zeros(O.mlp_nparams(), dtype=np.float32)
    P[-1] = 3.0  # the output bias only
    for k in (3, 4, 5, 8):
        tab = O.learned_table(P, 0, k)
        _check_rows(tab, k, lambda j, b0, bp, bc: 3.0)


def test_table_reads_the_candidate_bucket(O):
    tab = O.learned_table(_reader(O, {0: 1.0}), 2, 5)
    _check_rows(tab, 5, lambda j, b0, bp, bc: bc)
    # the row maximum holds 2^15, buckets 16 and more below it halve per bucket
    assert tab[2, 3, 4, 31] == 32768 and tab[2, 3, 4, 30] == 16384 and tab[2, 3, 4, 10] == 1


def test_table_reads_bucket_differences(O):
    # candidate minus v_{j-1}: directly, and through the separate features
    for w in ({4: 1.0}, {0: 1.0, 2: -1.0}):
        _check_rows(O.learned_table(_reader(O, w), 0, 6), 6, lambda j, b0, bp, bc: max(0, bc - bp))
    # candidate minus v0
    for w in ({5: 1.0}, {0: 1.0, 1: -1.0}):
        _check_rows(O.learned_table(_reader(O, w), 0, 6), 6, lambda j, b0, bp, bc: max(0, bc - b0))


def test_table_reads_step_and_pattern(O):
    # the step: j/8 weighted 8 with bias -2.5 shifts step 2 below step 3
    tab = O.learned_table(_reader(O, {0: 1.0, 3: 8.0}, -2.5), 0, 5)
    _check_rows(tab, 5, lambda j, b0, bp, bc: max(0.0, bc + 16 * (j - 2.5)))
    assert tab[2, 0, 0, 7] == 1 and tab[3, 0, 0, 7] == 1 and tab[3, 0, 0, 31] == 32768
    # the pattern slot: only the model's own slot opens the candidate ramp
    for q in range(8):
        P = _reader(O, {0: 1.0, 7 + q: 4.0}, -3.0)
        for pat in (0, 3, 7):
            tab = O.learned_table(P, pat, 4)
            if pat == q:
                _check_rows(tab, 4, lambda j, b0, bp, bc: bc + 16)
            else:
                _check_rows(tab, 4, lambda j, b0, bp, bc: 0.0)
