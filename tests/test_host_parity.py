"""Host parts of the library (graph loader, pattern compiler, statistics,
window schedule) against the oracle, bit for bit, on the CPU."""
import math

import numpy as np
import pytest

NAMES = ["edge", "triangle", "wedge", "4-clique", "5-clique", "6-clique", "4-cycle", "5-cycle", "4-path", "5-path",
         "3-star", "tailed-triangle", "diamond", "house", "dumbbell"]


@pytest.fixture(scope="module")
def S():
    from paper_2405_03488_amd import sgpm
    return sgpm


@pytest.mark.parametrize("gen", ["er", "rmat", "cl", "ring", "empty"])
def test_canonical_graph_matches_oracle(S, O, synth, gen):
    if gen == "er":
        n, pairs = 1000, synth.er_pairs(1000, 8000, 3)
    elif gen == "rmat":
        n, pairs = 1 << 12, synth.rmat_pairs(12, 16, seed=5)
    elif gen == "cl":
        n, pairs = 3000, synth.chung_lu_pairs(3000, 12, 2.1, 2)
    elif gen == "ring":
        n, pairs = 17, synth.ring_pairs(17)
    else:
        n, pairs = 9, np.zeros((0, 2), dtype=np.int32)
    off, nbr = synth.pairs_to_csr(n, pairs)
    m, o2, n2, p2 = S.sgpm_host_canonicalise(n, off, nbr)
    og = O.OGraph.from_raw_csr(n, off, nbr)
    assert m == og.m
    assert np.array_equal(o2, og.off)
    assert np.array_equal(n2, og.nbr)
    assert np.array_equal(p2, og.perm)
    # already canonical input is accepted as is
    m3, o3, n3, p3 = S.sgpm_host_canonicalise(n, og.off, og.nbr, S.SGPM_ASSUME_CANONICAL)
    assert m3 == m and np.array_equal(n3, og.nbr) and np.array_equal(p3, np.arange(n))


def test_assume_canonical_rejects_raw_input(S, synth):
    off, nbr = synth.pairs_to_csr(50, synth.er_pairs(50, 100, 1))
    with pytest.raises(S.SgpmError) as ei:
        S.sgpm_host_canonicalise(50, off, nbr, S.SGPM_ASSUME_CANONICAL)
    assert ei.value.status == S.SGPM_EBADGRAPH


def test_graph_flags_checked(S, synth):
    """Host canonicalisation takes host arrays only; unknown flags and the
    contradictory SYMMETRIZE | ASSUME_CANONICAL are rejected."""
    off, nbr = synth.pairs_to_csr(50, synth.er_pairs(50, 100, 1))
    for flags in (S.SGPM_DEVICE_PTRS, 0x100, S.SGPM_SYMMETRIZE | S.SGPM_ASSUME_CANONICAL):
        with pytest.raises(S.SgpmError) as ei:
            S.sgpm_host_canonicalise(50, off, nbr, flags)
        assert ei.value.status == S.SGPM_EINVAL
    a = S.sgpm_host_canonicalise(50, off, nbr, S.SGPM_SYMMETRIZE)
    b = S.sgpm_host_canonicalise(50, off, nbr, 0)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_bad_csr_rejected(S):
    with pytest.raises(S.SgpmError) as ei:
        S.sgpm_host_canonicalise(3, np.array([0, 1, 1, 1]), np.array([5], dtype=np.int32))
    assert ei.value.status == S.SGPM_EBADGRAPH
    with pytest.raises(S.SgpmError):
        S.sgpm_host_canonicalise(3, np.array([0, 2, 1, 2]), np.array([1, 2], dtype=np.int32))


@pytest.mark.parametrize("induced", [False, True])
@pytest.mark.parametrize("name", NAMES)
def test_plan_matches_oracle(S, O, synth, name, induced):
    k, e = synth.pattern(name)
    assert S.sgpm_host_plan(k, e, induced) == O.plan_dict(O.compile_plan(k, e, induced))


def test_plan_errors(S):
    with pytest.raises(S.SgpmError) as ei:
        S.sgpm_host_plan(4, [(0, 1), (2, 3)])
    assert ei.value.status == S.SGPM_EUNSUPPORTED
    with pytest.raises(S.SgpmError):
        S.sgpm_host_plan(9, [(i, i + 1) for i in range(8)])
    with pytest.raises(S.SgpmError) as ei:
        S.sgpm_host_plan(3, [(0, 5)])
    assert ei.value.status == S.SGPM_EINVAL


def test_normal_quantile_matches_oracle(S, O):
    for conf in [0.5, 0.8, 0.9, 0.95, 0.98, 0.99, 0.995, 0.999]:
        p = 1 - (1 - conf) / 2
        a, b = S.sgpm_host_normal_quantile(p), O.norm_ppf(p)
        assert abs(a - b) <= 2.3e-16 * b, (conf, a, b)


def test_predicted_error_bit_exact(S, O):
    rng = np.random.default_rng(1)
    z = O.norm_ppf(0.975)
    for _ in range(300):
        n = int(rng.integers(1, 2**40))
        k = int(rng.integers(1, 100))
        xs = [int(rng.integers(0, 2**62)) << int(rng.integers(0, 60)) for _ in range(k)]
        S1 = sum(xs)
        S2 = sum(x * x for x in xs) * max(1, n // k)
        if n * S2 < S1 * S1:
            continue
        assert S.sgpm_host_predicted_error(z, n, S1, S2) == O.eps_hat(z, n, S1, S2)
    assert S.sgpm_host_predicted_error(z, 10, 0, 0) == float("inf")


def test_t_quantile_matches_oracle(S, O):
    """The GS rule's Student t quantile: the library (incomplete beta, Newton)
    and the oracle (closed-form CDF, bisection) each work in extended
    precision and round to double; where the exact value lies near the
    midpoint of two doubles they may round apart, by one unit in the last
    place at most."""
    same = total = 0
    for nu in range(1, 130):
        for conf in (0.8, 0.9, 0.95, 0.99, 0.999):
            a, b = S.sgpm_host_t_quantile(conf, nu), O.t_ppf(conf, nu)
            assert a == b or math.nextafter(a, b) == b, (nu, conf, a, b)
            same += a == b
            total += 1
    assert same >= 0.9 * total
    assert math.isnan(S.sgpm_host_t_quantile(0.95, 0)) and math.isnan(S.sgpm_host_t_quantile(1.0, 3))


def test_predicted_error_t_bit_exact(S, O):
    rng = np.random.default_rng(12)
    for _ in range(300):
        n = int(rng.integers(2, 70))
        xs = [int(x) for x in rng.integers(0, 2**62, size=n)] if rng.random() < 0.5 else \
             [int(x) << int(rng.integers(0, 60)) for x in rng.integers(0, 1000, size=n)]
        S1, S2 = sum(xs), sum(x * x for x in xs)
        t = O.t_ppf(0.95, n - 1)
        assert S.sgpm_host_predicted_error_t(t, n, S1, S2) == O.eps_hat_t(t, n, S1, S2)
    assert S.sgpm_host_predicted_error_t(12.7, 1, 5, 25) == float("inf")


def test_window_schedule_matches_oracle(S, O):
    for n_min, w_min, q, g, mx in [(1 << 20, 1 << 20, 1 << 16, 0.1, 1 << 40), (1000, 300, 7, 0.25, 50000),
                                   (5, 5, 1, 0.0, 100)]:
        so = S.sgpm_options_default(n_min=n_min, w_min=w_min, quantum=q, window_growth=g, max_samples=mx)
        oo = O.make_opts(n_min=n_min, w_min=w_min, quantum=q, growth=g, max_samples=mx)
        n = 0
        for _ in range(200):
            a, b = S.sgpm_host_next_window(n, so), O.window_next(n, oo)
            assert a == b
            if a <= n:
                break
            n = a
