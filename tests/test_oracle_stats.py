"""Pins for the oracle's statistics and stop rule (Sec. 4.1, the NS-online
algorithm and the error equation; Theorem on confidence)."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest


def test_norm_ppf_against_scipy(O):
    from scipy.stats import norm
    for conf in [0.5, 0.8, 0.9, 0.95, 0.98, 0.99, 0.995, 0.999, 0.9999]:
        p = 1 - (1 - conf) / 2
        assert abs(O.norm_ppf(p) - norm.ppf(p)) <= 5e-16 * norm.ppf(p)  # two ulps
    assert abs(O.norm_ppf(0.975) - 1.959963984540054) < 1e-15
    assert abs(O.norm_ppf(0.995) - 2.5758293035489004) < 1e-15


def _paper_eps(z, xs):
    """The paper's sequence of operations in 60-digit decimals:
    mu = sum/n, var = squaredSum/n - mu^2, sigma = sqrt(var/n), eps = z*sigma/mu."""
    getcontext().prec = 60
    n = Decimal(len(xs))
    s = Decimal(sum(xs))
    ss = Decimal(sum(x * x for x in xs))
    mu = s / n
    var = ss / n - mu * mu
    sigma = (var / n).sqrt()
    return float(Decimal(z) * sigma / mu)


@pytest.mark.parametrize("case", [
    [1, 2, 3, 4, 5],
    [0, 0, 0, 7, 0, 0, 9, 0],
    [10**20, 3 * 10**20, 0, 5 * 10**19],
    [2**100 + 17, 2**99, 0, 0, 2**101],
    [123456789] * 9 + [123456790],
])
def test_eps_hat_matches_paper_formula(O, case):
    z = 1.959963984540054
    S1 = sum(case)
    S2 = sum(x * x for x in case)
    got = O.eps_hat(z, len(case), S1, S2)
    want = _paper_eps(z, case)
    assert abs(got - want) <= 1e-13 * want


def test_eps_hat_against_numpy_population_std(O):
    rng = np.random.default_rng(0)
    xs = rng.integers(0, 1000, size=5000) * (rng.random(5000) < 0.3)
    z = O.norm_ppf(0.975)
    got = O.eps_hat(z, len(xs), int(xs.sum()), int((xs.astype(object) ** 2).sum()))
    want = z * np.std(xs.astype(np.float64)) / math.sqrt(len(xs)) / np.mean(xs)
    assert abs(got - want) < 1e-9 * want


def test_eps_hat_special_cases(O):
    assert O.eps_hat(1.96, 10, 0, 0) == float("inf")
    assert O.eps_hat(1.96, 4, 20, 100) == 0.0  # all samples equal 5


def test_window_schedule(O):
    o = O.make_opts(n_min=1 << 20, w_min=1 << 20, quantum=1 << 16, max_samples=1 << 30, growth=0.10)
    n = 0
    seq = []
    while True:
        nx = O.window_next(n, o)
        if nx <= n:
            break
        seq.append(nx)
        n = nx
    assert seq[0] == 1 << 20
    assert all(x % (1 << 16) == 0 for x in seq)
    for a, b in zip(seq, seq[1:]):
        inc = max(1 << 20, math.ceil(0.1 * a))
        assert b == min(1 << 30, -(-(a + inc) // (1 << 16)) * (1 << 16))
    assert seq[-1] == 1 << 30


def test_stop_rule_first_window_below_eps(O, synth):
    g = O.OGraph.from_pairs(2000, synth.er_pairs(2000, 16000, 1))
    k, e = synth.pattern("triangle")
    p = O.compile_plan(k, e)
    o = O.make_opts(eps=0.05, n_min=20000, w_min=20000, quantum=1000, seed=3)
    r, et, nt = O.run(g, p, o, trace_cap=200)
    assert r.converged == 1
    assert et[-1] <= 0.05 and all(x > 0.05 for x in et[:-1])
    assert nt[-1] == r.n


def test_coverage(O, synth):
    """Theorem (Sec. 4.1): P(|mu - C|/C < eps_hat) -> 1 - delta; check the
    empirical coverage at fixed n over 200 seeds sits in the binomial 99% band."""
    g = O.OGraph.from_pairs(500, synth.er_pairs(500, 5000, 2))
    k, e = synth.pattern("triangle")
    p = O.compile_plan(k, e)
    C = O.plan_count(g, p)
    R = 200
    inside = 0
    for seed in range(R):
        r = O.run(g, p, O.make_opts(fixed_n=20000, seed=1000 + seed, confidence=0.95))
        inside += abs(r.estimate - C) / C < r.eps_hat
    # Binomial(200, 0.95): mean 190, sd 3.08; 99% band ~ [182, 198]
    assert 180 <= inside <= 200, inside


def test_big_integer_to_double_is_correctly_rounded(O):
    """Python's int -> float conversion rounds to nearest, ties to even."""
    rng = np.random.default_rng(5)
    cases = [0, 1, 2**53 - 1, 2**53, 2**53 + 1, 2**53 + 3, 2**64 + 2**11, 2**64 + 2**11 + 1, (2**53 + 1) << 70]
    for _ in range(500):
        bits = int(rng.integers(1, 700))
        cases.append(int.from_bytes(rng.bytes(88), "little") >> (704 - bits))
    for x in cases:
        assert O.digits_to_double(x) == float(x), x


def _mp_t_quantile(conf, nu):
    """Two-sided t quantile from the regularised incomplete beta in 40-digit
    arithmetic: P(|T| <= t) = 1 - I_{nu/(nu+t^2)}(nu/2, 1/2), solved by bisection."""
    import mpmath as mp
    mp.mp.dps = 40
    f = lambda t: 1 - mp.betainc(mp.mpf(nu) / 2, mp.mpf(1) / 2, 0, nu / (nu + t * t), regularized=True) - conf
    lo, hi = mp.mpf(0), mp.mpf(1)
    while f(hi) < 0:
        hi *= 2
    for _ in range(200):
        mid = (lo + hi) / 2
        if f(mid) < 0:
            lo = mid
        else:
            hi = mid
    return (lo + hi) / 2


@pytest.mark.parametrize("nu", [1, 2, 3, 4, 5, 8, 13, 30, 63, 100])
def test_t_ppf_against_high_precision(O, nu):
    """The GS interval's Student t quantile (closed-form CDF for integer
    degrees of freedom) against 40-digit arithmetic and scipy."""
    from scipy import stats
    for conf in [0.5, 0.9, 0.95, 0.99]:
        want = _mp_t_quantile(conf, nu)
        got = O.t_ppf(conf, nu)
        assert abs(got - float(want)) <= 2e-16 * float(want), (nu, conf)
        assert abs(got - stats.t.ppf(0.5 + conf / 2, nu)) <= 1e-9 * got
    # textbook values: t_1(0.975) = tan(0.475 pi), t_2(0.975) = 4.302652729...
    assert abs(O.t_ppf(0.95, 1) - math.tan(0.475 * math.pi)) < 1e-13
    # t approaches the normal quantile
    assert O.t_ppf(0.95, 5000) > O.norm_ppf(0.975) and O.t_ppf(0.95, 5000) - O.norm_ppf(0.975) < 1e-3


@pytest.mark.parametrize("case", [
    [1, 2, 3, 4, 5],
    [0, 0, 7, 0, 9],
    [10**20, 3 * 10**20, 5 * 10**19],
    [2**100 + 17, 2**99, 2**101],
])
def test_eps_hat_t_is_unbiased_standard_error(O, case):
    """t * s / sqrt(n) / mean with s^2 the unbiased sample variance, in 60-digit decimals."""
    getcontext().prec = 60
    n = len(case)
    mean = Decimal(sum(case)) / n
    s2 = sum((Decimal(x) - mean) ** 2 for x in case) / (n - 1)
    t = 2.7764451051977987
    want = float(Decimal(t) * (s2 / n).sqrt() / mean)
    got = O.eps_hat_t(t, n, sum(case), sum(x * x for x in case))
    assert abs(got - want) <= 1e-13 * want
    assert O.eps_hat_t(t, 1, 5, 25) == float("inf")
    assert O.eps_hat_t(t, 3, 0, 0) == float("inf")


def test_gs_sums_beyond_32_bits(O, synth):
    """GS repetition statistics with X_r = c^(k-1) Y_r far above 2^32: the
    oracle's digit sums equal Python big-integer sums of its per-colouring
    counts, and its interval is the t interval of those values."""
    n = 140
    g = O.OGraph.from_pairs(n, synth.complete_pairs(n))
    k, e = synth.pattern("6-clique")
    p = O.compile_plan(k, e)
    c = 4
    r, ys = O.gs_run(g, p, c, 5, eps=-1.0, reps_max=6)  # eps < 0: never stops early
    xs = [y * c ** (k - 1) for y in ys]
    assert r.reps == 6 and min(xs) > 2**32 and len(set(xs)) > 1
    assert r.S1 == sum(xs) and r.S2 == sum(x * x for x in xs)
    t = O.t_ppf(0.95, 5)
    assert r.z == t
    assert r.eps_hat == O.eps_hat_t(t, 6, sum(xs), sum(x * x for x in xs))
    assert r.estimate == O.digits_to_double(sum(xs)) / 6


def _gs_coverage(O, g, p, C, c, eps, seeds):
    """Among converged GS runs: (runs, count inside the interval)."""
    runs = inside = 0
    for seed in seeds:
        r, _ = O.gs_run(g, p, c, seed, eps=eps, reps_max=64, threads=1)
        if r.converged:
            runs += 1
            half = r.estimate * r.eps_hat
            inside += abs(r.estimate - C) <= half
    return runs, inside


def test_gs_interval_coverage(O, synth):
    """The GS stop rule (Student t interval, unbiased variance, tested from the
    third colouring on) on a light-tailed count: among 100 seeds the exact
    count lies inside the reported 95 % interval in at least 85 (binomial:
    mean 95, sd 2.2 at the nominal rate; optional stopping costs a few).  The
    normal quantile with the 1/n variance and a test from the second colouring
    on, applied to the same colourings, falls far short -- which is why the
    rule changed."""
    n = 1500
    g = O.OGraph.from_raw_csr(n, *synth.pairs_to_csr(n, synth.chung_lu_pairs(n, 10, 2.1, 3)))
    k, e = synth.pattern("triangle")
    p = O.compile_plan(k, e)
    C = O.plan_count(g, p)
    runs, inside = _gs_coverage(O, g, p, C, 2, 0.1, range(100))
    assert runs >= 98 and inside >= 85, (runs, inside)
    # the former rule on the same colourings
    z = O.norm_ppf(0.975)
    old_in = 0
    for seed in range(100):
        _, ys = O.gs_run(g, p, 2, seed, eps=0.0, reps_max=12, threads=1)
        S1 = S2 = 0
        for m, y in enumerate(ys, 1):
            x = y * 2 ** (k - 1)
            S1 += x
            S2 += x * x
            eh = O.eps_hat(z, m, S1, S2)
            if m >= 2 and eh <= 0.1:
                old_in += abs(S1 / m - C) <= eh * S1 / m
                break
    assert old_in <= 75, old_in
