"""Loose-mode selection rule (Sec. 5.1) on the host, and the premise of its
NS prediction checked with the oracle.

The rule: pilot slices of different sizes fit each launch's time as t0 + n/rate;
slice i predicts N_i = n_i (eps_hat_i / eps)^2 samples, taking N_i / rate plus t0
per window up to N_i, and the slices' minimum and maximum form the NS cone; two GS pilot colourings with relative
spread cv predict the smallest R >= 3 with t_{R-1} cv / sqrt(R) <= eps
colourings (the GS stop rule's Student t interval) at the mean colouring time;
GS runs only when its prediction lies entirely below the cone."""
import math

import numpy as np
import pytest
from scipy import stats


def _reps(cv, eps, cap, conf=0.95):
    """Colourings the GS stop rule needs, by scipy's t quantile."""
    for R in range(3, cap + 1):
        if stats.t.ppf(0.5 + conf / 2, R - 1) * cv / math.sqrt(R) <= eps:
            return R
    return None


@pytest.fixture(scope="module")
def S():
    from paper_2405_03488_amd import sgpm
    return sgpm


def test_cone_fit_and_windows(S, O):
    """Slices of 1/8, 1/8, 1/4, 1/2 of the pilot: times t0 + n/rate exactly,
    so the fit recovers t0 and rate; slice i predicts N_i = n_i (e_i/eps)^2
    samples in N_i / rate + t0 per window of the schedule up to N_i."""
    o = S.sgpm_options_default(n_min=1 << 16, w_min=1 << 15, quantum=1 << 10, window_growth=0.1)
    n = [8192, 8192, 16384, 32768]
    t0, rate = 5e-5, 1e9
    sec = [t0 + x / rate for x in n]
    eh = [0.05, 0.04, 0.045, 0.03]
    lo, hi, ft0, frate = S.sgpm_host_ns_cone(n, sec, eh, o)
    assert ft0 == pytest.approx(t0, rel=1e-9) and frate == pytest.approx(rate, rel=1e-9)
    oo = O.make_opts(n_min=1 << 16, w_min=1 << 15, quantum=1 << 10, growth=0.1)
    preds = []
    for ni, ei in zip(n, eh):
        need = ni * (ei / 0.01) ** 2
        w, e = 0, 0
        while True:
            nx = O.window_next(e, oo)
            w += 1
            if nx >= need or nx <= e:
                break
            e = nx
        preds.append(need / rate + t0 * w)
    assert lo == pytest.approx(min(preds), rel=1e-12) and hi == pytest.approx(max(preds), rel=1e-12)


def test_cone_fallback_and_missing_hits(S):
    o = S.sgpm_options_default(n_min=1 << 16, w_min=1 << 16, quantum=1 << 10)
    # times falling with size: no positive rate in the fit -> the slices' mean rate, t0 = 0
    lo, hi, t0, rate = S.sgpm_host_ns_cone([1000, 2000], [2e-3, 1e-3], [0.1, 0.1], o)
    assert t0 == 0.0 and rate == pytest.approx(3000 / 3e-3)
    # a slice without hits makes the upper end infinite; all without: the lower end too
    inf = float("inf")
    lo, hi, *_ = S.sgpm_host_ns_cone([1000, 2000], [1e-4, 2e-4], [0.1, inf], o)
    assert math.isfinite(lo) and math.isinf(hi)
    lo, hi, *_ = S.sgpm_host_ns_cone([1000, 2000], [1e-4, 2e-4], [inf, inf], o)
    assert math.isinf(lo) and math.isinf(hi)
    with pytest.raises(S.SgpmError):
        S.sgpm_host_ns_cone([], [], [], o)


def test_gs_prediction_and_choice(S):
    # three colourings (the rule's minimum) when they agree exactly
    sc, gs = S.sgpm_host_hybrid_choice(0.025, 0.01, 2, 0.5, 0.0)
    assert gs == pytest.approx(1.5) and sc == S.SCHEME_NS  # 1.5 s is above the cone's lower end
    sc, gs = S.sgpm_host_hybrid_choice(100.0, 0.01, 2, 0.2, 0.03)
    R = _reps(0.03, 0.01, 64)
    assert 36 < R < 64 and gs == pytest.approx(R * 0.2) and sc == S.SCHEME_GS
    # exactly at the lower end is not below it
    sc, gs = S.sgpm_host_hybrid_choice(1.0, 0.01, 2, 1 / 3, 0.0)
    assert gs == 1.0 and sc == S.SCHEME_NS


def test_one_colouring_never_selects_gs(S):
    sc, gs = S.sgpm_host_hybrid_choice(1.0, 0.01, 1, 1e-9, float("nan"))
    assert gs == pytest.approx(3e-9) and sc == S.SCHEME_NS  # the stop rule's three colourings


def test_missing_hits_and_caps(S):
    inf = float("inf")
    # no NS pilot hits: the cone is unbounded, a finite GS wins
    sc, gs = S.sgpm_host_hybrid_choice(inf, 0.01, 2, 5.0, 0.0)
    assert sc == S.SCHEME_GS
    # GS colourings all zero as well: nothing can be predicted, NS runs
    sc, gs = S.sgpm_host_hybrid_choice(inf, 0.01, 2, 5.0, inf)
    assert math.isinf(gs) and sc == S.SCHEME_NS
    # more colourings than gs_reps_max: GS cannot meet eps
    sc, gs = S.sgpm_host_hybrid_choice(1000.0, 0.01, 2, 1e-6, 0.2, 64)
    assert math.isinf(gs) and sc == S.SCHEME_NS
    sc, gs = S.sgpm_host_hybrid_choice(1000.0, 0.01, 2, 1e-6, 0.2, 4000)
    R = _reps(0.2, 0.01, 4000)
    assert R > 1000 and gs == pytest.approx(R * 1e-6) and sc == S.SCHEME_GS
    # a stricter confidence needs more colourings
    sc, gs99 = S.sgpm_host_hybrid_choice(1000.0, 0.01, 2, 1e-6, 0.2, 4000, confidence=0.99)
    assert gs99 == pytest.approx(_reps(0.2, 0.01, 4000, 0.99) * 1e-6) and gs99 > gs


def test_invalid_arguments(S):
    with pytest.raises(S.SgpmError):
        S.sgpm_host_hybrid_choice(1.0, 0.0, 2, 1.0, 0.0)
    with pytest.raises(S.SgpmError):
        S.sgpm_host_hybrid_choice(1.0, 0.01, 2, 1.0, 0.0, confidence=1.0)


@pytest.mark.parametrize("name,eps", [("triangle", 0.02), ("4-cycle", 0.005)])
def test_pilot_scaling_predicts_the_stop_point(O, synth, name, eps):
    """The NS prediction rests on the error equation: eps_hat falls as
    1/sqrt(n), so a pilot of n_p samples with error e_p predicts
    n_p (e_p / eps)^2 samples.  The oracle's strict run must stop within a
    small factor of that (windows grow by 10 %, the estimate is noisy).
    Light-tailed weights only: with heavy-tailed ones (the diamond on this
    power-law graph) a small pilot rarely sees the large weights and
    under-predicts, by 2.4x here, which is why an overlap with the cone
    selects NS."""
    n = 3000
    og = O.OGraph.from_raw_csr(n, *synth.pairs_to_csr(n, synth.chung_lu_pairs(n, 12, 2.1, 3)))
    op = O.compile_plan(*synth.pattern(name))
    z = O.norm_ppf(0.975)
    n_p = 1 << 14
    pilot = O.run(og, op, O.make_opts(fixed_n=n_p, seed=7, tag=0x80000000))
    assert pilot.eps_hat > eps
    predicted = n_p * (pilot.eps_hat / eps) ** 2
    full = O.run(og, op, O.make_opts(eps=eps, seed=7, n_min=1 << 12, w_min=1 << 12, quantum=1 << 10))
    assert full.converged == 1
    assert 0.5 * predicted <= full.n <= 2.0 * predicted, (predicted, full.n)
    assert z == pilot.z


def test_colour_choice_window(S):
    """colours = 0: the fewest colours whose predicted colouring time is within
    25 % of the time at 16 colours (Sec. 4.4 stabilisation window).  A colouring
    costs 2m / 1e11 + 3e-4 s of sparsification plus leaves16 (16 / c)^(k-1) / 3e9
    s of search."""
    def model(m, k, y16):
        sp = 2 * m / 1e11 + 3e-4
        at16 = sp + y16 / 3e9
        for c in (4, 5, 6, 8, 10, 12, 16):
            if sp + y16 * (16 / c) ** (k - 1) / 3e9 <= 1.25 * at16:
                return c
        return 16
    # no leaves: the search costs nothing, four colours keep the most matches
    assert S.sgpm_host_colours_choice(10**7, 4, 0.0) == 4
    # a search far dearer than the sparsification: as many colours as allowed
    assert S.sgpm_host_colours_choice(10**6, 5, 1e12) == 16
    for m in (10**5, 10**7, 10**9):
        for k in (3, 4, 5, 6):
            for y in (0.0, 1e3, 1e5, 1e7, 1e9):
                assert S.sgpm_host_colours_choice(m, k, y) == model(m, k, y), (m, k, y)
    # more leaves never choose fewer colours
    for k in (3, 5):
        cs = [S.sgpm_host_colours_choice(10**7, k, y) for y in np.logspace(0, 12, 40)]
        assert cs == sorted(cs)
    assert S.sgpm_host_colours_choice(10, 9, 1.0) == S.SGPM_EINVAL
    assert S.sgpm_host_colours_choice(10, 4, -1.0) == S.SGPM_EINVAL
