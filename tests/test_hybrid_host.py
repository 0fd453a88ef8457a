"""Loose-mode selection rule (Sec. 5.1) on the host, and the premise of its
NS prediction checked with the oracle.

The rule: each NS pilot slice predicts t_i (eps_hat_i / eps)^2 and the slices'
minimum and maximum form the NS cone; two GS pilot colourings predict
R = max(2, ceil(2 (eps_hat_2 / eps)^2)) colourings at the mean colouring time;
GS runs only when its prediction lies entirely below the cone."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def S():
    from paper_2405_03488_amd import sgpm
    return sgpm


def test_cone_from_slices(S):
    sc, lo, hi, gs = S.sgpm_host_hybrid_choice([1e-3, 2e-3, 1e-3, 1e-3], [0.1, 0.1, 0.2, 0.05], 0.01, 2, 0.5, 0.0)
    assert lo == pytest.approx(1e-3 * 25) and hi == pytest.approx(1e-3 * 400)
    assert gs == pytest.approx(1.0)  # two colourings suffice when they agree exactly
    assert sc == S.SCHEME_NS  # 1.0 s is above the cone's lower end 0.025 s


def test_gs_below_cone_selects_gs(S):
    sc, lo, hi, gs = S.sgpm_host_hybrid_choice([0.01] * 4, [1.0, 2.0, 1.5, 1.2], 0.01, 2, 0.2, 0.03)
    # R = ceil(2 * 3^2) = 18 colourings of 0.2 s
    assert gs == pytest.approx(18 * 0.2)
    assert lo == pytest.approx(0.01 * 1e4) and sc == S.SCHEME_GS


def test_overlap_and_above_select_ns(S):
    # GS inside the cone: NS keeps the guarantee
    sc, lo, hi, gs = S.sgpm_host_hybrid_choice([1.0, 1.0], [0.01, 0.02], 0.01, 2, 1.5, 0.0)
    assert lo == 1.0 and hi == 4.0 and gs == 3.0 and sc == S.SCHEME_NS
    # GS above the cone
    sc, *_ = S.sgpm_host_hybrid_choice([1.0, 1.0], [0.01, 0.02], 0.01, 2, 10.0, 0.0)
    assert sc == S.SCHEME_NS
    # exactly at the lower end is not below it
    sc, *_ = S.sgpm_host_hybrid_choice([1.0], [0.01], 0.01, 2, 0.5, 0.0)
    assert sc == S.SCHEME_NS


def test_one_colouring_never_selects_gs(S):
    sc, lo, hi, gs = S.sgpm_host_hybrid_choice([1.0], [1.0], 0.01, 1, 1e-9, float("nan"))
    assert gs == pytest.approx(2e-9) and sc == S.SCHEME_NS


def test_missing_hits_and_caps(S):
    inf = float("inf")
    # no NS pilot hits anywhere: the cone is unbounded, a finite GS wins
    sc, lo, hi, gs = S.sgpm_host_hybrid_choice([1e-3] * 4, [inf] * 4, 0.01, 2, 5.0, 0.0)
    assert math.isinf(lo) and math.isinf(hi) and sc == S.SCHEME_GS
    # GS colourings all zero as well: nothing can be predicted, NS runs
    sc, lo, hi, gs = S.sgpm_host_hybrid_choice([1e-3] * 4, [inf] * 4, 0.01, 2, 5.0, inf)
    assert math.isinf(gs) and sc == S.SCHEME_NS
    # some slices without hits: the cone's upper end is unbounded
    sc, lo, hi, gs = S.sgpm_host_hybrid_choice([1e-3, 1e-3], [0.5, inf], 0.01, 2, 5.0, 0.0)
    assert lo == pytest.approx(2.5) and math.isinf(hi)
    # more colourings than gs_reps_max: GS cannot meet eps
    sc, lo, hi, gs = S.sgpm_host_hybrid_choice([1.0], [10.0], 0.01, 2, 1e-6, 0.2, 64)
    assert math.isinf(gs) and sc == S.SCHEME_NS
    sc, lo, hi, gs = S.sgpm_host_hybrid_choice([1.0], [10.0], 0.01, 2, 1e-6, 0.2, 1000)
    assert gs == pytest.approx(800 * 1e-6) and sc == S.SCHEME_GS


def test_invalid_arguments(S):
    with pytest.raises(S.SgpmError):
        S.sgpm_host_hybrid_choice([], [], 0.01, 2, 1.0, 0.0)
    with pytest.raises(S.SgpmError):
        S.sgpm_host_hybrid_choice([1.0], [1.0], 0.0, 2, 1.0, 0.0)


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
