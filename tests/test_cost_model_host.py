"""Loose-mode cost models (Sec. 4.3 NS performance cone, Sec. 4.4 GS cost model,
Sec. 5.3 profiler, Sec. 5.1 selection) on the host: the library's arithmetic
against the formulas written out again here, with the plans taken from the
oracle's pattern compiler."""
import math

import pytest
from scipy import stats

CANDS = (4, 5, 6, 8, 10, 12, 16)


@pytest.fixture(scope="module")
def S():
    from paper_2405_03488_amd import sgpm
    return sgpm


def _bits(x):
    return bin(x).count("1")


def _reps(cv, eps, conf, cap):
    if not math.isfinite(cv):
        return 0
    for R in range(3, cap + 1):
        if stats.t.ppf(0.5 + conf / 2, R - 1) * cv / math.sqrt(R) <= eps:
            return R
    return 0


def model(plan, ci):
    """The cost models, from their definitions."""
    k = plan.k
    d = 2 * ci.m / ci.n
    rows = [_bits(plan.connect[j] | plan.disconnect[j]) for j in range(k)]
    w_hi = 1 + sum(rows[j] * d for j in range(2, k))
    w_lo = 1 + rows[2] * d
    ns = ci.prof_samples * (ci.prof_eps_hat / ci.eps) ** 2 * (ci.z / ci.prof_z) ** 2 * ci.rho_sparse / ci.rho_g \
        if ci.rho_g > 0 and ci.rho_sparse > 0 else math.inf
    per_unit = ci.pilot_seconds / (ci.pilot_samples * math.sqrt(w_lo * w_hi))
    cone = (per_unit * w_lo * ns, per_unit * w_hi * ns)
    p2 = min(1.0, 3 * ci.triangles * ci.n / (2 * ci.m ** 2))

    def search(p):
        p1 = 2 * ci.m * p / ci.n ** 2
        levels = [(1 if plan.oriented else 2) * p * ci.m]
        work = 0.0
        prod = levels[0]
        for j in range(2, k):
            work += prod * rows[j] * d * p
            ij = ci.n * p1 * p2 ** (_bits(plan.connect[j]) - 1) * (0.5 if (plan.upper[j] or plan.lower[j]) else 1.0)
            prod *= ij
        return work

    pre = ci.sparsify_seconds / (ci.m * (1 + ci.sparsify_keep))
    unit = ci.probe_search_seconds / search(1 / ci.probe_colours)
    gs = []
    for c in CANDS:
        cv = math.sqrt((c ** (k - 1) - 1) / ci.count) if ci.count > 0 else math.inf
        R = _reps(cv, ci.eps, ci.confidence, ci.gs_reps_max) if ci.count > 0 else 3
        t = R * (pre * ci.m * (1 + 1 / c) + unit * search(1 / c)) if R else math.inf
        gs.append((t, R))
    return w_lo, w_hi, ns, cone, gs


def inputs(S, **kw):
    base = dict(n=1e6, m=1.5e7, triangles=2e8, count=1.7e10, eps=0.01, confidence=0.95, z=1.959963984540054,
                gs_reps_max=64, pilot_samples=65536, pilot_seconds=1e-4, rho_g=0.66, prof_samples=3e4,
                prof_eps_hat=0.45, prof_z=2.5758293035489004, rho_sparse=0.02, sparsify_seconds=5e-4,
                sparsify_keep=0.1, probe_colours=16, probe_search_seconds=2e-3)
    base.update(kw)
    return S.CostIn(**base)


@pytest.mark.parametrize("name,induced", [("triangle", False), ("4-clique", False), ("5-clique", False),
                                          ("4-cycle", False), ("diamond", True), ("house", False), ("wedge", False)])
@pytest.mark.parametrize("case", [{}, dict(count=3e4, triangles=5e9), dict(rho_sparse=1e-4, prof_samples=1e5),
                                  dict(m=2e5, n=1e5, count=50.0, probe_search_seconds=1e-5)])
def test_cost_model_matches_definition(S, O, synth, name, induced, case):
    k, e = synth.pattern(name)
    plan = O.compile_plan(k, e, induced)
    ci = inputs(S, **case)
    out = S.sgpm_host_cost_model(k, e, ci, induced)
    w_lo, w_hi, ns, cone, gs = model(plan, ci)
    assert out.w_lo == pytest.approx(w_lo, rel=1e-12) and out.w_hi == pytest.approx(w_hi, rel=1e-12)
    assert out.ns_samples == pytest.approx(ns, rel=1e-12)
    assert out.ns_lo == pytest.approx(cone[0], rel=1e-12) and out.ns_hi == pytest.approx(cone[1], rel=1e-12)
    for i, (t, R) in enumerate(gs):
        assert out.gs_reps[i] == R, (i, R)
        assert (math.isinf(out.gs_seconds[i]) and math.isinf(t)) or out.gs_seconds[i] == pytest.approx(t, rel=1e-12)
    finite = [(t, c) for (t, _), c in zip(gs, CANDS) if math.isfinite(t)]
    best_t, best_c = min(finite) if finite else (math.inf, 0)
    assert out.gs_colours == best_c and (out.gs_best == pytest.approx(best_t, rel=1e-12) or math.isinf(best_t))
    assert out.choice == (S.SCHEME_GS if best_t < cone[0] else S.SCHEME_NS)


def test_cone_orders_and_limits(S, synth):
    k, e = synth.pattern("5-clique")
    out = S.sgpm_host_cost_model(k, e, inputs(S))
    # the full walk reads more rows than the first break point
    assert out.w_lo < out.w_hi and out.ns_lo < out.ns_hi
    # more work per unit time on the pilot scales both ends
    out2 = S.sgpm_host_cost_model(k, e, inputs(S, pilot_seconds=2e-4))
    assert out2.ns_lo == pytest.approx(2 * out.ns_lo) and out2.ns_hi == pytest.approx(2 * out.ns_hi)
    # halving eps quadruples the samples
    out3 = S.sgpm_host_cost_model(k, e, inputs(S, eps=0.005))
    assert out3.ns_samples == pytest.approx(4 * out.ns_samples)
    # no hits on the pilot: NS cannot be predicted, a feasible GS is chosen
    out4 = S.sgpm_host_cost_model(k, e, inputs(S, rho_g=0.0))
    assert math.isinf(out4.ns_samples) and math.isinf(out4.ns_lo) and out4.choice == S.SCHEME_GS
    # GS inside or above the cone selects NS
    out5 = S.sgpm_host_cost_model(k, e, inputs(S, probe_search_seconds=10.0))
    assert out5.choice == S.SCHEME_NS and out5.gs_best > out5.ns_lo


def test_gs_variance_drives_the_colour_count(S, synth):
    """A rare pattern (small count) needs more colourings at many colours: the
    fastest colour count moves down as the count falls (Sec. 4.4: few colours,
    high keep probability, for accuracy)."""
    k, e = synth.pattern("4-clique")
    cols = [S.sgpm_host_cost_model(k, e, inputs(S, count=C, probe_search_seconds=1e-4)).gs_colours
            for C in (1e12, 1e8, 1e6, 1e5)]
    assert cols == sorted(cols, reverse=True) and cols[0] > cols[-1]
