"""Pins for the oracle's Philox4x32-10 and index mapping.

Philox (Salmon et al., SC'11) is pinned to rocRAND's host-callable
Philox4x32-10 engine, an independent implementation; the multiply-high index
map is pinned to exact big-integer floor division.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HELPER = os.path.join(os.path.dirname(__file__), "helpers", "rocrand_philox.cpp")


@pytest.fixture(scope="module")
def rocrand_bin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("rr") / "rr")
    subprocess.check_call([hipcc, "-O1", HELPER, "-o", out])
    return out


def test_philox_matches_rocrand(O, rocrand_bin):
    rng = np.random.default_rng(12345)
    # rocRAND addresses the counter through offset = 4 s, so s stays below 2^62 here
    rows = [(0, 0, 0, 0), (1, 5, 2, 7), (2**64 - 1, 2**62 - 1, 2**32 - 1, 2**32 - 1)]
    for _ in range(300):
        rows.append((int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2)),
                     int(rng.integers(0, 2**62)), int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))))
    text = "".join(f"{a} {b} {c} {d}\n" for a, b, c, d in rows)
    res = subprocess.run([rocrand_bin], input=text, capture_output=True, text=True, check=True).stdout.split("\n")
    for (seed, s, d, tag), line in zip(rows, res):
        want = [int(x) for x in line.split()]
        got = O.philox([s & 0xFFFFFFFF, s >> 32, d, tag], [seed & 0xFFFFFFFF, seed >> 32])
        assert got == want, (seed, s, d, tag)


def test_draw_layout(O):
    for seed, s, d, tag in [(1, 0, 0, 0), (7, 2**40 + 3, 5, 0x80000001)]:
        w = O.philox([s & 0xFFFFFFFF, s >> 32, d, tag], [seed & 0xFFFFFFFF, seed >> 32])
        assert O.draw(seed, s, d, tag) == (w[1] << 32) | w[0]


def test_mulhi_exact(O):
    rng = np.random.default_rng(3)
    for _ in range(2000):
        n = int(rng.integers(1, 2**62))
        r = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        assert O.mulhi(n, r) == (n * r) >> 64
    assert O.mulhi(7, 0) == 0
    assert O.mulhi(7, 2**64 - 1) == 6
    # every index of a small set is reachable and the preimages differ in size by at most one
    N = 5
    edges = [-((-i << 64) // N) for i in range(N + 1)]
    sizes = [edges[i + 1] - edges[i] for i in range(N)]
    assert max(sizes) - min(sizes) <= 1
    for i in range(N):
        assert O.mulhi(N, edges[i]) == i


def test_draw_uniformity(O):
    bins = np.zeros(64, dtype=np.int64)
    n = 64000
    for s in range(n):
        bins[O.mulhi(64, O.draw(99, s, 3, 0))] += 1
    chi2 = float(((bins - n / 64) ** 2 / (n / 64)).sum())
    assert chi2 < 120.0  # 63 dof, p ~ 1e-5
