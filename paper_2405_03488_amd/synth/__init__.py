"""Seeded synthetic inputs shared by the HIP path's callers and the CPU oracle's tests.

Nothing here computes any part of the estimator: these functions only produce
raw graphs (edge pairs or an unsorted, possibly duplicated CSR) and small pattern
edge lists.  Large random graphs come from ``gen.c`` (SplitMix64 counter streams);
structured graphs with closed-form pattern counts are built directly here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsgpm_synth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into libsgpm_synth.so (plain gcc, host only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-std=c11",
                               os.path.join(_HERE, "gen.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        p = ctypes.c_void_p
        lib.sgpm_gen_er.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, p]
        lib.sgpm_gen_er.restype = ctypes.c_int64
        lib.sgpm_gen_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_uint64, p, ctypes.c_int]
        lib.sgpm_gen_rmat.restype = ctypes.c_int64
        lib.sgpm_gen_chung_lu.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                          p, ctypes.c_int]
        lib.sgpm_gen_chung_lu.restype = ctypes.c_int64
        lib.sgpm_pairs_to_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, p, p, p]
        lib.sgpm_pairs_to_csr.restype = ctypes.c_int
        _lib = lib
    return _lib


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def er_pairs(n: int, m: int, seed: int) -> np.ndarray:
    out = np.empty((m, 2), dtype=np.int32)
    got = _load().sgpm_gen_er(n, m, seed, out.ctypes.data)
    if got != m:
        raise ValueError(f"ER generator failed ({got})")
    return out


def rmat_pairs(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
               seed: int = 1) -> np.ndarray:
    npairs = edge_factor << scale
    out = np.empty((npairs, 2), dtype=np.int32)
    got = _load().sgpm_gen_rmat(scale, npairs, a, b, c, seed, out.ctypes.data, _threads())
    if got != npairs:
        raise ValueError("R-MAT generator failed")
    return out


def chung_lu_pairs(n: int, avg_degree: float, gamma: float, seed: int) -> np.ndarray:
    npairs = int(n * avg_degree // 2)
    out = np.empty((npairs, 2), dtype=np.int32)
    got = _load().sgpm_gen_chung_lu(n, npairs, gamma, seed, out.ctypes.data, _threads())
    if got != npairs:
        raise ValueError("Chung-Lu generator failed")
    return out


def pairs_to_csr(n: int, pairs: np.ndarray):
    """Raw CSR (int64 offsets, int32 neighbours) listing each pair once under its first id."""
    pairs = np.ascontiguousarray(pairs, dtype=np.int32)
    off = np.empty(n + 1, dtype=np.int64)
    nbr = np.empty(len(pairs), dtype=np.int32)
    rc = _load().sgpm_pairs_to_csr(n, len(pairs), pairs.ctypes.data, off.ctypes.data, nbr.ctypes.data)
    if rc != 0:
        raise ValueError("pairs_to_csr: vertex id out of range")
    return off, nbr


# ------------------------------------------------------------------ structured graphs
def complete_pairs(n: int) -> np.ndarray:
    return np.array([(i, j) for i in range(n) for j in range(i + 1, n)], dtype=np.int32).reshape(-1, 2)


def ring_pairs(n: int) -> np.ndarray:
    return np.array([(i, (i + 1) % n) for i in range(n)], dtype=np.int32)


def grid_pairs(a: int, b: int) -> np.ndarray:
    e = []
    for i in range(a):
        for j in range(b):
            v = i * b + j
            if j + 1 < b:
                e.append((v, v + 1))
            if i + 1 < a:
                e.append((v, v + b))
    return np.array(e, dtype=np.int32).reshape(-1, 2)


def hypercube_pairs(d: int) -> np.ndarray:
    e = [(v, v ^ (1 << t)) for v in range(1 << d) for t in range(d) if v < v ^ (1 << t)]
    return np.array(e, dtype=np.int32).reshape(-1, 2)


def complete_bipartite_pairs(a: int, b: int) -> np.ndarray:
    return np.array([(i, a + j) for i in range(a) for j in range(b)], dtype=np.int32).reshape(-1, 2)


def petersen_pairs() -> np.ndarray:
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return np.array(outer + spokes + inner, dtype=np.int32)


def star_pairs(t: int) -> np.ndarray:
    return np.array([(0, i) for i in range(1, t + 1)], dtype=np.int32).reshape(-1, 2)


def relabel_pairs(pairs: np.ndarray, n: int, seed: int) -> np.ndarray:
    """Apply a seeded random vertex permutation (to test label independence)."""
    rng = np.random.default_rng(seed)
    p = rng.permutation(n).astype(np.int32)
    return p[pairs]


# ------------------------------------------------------------------ patterns (edge lists)
PATTERNS = {
    "edge": (2, [(0, 1)]),
    "triangle": (3, [(0, 1), (1, 2), (0, 2)]),
    "wedge": (3, [(0, 1), (0, 2)]),          # 3-path
    "4-clique": (4, [(a, b) for a in range(4) for b in range(a + 1, 4)]),
    "5-clique": (5, [(a, b) for a in range(5) for b in range(a + 1, 5)]),
    "6-clique": (6, [(a, b) for a in range(6) for b in range(a + 1, 6)]),
    "4-cycle": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),
    "5-cycle": (5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)]),
    "4-path": (4, [(0, 1), (1, 2), (2, 3)]),
    "5-path": (5, [(0, 1), (1, 2), (2, 3), (3, 4)]),
    "3-star": (4, [(0, 1), (0, 2), (0, 3)]),
    "tailed-triangle": (4, [(0, 1), (1, 2), (0, 2), (2, 3)]),
    "diamond": (4, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)]),
    "house": (5, [(0, 1), (1, 2), (2, 3), (3, 0), (2, 4), (3, 4)]),
    "dumbbell": (6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (2, 3)]),
    "7-clique": (7, [(a, b) for a in range(7) for b in range(a + 1, 7)]),
    "8-clique": (8, [(a, b) for a in range(8) for b in range(a + 1, 8)]),
    "7-cycle": (7, [(a, (a + 1) % 7) for a in range(7)]),
    "8-path": (8, [(a, a + 1) for a in range(7)]),
    "wheel-7": (7, [(0, a) for a in range(1, 7)] + [(a, a % 6 + 1) for a in range(1, 7)]),
}


def pattern(name: str):
    k, e = PATTERNS[name]
    return k, np.array(e, dtype=np.int32).reshape(-1, 2)
