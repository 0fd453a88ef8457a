"""Thin ctypes binding of libsgpm (include/sgpm.h): argument marshalling only.

Every step of the estimator runs inside libsgpm's HIP kernels and C++ host
code.  Importing this module never falls back to anything else: if the built
library is missing, it raises.  PyTorch is only used, when present, to hand the
library the current HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libsgpm.so")

SGPM_OK = 0
SGPM_EINVAL = -1
SGPM_ENOMEM = -2
SGPM_EHIP = -3
SGPM_EUNSUPPORTED = -4
SGPM_NOT_CONVERGED = -5
SGPM_EBADGRAPH = -6
SGPM_EOVERFLOW = -7
SGPM_ASSUME_CANONICAL = 0x1
SGPM_DEVICE_PTRS = 0x2
SGPM_SYMMETRIZE = 0x4

MODE_STRICT_NS, MODE_FIXED_N, MODE_GS, MODE_HYBRID = 0, 1, 2, 3
SAMPLER_PRUNE, SAMPLER_BASE = 0, 1
HYBRID_PILOTS, HYBRID_COST_MODEL = 0, 1
GS_COLOUR, GS_BERNOULLI = 0, 1
SCHEME_NS, SCHEME_GS, SCHEME_EXACT = 0, 1, 2


class TraceRec(C.Structure):
    _fields_ = [("s", C.c_uint64), ("v", C.c_int32 * 8), ("status", C.c_uint32), ("k", C.c_uint32),
                ("alpha_lo", C.c_uint64), ("alpha_hi", C.c_uint64)]

    @property
    def alpha(self) -> int:
        return (self.alpha_hi << 64) | self.alpha_lo


class Options(C.Structure):
    _fields_ = [("eps", C.c_double), ("confidence", C.c_double), ("seed", C.c_uint64), ("query_tag", C.c_uint32),
                ("mode", C.c_int32), ("fixed_n", C.c_uint64), ("n_min", C.c_uint64), ("w_min", C.c_uint64),
                ("quantum", C.c_uint64), ("max_samples", C.c_uint64), ("window_growth", C.c_double),
                ("colours", C.c_int32), ("gs_reps_max", C.c_int32), ("proposal", C.c_void_p),
                ("lanes_per_sample", C.c_int32), ("checksum", C.c_int32), ("trace_lo", C.c_uint64),
                ("trace_hi", C.c_uint64), ("trace_buf", C.c_void_p), ("sampler", C.c_int32),
                ("gs_scheme", C.c_int32), ("hybrid_selector", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("estimate", C.c_double), ("eps_hat", C.c_double), ("ci_lo", C.c_double), ("ci_hi", C.c_double),
                ("z", C.c_double), ("n_samples", C.c_uint64), ("n_hits", C.c_uint64),
                ("sum_digits", C.c_uint32 * 8), ("sumsq_digits", C.c_uint32 * 12), ("scheme", C.c_int32),
                ("colours", C.c_int32), ("converged", C.c_int32), ("windows", C.c_int32),
                ("lanes_per_sample", C.c_int32), ("launches", C.c_int32), ("checksum", C.c_uint64),
                ("bytes", C.c_uint64), ("seconds_sampling", C.c_double), ("seconds_total", C.c_double),
                ("seconds_kernel", C.c_double), ("tile", C.c_int32), ("weight_shift", C.c_int32),
                ("reserved0", C.c_int32), ("pred_ns_lo", C.c_double), ("pred_ns_hi", C.c_double),
                ("pred_gs", C.c_double), ("seconds_pilot", C.c_double), ("seconds_kernel_busy", C.c_double),
                ("pred_samples", C.c_double)]

    @property
    def S1(self) -> int:
        return sum(int(d) << (32 * i) for i, d in enumerate(self.sum_digits))

    @property
    def S2(self) -> int:
        return sum(int(d) << (32 * i) for i, d in enumerate(self.sumsq_digits))


class CostIn(C.Structure):
    _fields_ = [("n", C.c_double), ("m", C.c_double), ("triangles", C.c_double), ("count", C.c_double),
                ("eps", C.c_double), ("confidence", C.c_double), ("z", C.c_double), ("gs_reps_max", C.c_int32),
                ("reserved", C.c_int32), ("pilot_samples", C.c_double), ("pilot_seconds", C.c_double),
                ("rho_g", C.c_double), ("prof_samples", C.c_double), ("prof_eps_hat", C.c_double),
                ("prof_z", C.c_double), ("rho_sparse", C.c_double), ("sparsify_seconds", C.c_double),
                ("sparsify_keep", C.c_double), ("probe_colours", C.c_double), ("probe_search_seconds", C.c_double)]


class CostOut(C.Structure):
    _fields_ = [("w_lo", C.c_double), ("w_hi", C.c_double), ("ns_samples", C.c_double), ("ns_lo", C.c_double),
                ("ns_hi", C.c_double), ("gs_seconds", C.c_double * 7), ("gs_reps", C.c_int32 * 7),
                ("gs_colours", C.c_int32), ("gs_best", C.c_double), ("choice", C.c_int32), ("reserved", C.c_int32)]


class TrainCfg(C.Structure):
    _fields_ = [("pilot_samples", C.c_uint64), ("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("seed", C.c_uint64)]


_lib = None


def lib():
    """Load libsgpm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(f"{SO_PATH} is missing: build it with __graft_entry__.build()")
        # PyTorch ships its own HIP runtime; loading it first makes libsgpm bind to
        # that same runtime (same soname), so torch streams and device pointers are
        # valid inside the library and only one runtime owns the device.
        try:
            import torch  # noqa: F401
        except Exception:
            pass
        L = C.CDLL(SO_PATH)
        P = C.c_void_p
        PP = C.POINTER(C.c_void_p)
        st = C.c_int
        sig = {
            "sgpm_create": ([PP, C.c_int, P], st),
            "sgpm_destroy": ([P], st),
            "sgpm_last_error": ([P], C.c_char_p),
            "sgpm_device_count": ([], C.c_int),
            "sgpm_graph_from_csr": ([P, C.c_int64, P, C.c_int, P, C.c_uint32, PP], st),
            "sgpm_graph_stats": ([P, P, P, P, P], st),
            "sgpm_graph_export": ([P, P, P], st),
            "sgpm_graph_free": ([P], st),
            "sgpm_pattern_create": ([P, C.c_int, C.c_int, P, C.c_int, PP], st),
            "sgpm_pattern_plan": ([P, P, P, P, P, P, P, P], st),
            "sgpm_pattern_free": ([P], st),
            "sgpm_options_default": ([C.POINTER(Options)], None),
            "sgpm_estimate": ([P, P, P, C.POINTER(Options), C.POINTER(Result)], st),
            "sgpm_estimate_counted": ([P, P, P, C.POINTER(Options), C.POINTER(Result)], st),
            "sgpm_estimate_batch": ([P, C.c_int, P, P, P, P], st),
            "sgpm_exact_count": ([P, P, P, P, P], st),
            "sgpm_exact_count_noalloc": ([P, P, P, P, P], st),
            "sgpm_gs_sparsify": ([P, P, C.c_uint32, C.c_uint64, C.c_uint32, PP], st),
            "sgpm_bes_sparsify": ([P, P, C.c_uint32, C.c_uint64, C.c_uint32, PP], st),
            "sgpm_model_train": ([P, P, P, C.c_int, P, PP], st),
            "sgpm_model_free": ([P], st),
            "sgpm_model_from_tables": ([P, C.c_int, P, P, PP], st),
            "sgpm_model_table": ([P, C.c_int, P], st),
            "sgpm_model_info": ([P, P, P, P, P], st),
            "sgpm_mlp_forward": ([P, P, P, C.c_int64, P], st),
            "sgpm_mlp_grad": ([P, P, P, P, C.c_int64, P], st),
            "sgpm_mlp_adam_steps": ([P, P, P, P, P, P, C.c_int64, C.c_int64, C.c_float, P], st),
            "sgpm_probe_copy": ([P, C.c_uint64, C.c_int, C.POINTER(C.c_double)], st),
            "sgpm_probe_gather": ([P, C.c_uint64, C.c_int, C.c_int, C.POINTER(C.c_double)], st),
            "sgpm_probe_mlp": ([P, C.c_int64, C.c_int, P], st),
            "sgpm_host_canonicalise": ([C.c_int64, P, C.c_int, P, C.c_uint32, P, P, P, P], st),
            "sgpm_host_plan": ([C.c_int, C.c_int, P, C.c_int, P, P, P, P, P, P, P], st),
            "sgpm_host_normal_quantile": ([C.c_double], C.c_double),
            "sgpm_host_predicted_error": ([C.c_double, C.c_uint64, P, C.c_int, P, C.c_int], C.c_double),
            "sgpm_host_next_window": ([C.c_uint64, C.POINTER(Options)], C.c_uint64),
            "sgpm_host_t_quantile": ([C.c_double, C.c_int], C.c_double),
            "sgpm_host_cost_model": ([C.c_int, C.c_int, P, C.c_int, C.POINTER(CostIn), C.POINTER(CostOut)], C.c_int),
            "sgpm_host_colours_choice": ([C.c_int64, C.c_int, C.c_double], C.c_int),
            "sgpm_host_predicted_error_t": ([C.c_double, C.c_uint64, P, C.c_int, P, C.c_int], C.c_double),
            "sgpm_host_hybrid_choice": ([C.c_double, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double,
                                         C.c_int, P], C.c_int),
            "sgpm_host_ns_cone": ([C.c_int, P, P, P, C.POINTER(Options), P, P, P, P], C.c_int),
        }
        for name, (args, res) in sig.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.argtypes = args
                f.restype = res
        _lib = L
    return _lib


EXPORTED = ["sgpm_create", "sgpm_destroy", "sgpm_last_error", "sgpm_device_count", "sgpm_graph_from_csr",
            "sgpm_graph_stats", "sgpm_graph_export", "sgpm_graph_free", "sgpm_pattern_create", "sgpm_pattern_plan",
            "sgpm_pattern_free", "sgpm_options_default", "sgpm_estimate", "sgpm_estimate_counted",
            "sgpm_estimate_batch", "sgpm_exact_count", "sgpm_exact_count_noalloc", "sgpm_gs_sparsify", "sgpm_bes_sparsify",
            "sgpm_model_train", "sgpm_model_free",
            "sgpm_model_from_tables", "sgpm_model_table", "sgpm_model_info", "sgpm_mlp_forward", "sgpm_mlp_grad",
            "sgpm_mlp_adam_steps",
            "sgpm_probe_copy", "sgpm_probe_gather", "sgpm_probe_mlp", "sgpm_host_canonicalise", "sgpm_host_plan", "sgpm_host_normal_quantile", "sgpm_host_predicted_error",
            "sgpm_host_t_quantile", "sgpm_host_predicted_error_t", "sgpm_host_colours_choice", "sgpm_host_cost_model", "sgpm_host_next_window", "sgpm_host_hybrid_choice",
            "sgpm_host_ns_cone"]


class SgpmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"sgpm status {status}: {msg}")
        self.status = status


def _check(ctx, rc, allow=()):
    if rc != SGPM_OK and rc not in allow:
        msg = lib().sgpm_last_error(ctx).decode() if ctx else ""
        raise SgpmError(rc, msg)
    return rc


# ------------------------------------------------------------------ C-ABI mirrors (same names)
def sgpm_create(device=0, stream=None):
    if stream is None:
        try:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        except Exception:
            stream = 0
    h = C.c_void_p()
    _check(None, lib().sgpm_create(C.byref(h), device, C.c_void_p(stream)))
    return h


def sgpm_destroy(ctx):
    return lib().sgpm_destroy(ctx)


def sgpm_options_default(**kw) -> Options:
    o = Options()
    lib().sgpm_options_default(C.byref(o))
    names = {f[0] for f in Options._fields_}
    for k, v in kw.items():
        if k not in names:
            raise AttributeError(f"sgpm_options has no field {k!r}")
        setattr(o, k, v)
    return o


def sgpm_graph_from_csr(ctx, n, off, nbr, flags=0):
    """off, nbr: host arrays, or device tensors (torch, on the context's
    device: int32 or int64 offsets, int32 neighbours), passed with
    SGPM_DEVICE_PTRS."""
    h = C.c_void_p()
    if hasattr(off, "data_ptr") and getattr(off, "is_cuda", False):
        import torch
        if nbr.dtype != torch.int32 or off.dtype not in (torch.int32, torch.int64):
            raise TypeError("device CSR: offsets int32/int64, neighbours int32")
        off, nbr = off.contiguous(), nbr.contiguous()
        _check(ctx, lib().sgpm_graph_from_csr(ctx, n, C.c_void_p(off.data_ptr()), int(off.dtype == torch.int64),
                                              C.c_void_p(nbr.data_ptr()) if nbr.numel() else None,
                                              flags | SGPM_DEVICE_PTRS, C.byref(h)))
        return h
    off = np.ascontiguousarray(off, dtype=np.int64)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    _check(ctx, lib().sgpm_graph_from_csr(ctx, n, off.ctypes.data, 1, nbr.ctypes.data if len(nbr) else None,
                                          flags, C.byref(h)))
    return h


def sgpm_graph_stats(g):
    n, m, md = C.c_int64(), C.c_int64(), C.c_int64()
    lib().sgpm_graph_stats(g, C.byref(n), C.byref(m), C.byref(md), None)
    perm = np.zeros(max(1, n.value), dtype=np.int32)
    lib().sgpm_graph_stats(g, None, None, None, perm.ctypes.data)
    return int(n.value), int(m.value), int(md.value), perm[:n.value]


def sgpm_graph_export(ctx, g):
    n, m, _, _ = sgpm_graph_stats(g)
    off = np.zeros(n + 1, dtype=np.int64)
    nbr = np.zeros(max(1, 2 * m), dtype=np.int32)
    _check(ctx, lib().sgpm_graph_export(g, off.ctypes.data, nbr.ctypes.data))
    return off, nbr[:2 * m]


def sgpm_graph_free(g):
    return lib().sgpm_graph_free(g)


def sgpm_pattern_create(ctx, k, edges, induced=False):
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    h = C.c_void_p()
    _check(ctx, lib().sgpm_pattern_create(ctx, k, len(e), e.ctypes.data, int(induced), C.byref(h)))
    return h


def sgpm_pattern_plan(p, k):
    order = np.zeros(8, dtype=np.int32)
    arrs = [np.zeros(8, dtype=np.uint8) for _ in range(4)]
    aut, ori = C.c_int32(), C.c_int32()
    lib().sgpm_pattern_plan(p, order.ctypes.data, *[a.ctypes.data for a in arrs], C.byref(aut), C.byref(ori))
    return {"k": k, "oriented": ori.value, "aut": aut.value, "order": order[:k].tolist(),
            "connect": arrs[0][:k].tolist(), "disconnect": arrs[1][:k].tolist(), "upper": arrs[2][:k].tolist(),
            "lower": arrs[3][:k].tolist()}


def sgpm_pattern_free(p):
    return lib().sgpm_pattern_free(p)


def sgpm_estimate(ctx, g, p, opts: Options, counted=False, allow_not_converged=True):
    r = Result()
    f = lib().sgpm_estimate_counted if counted else lib().sgpm_estimate
    allow = (SGPM_NOT_CONVERGED,) if allow_not_converged else ()
    rc = _check(ctx, f(ctx, g, p, C.byref(opts), C.byref(r)), allow)
    return r, rc


def trace_buffer(count):
    return (TraceRec * count)()


def sgpm_estimate_batch(ctx, graphs, patterns, opts_list):
    nq = len(graphs)
    G = (C.c_void_p * nq)(*[g.value for g in graphs])
    P = (C.c_void_p * nq)(*[p.value for p in patterns])
    O = (Options * nq)(*opts_list)
    R = (Result * nq)()
    _check(ctx, lib().sgpm_estimate_batch(ctx, nq, G, P, O, R), (SGPM_NOT_CONVERGED,))
    return list(R)


def sgpm_exact_count(ctx, g, p) -> int:
    lo, hi = C.c_uint64(), C.c_uint64()
    _check(ctx, lib().sgpm_exact_count(ctx, g, p, C.byref(lo), C.byref(hi)))
    return (hi.value << 64) | lo.value


def sgpm_exact_count_noalloc(ctx, g, p) -> int:
    """sgpm_exact_count with its scratch in the library's fixed device array."""
    lo, hi = C.c_uint64(), C.c_uint64()
    _check(ctx, lib().sgpm_exact_count_noalloc(ctx, g, p, C.byref(lo), C.byref(hi)))
    return (hi.value << 64) | lo.value


def sgpm_gs_sparsify(ctx, g, colours, seed, rep):
    h = C.c_void_p()
    _check(ctx, lib().sgpm_gs_sparsify(ctx, g, colours, seed, rep, C.byref(h)))
    return h


def sgpm_bes_sparsify(ctx, g, inv_p, seed, rep):
    h = C.c_void_p()
    _check(ctx, lib().sgpm_bes_sparsify(ctx, g, inv_p, seed, rep, C.byref(h)))
    return h


def sgpm_model_train(ctx, g, patterns, cfg: TrainCfg | None = None):
    P = (C.c_void_p * len(patterns))(*[p.value for p in patterns])
    h = C.c_void_p()
    _check(ctx, lib().sgpm_model_train(ctx, g, P, len(patterns), C.byref(cfg) if cfg else None, C.byref(h)))
    return h


def sgpm_model_free(m):
    return lib().sgpm_model_free(m)


# ------------------------------------------------------------------ host-only utilities
def sgpm_host_canonicalise(n, off, nbr, flags=0):
    off = np.ascontiguousarray(off, dtype=np.int64)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    m = C.c_int64()
    rc = lib().sgpm_host_canonicalise(n, off.ctypes.data, 1, nbr.ctypes.data if len(nbr) else None, flags,
                                      C.byref(m), None, None, None)
    if rc != SGPM_OK:
        raise SgpmError(rc, "host canonicalisation failed")
    o = np.zeros(n + 1, dtype=np.int64)
    nb = np.zeros(max(1, 2 * m.value), dtype=np.int32)
    pm = np.zeros(max(1, n), dtype=np.int32)
    lib().sgpm_host_canonicalise(n, off.ctypes.data, 1, nbr.ctypes.data if len(nbr) else None, flags, None,
                                 o.ctypes.data, nb.ctypes.data, pm.ctypes.data)
    return int(m.value), o, nb[:2 * m.value], pm[:n]


def sgpm_host_plan(k, edges, induced=False):
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    order = np.zeros(8, dtype=np.int32)
    arrs = [np.zeros(8, dtype=np.uint8) for _ in range(4)]
    aut, ori = C.c_int32(), C.c_int32()
    rc = lib().sgpm_host_plan(k, len(e), e.ctypes.data, int(induced), order.ctypes.data,
                              *[a.ctypes.data for a in arrs], C.byref(aut), C.byref(ori))
    if rc != SGPM_OK:
        raise SgpmError(rc, "pattern compile failed")
    return {"k": k, "induced": int(bool(induced)), "oriented": ori.value, "aut": aut.value,
            "order": order[:k].tolist(), "connect": arrs[0][:k].tolist(), "disconnect": arrs[1][:k].tolist(),
            "upper": arrs[2][:k].tolist(), "lower": arrs[3][:k].tolist()}


def sgpm_host_normal_quantile(p):
    return float(lib().sgpm_host_normal_quantile(p))


def sgpm_host_predicted_error(z, n, S1: int, S2: int):
    d1 = np.array([(S1 >> (32 * i)) & 0xFFFFFFFF for i in range(8)], dtype=np.uint32)
    d2 = np.array([(S2 >> (32 * i)) & 0xFFFFFFFF for i in range(12)], dtype=np.uint32)
    return float(lib().sgpm_host_predicted_error(z, n, d1.ctypes.data, 8, d2.ctypes.data, 12))


def sgpm_host_t_quantile(conf, nu):
    return float(lib().sgpm_host_t_quantile(conf, nu))


def sgpm_host_predicted_error_t(t, n, S1: int, S2: int):
    d1 = np.array([(S1 >> (32 * i)) & 0xFFFFFFFF for i in range(8)], dtype=np.uint32)
    d2 = np.array([(S2 >> (32 * i)) & 0xFFFFFFFF for i in range(12)], dtype=np.uint32)
    return float(lib().sgpm_host_predicted_error_t(t, n, d1.ctypes.data, 8, d2.ctypes.data, 12))


def sgpm_host_cost_model(k, edges, cin: CostIn, induced=False) -> CostOut:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    out = CostOut()
    rc = lib().sgpm_host_cost_model(k, len(e), e.ctypes.data, int(bool(induced)), C.byref(cin), C.byref(out))
    if rc != SGPM_OK:
        raise SgpmError(rc, "cost model: pattern compile failed")
    return out


def sgpm_host_colours_choice(m, k, leaves16):
    return int(lib().sgpm_host_colours_choice(m, k, leaves16))


def sgpm_host_next_window(n_t, opts: Options):
    return int(lib().sgpm_host_next_window(n_t, C.byref(opts)))


def sgpm_host_hybrid_choice(ns_lo, eps, gs_reps_run, gs_rep_seconds, gs_cv, gs_reps_max=64, confidence=0.95):
    """(scheme, gs_pred) from the NS cone's lower end and GS pilot figures; see include/sgpm.h."""
    gs = C.c_double()
    rc = lib().sgpm_host_hybrid_choice(ns_lo, eps, confidence, gs_reps_run, gs_rep_seconds, gs_cv, gs_reps_max,
                                       C.byref(gs))
    if rc < 0:
        raise SgpmError(rc, "invalid hybrid pilot figures")
    return rc, gs.value


def sgpm_host_ns_cone(slice_n, slice_seconds, slice_eps_hat, opts: Options):
    """(lo, hi, t0, rate) of the NS time cone from pilot slices; see include/sgpm.h."""
    n = np.ascontiguousarray(slice_n, dtype=np.float64)
    sec = np.ascontiguousarray(slice_seconds, dtype=np.float64)
    eh = np.ascontiguousarray(slice_eps_hat, dtype=np.float64)
    lo, hi, t0, rate = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    rc = lib().sgpm_host_ns_cone(len(n), n.ctypes.data, sec.ctypes.data, eh.ctypes.data, C.byref(opts), C.byref(lo),
                                 C.byref(hi), C.byref(t0), C.byref(rate))
    if rc < 0:
        raise SgpmError(rc, "invalid pilot slices")
    return lo.value, hi.value, t0.value, rate.value


def sgpm_probe_copy(ctx, nbytes, iters=10) -> float:
    v = C.c_double()
    _check(ctx, lib().sgpm_probe_copy(ctx, nbytes, iters, C.byref(v)))
    return v.value


def sgpm_probe_mlp(ctx, N, iters=20):
    """{'fwd_ms', 'fwd_tflops', 'grad_ms', 'grad_tflops'} of the MLP kernels on N rows."""
    out = np.zeros(4, dtype=np.float64)
    _check(ctx, lib().sgpm_probe_mlp(ctx, N, iters, out.ctypes.data))
    return {"fwd_ms": float(out[0]), "fwd_tflops": float(out[1]), "grad_ms": float(out[2]),
            "grad_tflops": float(out[3])}


def sgpm_probe_gather(ctx, working_set_bytes, segment_bytes, rounds=8) -> float:
    v = C.c_double()
    _check(ctx, lib().sgpm_probe_gather(ctx, working_set_bytes, segment_bytes, rounds, C.byref(v)))
    return v.value


# ------------------------------------------------------------------ learned proposal
TABLE_WORDS = 8 * 32 * 32 * 32
MLP_NPARAMS = 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1


def sgpm_model_from_tables(ctx, patterns, tables):
    t = np.ascontiguousarray(np.asarray(tables, dtype=np.uint16).reshape(len(patterns), TABLE_WORDS))
    P = (C.c_void_p * len(patterns))(*[p.value for p in patterns])
    h = C.c_void_p()
    _check(ctx, lib().sgpm_model_from_tables(ctx, len(patterns), P, t.ctypes.data, C.byref(h)))
    return h


def sgpm_model_table(m, i):
    out = np.zeros(TABLE_WORDS, dtype=np.uint16)
    rc = lib().sgpm_model_table(m, i, out.ctypes.data)
    if rc != SGPM_OK:
        raise SgpmError(rc, "model table")
    return out.reshape(8, 32, 32, 32)


def sgpm_model_info(m):
    n = C.c_int()
    lib().sgpm_model_info(m, None, C.byref(n), None, None)
    params = np.zeros(max(1, n.value), dtype=np.float32)
    stats = np.zeros(4, dtype=np.float64)
    tuples = C.c_uint64()
    lib().sgpm_model_info(m, params.ctypes.data, None, stats.ctypes.data, C.byref(tuples))
    return {"params": params[:n.value], "pilot_seconds": float(stats[0]), "train_seconds": float(stats[1]),
            "loss_first": float(stats[2]), "loss_last": float(stats[3]), "tuples": int(tuples.value)}


def sgpm_mlp_forward(ctx, params, X):
    p = np.ascontiguousarray(params, dtype=np.float32)
    x = np.ascontiguousarray(X, dtype=np.float32)
    out = np.zeros(x.shape[0], dtype=np.float32)
    _check(ctx, lib().sgpm_mlp_forward(ctx, p.ctypes.data, x.ctypes.data, x.shape[0], out.ctypes.data))
    return out


def sgpm_mlp_grad(ctx, params, X, y):
    p = np.ascontiguousarray(params, dtype=np.float32)
    x = np.ascontiguousarray(X, dtype=np.float32)
    yy = np.ascontiguousarray(y, dtype=np.float32)
    out = np.zeros(MLP_NPARAMS, dtype=np.float32)
    _check(ctx, lib().sgpm_mlp_grad(ctx, p.ctypes.data, x.ctypes.data, yy.ctypes.data, x.shape[0], out.ctypes.data))
    return out


def sgpm_mlp_adam_steps(ctx, params, m, v, X, y, nsteps, B, lr, beta_pow):
    """Adam on nsteps minibatches of B rows; returns new (params, m, v, beta_pow)."""
    p = np.array(params, dtype=np.float32)
    mm = np.array(m, dtype=np.float32)
    vv = np.array(v, dtype=np.float32)
    bp = np.array(beta_pow, dtype=np.float32)
    x = np.ascontiguousarray(X, dtype=np.float32)
    yy = np.ascontiguousarray(y, dtype=np.float32)
    if x.shape != (nsteps * B, 16) or yy.shape != (nsteps * B,) or p.shape != (MLP_NPARAMS,) or bp.shape != (2,):
        raise ValueError("sgpm_mlp_adam_steps: shapes")
    _check(ctx, lib().sgpm_mlp_adam_steps(ctx, p.ctypes.data, mm.ctypes.data, vv.ctypes.data, x.ctypes.data,
                                          yy.ctypes.data, nsteps, B, lr, bp.ctypes.data))
    return p, mm, vv, bp
