#!/usr/bin/env python3
"""Benchmark: NS-prune time-to-eps and verified samples/s on one MI355X.

Workload: R-MAT scale 20 (2^20 vertices), edge factor 16, (a, b, c) =
(0.57, 0.19, 0.19), symmetrised / deduplicated / loop-free, int32 CSR; queries
4-clique and 5-clique by NS-prune in strict mode at eps = 1 %, 95 % confidence.
One step = both queries run to convergence with a fresh seed.  The graph is
resident on the device before timing starts.

value   = verified samples/s over the timed steps (all samples drawn / wall time)
roofline= the sampling kernel's algorithmic bytes (per-sample figure from the
          instrumented kernel x samples: 8 per first edge, 16 per opened row and 4 per
          entry of every row merged inside the step bounds) / its HIP-event time,
          against the HBM peak.  The time is the union of the launches' event
          intervals: a window queued ahead on the second stream starts while the
          previous one drains, and that overlap is counted once (the exclusive
          time per launch; the raw per-launch event average is reported beside it)
cpu_baseline = the CPU oracle on a bounded sample of the same workload
Every timed run is rerun by the CPU oracle after timing with the same
options; stop point, exact sums and the checksum over all samples must match
("verified").
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-ε (ε=1%, 95% conf) & verified samples/s; learned vs uniform NS"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the sampling kernel's sources (its two files and the types it
    takes, the part of sgpm_internal.h before the kernel declarations);
    counter figures are only reported while it matches the hash they were
    taken with."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2405_03488_amd", "csrc")
    for name in ("ns_kernels.hip", "ns_device.h"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    with open(os.path.join(csrc, "sgpm_internal.h"), "rb") as f:
        h.update(f.read().split(b"// kernels (ns_kernels.hip)")[0])
    return h.hexdigest()[:16]


def measured_traffic(runs, launches):
    """HBM bytes per sampling launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE per sample, scaled by the copy-kernel
    calibration), times the timed runs' samples per launch; None when the
    summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "ns_wave_rmat20_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    per_sample = t["hbm_bytes_per_sample"]
    total = sum(per_sample[x["q"]] * x["r"].n_samples for x in runs)
    return total / max(1, launches)


def other_legs(S, ctx, g, pats, queries, eps):
    """The rest of the hot path on the same graph: the GS engine (colour
    sparsification + exact count, two colourings at c = 16; two Bernoulli edge
    sparsifications at p = 1/16), the loose-mode choice between NS and GS at
    eps, the persistent batch against solo runs, NS-base against NS-prune, and
    the MLP kernels' MFMA throughput."""
    out = {"gs": {}, "hybrid": {}}
    # untimed: the GS kernels' first use in the process (code loading, scratch growth)
    S.sgpm_estimate(ctx, g, pats[queries[0]], S.sgpm_options_default(mode=S.MODE_GS, eps=eps, colours=16,
                                                                     gs_reps_max=2, seed=4))
    for q in queries:
        t0 = time.perf_counter()
        r, _ = S.sgpm_estimate(ctx, g, pats[q], S.sgpm_options_default(mode=S.MODE_GS, eps=eps, colours=16,
                                                                        gs_reps_max=2, seed=5))
        out["gs"][q] = {"colourings": int(r.n_samples), "estimate": r.estimate, "wall_s": time.perf_counter() - t0,
                        "count_kernel_s": r.seconds_kernel, "S1": int(r.S1)}
        t0 = time.perf_counter()
        r, _ = S.sgpm_estimate(ctx, g, pats[q], S.sgpm_options_default(mode=S.MODE_GS, eps=eps, colours=16,
                                                                        gs_reps_max=2, seed=5,
                                                                        gs_scheme=S.GS_BERNOULLI))
        out.setdefault("gs_bernoulli", {})[q] = {"reps": int(r.n_samples), "estimate": r.estimate,
                                                 "wall_s": time.perf_counter() - t0, "count_kernel_s": r.seconds_kernel}
        r, _ = S.sgpm_estimate(ctx, g, pats[q], S.sgpm_options_default(mode=S.MODE_HYBRID, eps=eps, colours=16,
                                                                        seed=6))
        out["hybrid"][q] = {"scheme": "GS" if r.scheme == S.SCHEME_GS else "NS", "ns_cone_s": [r.pred_ns_lo,
                                                                                             r.pred_ns_hi],
                            "gs_pred_s": r.pred_gs, "pilot_s": r.seconds_pilot, "total_s": r.seconds_total}
        # the paper's profiler and cost models choosing instead of the pilots
        r, _ = S.sgpm_estimate(ctx, g, pats[q], S.sgpm_options_default(mode=S.MODE_HYBRID, eps=eps, seed=6,
                                                                        hybrid_selector=S.HYBRID_COST_MODEL))
        out.setdefault("hybrid_cost_model", {})[q] = {
            "scheme": "GS" if r.scheme == S.SCHEME_GS else "NS", "ns_cone_s": [r.pred_ns_lo, r.pred_ns_hi],
            "gs_pred_s": r.pred_gs, "pred_samples": r.pred_samples, "samples": int(r.n_samples),
            "pred_over_actual_samples": r.pred_samples / r.n_samples if r.n_samples else None,
            "profile_s": r.seconds_pilot, "total_s": r.seconds_total, "estimate": r.estimate,
            "eps_hat": r.eps_hat}
    # the persistent batch: both queries x 4 seeds in one launch against the solo runs
    qs = [(q, 3000 + i) for q in queries for i in range(4)]
    bopts = [S.sgpm_options_default(eps=eps, seed=sd, query_tag=i, checksum=1) for i, (q, sd) in enumerate(qs)]
    S.sgpm_estimate_batch(ctx, [g] * len(qs), [pats[q] for q, _ in qs], bopts)  # tunes and captures
    t0 = time.perf_counter()
    solo = [S.sgpm_estimate(ctx, g, pats[q], o)[0] for (q, _), o in zip(qs, bopts)]
    t_solo = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = S.sgpm_estimate_batch(ctx, [g] * len(qs), [pats[q] for q, _ in qs], bopts)
    t_batch = time.perf_counter() - t0
    out["batch"] = {"queries": len(qs), "solo_s": t_solo, "batch_s": t_batch,
                    "identical": all((a.n_samples, a.S1, a.S2, a.checksum) == (b.n_samples, b.S1, b.S2, b.checksum)
                                     for a, b in zip(solo, res)), "tile": [int(r.tile) for r in res]}
    # NS-base (lazy verification, the paper's baseline sampler) against NS-prune
    # at equal samples: hit rate, predicted error, kernel rate, and the samples
    # and time to eps that the error predicts (n (eps_hat / eps)^2)
    out["ns_base_vs_prune"] = {}
    for q in queries:
        row = {}
        for name, smp in (("prune", S.SAMPLER_PRUNE), ("base", S.SAMPLER_BASE)):
            N = 1 << 20
            r, _ = S.sgpm_estimate(ctx, g, pats[q], S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=N, seed=7,
                                                                            sampler=smp, lanes_per_sample=64))
            rate = N / r.seconds_kernel
            need = N * (r.eps_hat / eps) ** 2 if r.eps_hat < float("inf") else None
            row[name] = {"samples": N, "hits": int(r.n_hits), "hit_rate": r.n_hits / N, "eps_hat": r.eps_hat
                         if r.eps_hat < float("inf") else None, "estimate": r.estimate, "samples_per_s": rate,
                         "pred_samples_to_eps": need, "pred_seconds_to_eps": need / rate if need else None}
        out["ns_base_vs_prune"][q] = row
    out["mlp_forward_1M_rows"] = S.sgpm_probe_mlp(ctx, 1 << 20, 10)
    out["mlp_train_batch_16K_rows"] = S.sgpm_probe_mlp(ctx, 1 << 14, 20)
    log(f"gs/hybrid/mlp: {json.dumps(out)}")
    return out


def learned_leg(S, ctx, g, pats, queries, eps, steps, lanes):
    """Learned proposal against uniform NS on the same graph: train the MLP
    proposal on the GPU (pilot samples of every query on their own Philox
    stream), then run both proposals to eps with the same seeds.  Returns
    time-to-eps and samples to the stop for each, and the training cost."""
    t0 = time.perf_counter()
    model = S.sgpm_model_train(ctx, g, [pats[q] for q in queries])
    train_s = time.perf_counter() - t0
    info = S.sgpm_model_info(model)
    # training work: 8 epochs over the tuples (whole minibatches of 2048 rows),
    # forward + backward of the 16-64-64-1 network = 3 x 2 x 5,248 flops per row
    rows = 8 * (info["tuples"] // 2048) * 2048
    flops = rows * 3 * 2 * (16 * 64 + 64 * 64 + 64)
    out = {"train_s": train_s, "pilot_s": info["pilot_seconds"], "tuples": info["tuples"],
           "loss_first": info["loss_first"], "loss_last": info["loss_last"],
           "train_flops": flops, "train_tflops_per_s": flops / max(train_s - info["pilot_seconds"], 1e-9) / 1e12,
           "train_mfma_frac_of_bf16_peak": flops / max(train_s - info["pilot_seconds"], 1e-9) / 2.5e15,
           "queries": {}}
    for q in queries:
        # warm both paths (the learned one runs one sample per wave)
        for prop in (None, model):
            o = S.sgpm_options_default(eps=eps, seed=800, lanes_per_sample=lanes[q] if prop is None else 64,
                                       proposal=prop.value if prop is not None else None)
            S.sgpm_estimate(ctx, g, pats[q], o)
        res = {}
        for name, prop in (("uniform", None), ("learned", model)):
            ts, ns, est, eh = [], [], [], []
            for step in range(steps):
                o = S.sgpm_options_default(eps=eps, seed=2000 + step, checksum=1,
                                           lanes_per_sample=lanes[q] if prop is None else 64,
                                           proposal=prop.value if prop is not None else None)
                r, _ = S.sgpm_estimate(ctx, g, pats[q], o)
                ts.append(r.seconds_total)
                ns.append(int(r.n_samples))
                est.append(float(r.estimate))
                eh.append(float(r.eps_hat))
            res[name] = {"time_to_eps_s": float(np.mean(ts)), "n_stop": ns, "estimate": est, "eps_hat": eh,
                         "samples_per_s": float(sum(ns) / sum(ts))}
        res["time_ratio_learned_over_uniform"] = res["learned"]["time_to_eps_s"] / res["uniform"]["time_to_eps_s"]
        out["queries"][q] = res
        log(f"learned vs uniform {q}: {res['learned']['time_to_eps_s'] * 1e3:.2f} ms "
            f"({np.mean(res['learned']['n_stop']):.0f} samples) vs {res['uniform']['time_to_eps_s'] * 1e3:.2f} ms "
            f"({np.mean(res['uniform']['n_stop']):.0f} samples)")
    S.sgpm_model_free(model)
    return out


def learned_c4_leg(S, synth, ctx, eps, steps):
    """The learned-vs-uniform comparison at the scale its figure is quoted on:
    R-MAT 24 (edge factor 16), 5-clique, same seeds and windows for both."""
    g, gi = load_graph(S, synth, ctx, "rmat24", 1 << 24, lambda: synth.rmat_pairs(24, 16, 0.57, 0.19, 0.19, seed=1))
    pats = {"5-clique": S.sgpm_pattern_create(ctx, *synth.pattern("5-clique"))}
    r, _ = S.sgpm_estimate(ctx, g, pats["5-clique"], S.sgpm_options_default(eps=eps, seed=700))
    lanes = {"5-clique": int(r.lanes_per_sample)}
    out = learned_leg(S, ctx, g, pats, ["5-clique"], eps, steps, lanes)
    out["graph"] = gi
    S.sgpm_pattern_free(pats["5-clique"])
    S.sgpm_graph_free(g)
    return out


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def load_graph(S, synth, ctx, name, n, pairs_fn):
    t0 = time.time()
    pairs = pairs_fn()
    log(f"{name}: {len(pairs)} generated pairs in {time.time() - t0:.1f}s")
    off, nbr = synth.pairs_to_csr(n, pairs)
    del pairs
    g = S.sgpm_graph_from_csr(ctx, n, off, nbr)
    gn, gm, md, _ = S.sgpm_graph_stats(g)
    log(f"{name}: n={gn} m={gm} maxdeg={md}, resident after {time.time() - t0:.1f}s")
    return g, {"name": name, "n": gn, "m": gm, "max_degree": md, "build_s": time.time() - t0}


def workload_c3(S, synth, args):
    """24 queries (the six vertex-induced 4-vertex motifs, the induced 3-path
    and the triangle on three Chung-Lu graphs, gamma 2.1, average degree 32,
    2^18, 2^20 and 2^22 vertices), each to eps at 95 %: the sum of solo runs
    against one persistent batched launch (results must be identical)."""
    ctx = S.sgpm_create(0)
    graphs, info = [], []
    for lg in (18, 20, 22):
        g, gi = load_graph(S, synth, ctx, f"chung-lu 2^{lg}", 1 << lg,
                           lambda lg=lg: synth.chung_lu_pairs(1 << lg, 32, 2.1, lg))
        graphs.append(g)
        info.append(gi)
    motifs = [("3-star", 1), ("4-path", 1), ("tailed-triangle", 1), ("4-cycle", 1), ("diamond", 1), ("4-clique", 1),
              ("wedge", 1), ("triangle", 0)]
    qs = [(g, S.sgpm_pattern_create(ctx, *synth.pattern(m), ind), m, gi) for gi, g in enumerate(graphs)
          for m, ind in motifs]
    cap = 1 << 28

    def opts(i, seed):
        return S.sgpm_options_default(eps=args.eps, seed=seed + i, query_tag=i, checksum=1, max_samples=cap)

    for i, (g, p, m, gi) in enumerate(qs):  # tune lanes per query (cached per graph and plan)
        S.sgpm_estimate(ctx, g, p, opts(i, 7))
    out = {"metric": "C3 batched motif queries: persistent-launch makespan vs sum of solo runs",
           "eps": args.eps, "confidence": 0.95, "max_samples": cap, "graphs": info, "runs": []}
    for seed in (100, 200):
        torch_sync()
        t0 = time.perf_counter()
        solo = [S.sgpm_estimate(ctx, g, p, opts(i, seed))[0] for i, (g, p, _, _) in enumerate(qs)]
        torch_sync()
        t_solo = time.perf_counter() - t0
        t0 = time.perf_counter()
        res = S.sgpm_estimate_batch(ctx, [q[0] for q in qs], [q[1] for q in qs], [opts(i, seed) for i in range(len(qs))])
        torch_sync()
        t_batch = time.perf_counter() - t0
        same = all((a.n_samples, a.S1, a.S2, a.checksum) == (b.n_samples, b.S1, b.S2, b.checksum)
                   for a, b in zip(solo, res))
        run = {"seed": seed, "solo_s": t_solo, "batch_s": t_batch, "identical": same,
               "samples": int(sum(r.n_samples for r in solo)),
               "queries": [{"graph": gi, "motif": m, "n": int(r.n_samples), "converged": int(r.converged),
                            "eps_hat": r.eps_hat, "solo_ms": r.seconds_total * 1e3} for (_, _, m, gi), r in zip(qs, solo)]}
        out["runs"].append(run)
        log(f"c3 seed {seed}: solo {t_solo:.2f}s batch {t_batch:.2f}s identical={same}")
    return out


def workload_c4(S, synth, args):
    """R-MAT 24 (edge factor 16), 5-clique to eps at 95 %: the trained MLP
    proposal against uniform NS-prune, same seeds and windows; training time
    reported separately."""
    ctx = S.sgpm_create(0)
    g, gi = load_graph(S, synth, ctx, "rmat24", 1 << 24, lambda: synth.rmat_pairs(24, 16, 0.57, 0.19, 0.19, seed=1))
    p = S.sgpm_pattern_create(ctx, *synth.pattern("5-clique"))
    t0 = time.perf_counter()
    model = S.sgpm_model_train(ctx, g, [p])
    info = S.sgpm_model_info(model)
    train_s = time.perf_counter() - t0
    log(f"c4: trained in {train_s:.2f}s on {info['tuples']} tuples")
    out = {"metric": "C4 learned vs uniform NS, time-to-eps", "graph": gi, "eps": args.eps, "train_s": train_s,
           "tuples": info["tuples"], "runs": {}}
    for name, prop in (("uniform", None), ("learned", model.value)):
        S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(eps=args.eps, seed=3, proposal=prop))
        rs = []
        for seed in range(10, 13):
            r, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(eps=args.eps, seed=seed, proposal=prop, checksum=1))
            rs.append({"n": int(r.n_samples), "time_s": r.seconds_total, "estimate": r.estimate, "eps_hat": r.eps_hat,
                       "kernel_samples_per_s": r.n_samples / max(r.seconds_kernel, 1e-12)})
        out["runs"][name] = rs
        log(f"c4 {name}: " + ", ".join(f"{x['n']} samples {x['time_s'] * 1e3:.2f} ms" for x in rs))
    S.sgpm_model_free(model)
    return out


def workload_c5(S, synth, args):
    """R-MAT 26 (edge factor 16, about a billion edges, int64 offsets): 6-clique,
    5-cycle and diamond (edge-induced) in loose mode, where pilots choose
    between NS-prune and colour sparsification with 16 colours; then strict NS
    with the learned proposal against uniform on the same seeds."""
    ctx = S.sgpm_create(0)
    g, gi = load_graph(S, synth, ctx, "rmat26", 1 << 26, lambda: synth.rmat_pairs(26, 16, 0.57, 0.19, 0.19, seed=1))
    out = {"metric": "C5 loose-mode estimates on R-MAT 26", "graph": gi, "eps": args.eps, "queries": {}}
    for q in ("6-clique", "5-cycle", "diamond"):
        p = S.sgpm_pattern_create(ctx, *synth.pattern(q))
        log(f"c5 {q} ...")
        r, rc = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_HYBRID, eps=args.eps, colours=16,
                                                                   gs_reps_max=8, seed=4, max_samples=1 << 30))
        out["queries"][q] = {"scheme": "GS" if r.scheme == S.SCHEME_GS else "NS", "estimate": r.estimate,
                             "eps_hat": r.eps_hat, "n": int(r.n_samples), "converged": int(r.converged),
                             "ns_cone_s": [r.pred_ns_lo, r.pred_ns_hi], "gs_pred_s": r.pred_gs,
                             "pilot_s": r.seconds_pilot, "total_s": r.seconds_total,
                             "lanes": r.lanes_per_sample}
        log(f"c5 {q}: {out['queries'][q]}")
    # learned proposal on the NS path: one model for the three patterns, then
    # strict NS with the uniform and the learned proposal on the same seeds
    pats = [S.sgpm_pattern_create(ctx, *synth.pattern(q)) for q in ("6-clique", "5-cycle", "diamond")]
    t0 = time.perf_counter()
    model = S.sgpm_model_train(ctx, g, pats)
    out["learned"] = {"train_s": time.perf_counter() - t0, "tuples": S.sgpm_model_info(model)["tuples"], "runs": {}}
    for q, p in zip(("6-clique", "5-cycle", "diamond"), pats):
        row = {}
        for name, prop in (("uniform", None), ("learned", model.value)):
            r, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(eps=args.eps, seed=9, proposal=prop, checksum=1,
                                                                     max_samples=1 << 30))
            row[name] = {"n": int(r.n_samples), "time_s": r.seconds_total, "estimate": r.estimate,
                         "eps_hat": r.eps_hat, "converged": int(r.converged)}
        row["time_ratio_learned_over_uniform"] = row["learned"]["time_s"] / row["uniform"]["time_s"]
        out["learned"]["runs"][q] = row
        log(f"c5 learned vs uniform {q}: {row}")
    S.sgpm_model_free(model)
    return out


def workload_c1(S, synth, args):
    """ER G(10,000, 80,000) (L2-resident), triangle: 2^30 samples for throughput
    in each lane configuration, then with the lane count autotuned (0); its
    parity with the oracle is a test case."""
    ctx = S.sgpm_create(0)
    n = 10000
    off, nbr = synth.pairs_to_csr(n, synth.er_pairs(n, 80000, 1))
    g = S.sgpm_graph_from_csr(ctx, n, off, nbr)
    k, e = synth.pattern("triangle")
    p = S.sgpm_pattern_create(ctx, k, e)
    out = {"metric": "C1 ER(10000, 80000) triangle samples/s", "throughput": {}}
    for lanes in (64, 16, 4, 1, 0):
        NT = 1 << 30
        r, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=NT, seed=2,
                                                                   lanes_per_sample=lanes))
        out["throughput"][lanes] = {"samples": NT, "estimate": r.estimate, "hits": int(r.n_hits),
                                    "kernel_samples_per_s": NT / r.seconds_kernel,
                                    "wall_samples_per_s": NT / r.seconds_total,
                                    "lanes_used": int(r.lanes_per_sample)}
        log(f"c1 lanes {lanes}: {out['throughput'][lanes]}")
    return out


def workload_coverage(S, synth, args):
    """R-MAT 20, 4-clique and 5-clique: the exact counts (the GS exact count with
    one colour class, i.e. the whole graph), then 100 strict NS runs to eps with
    different seeds: the fraction of 95 % intervals that contain the exact count
    and the stop points reached (the stop rule's coverage)."""
    ctx = S.sgpm_create(0)
    g, gi = load_graph(S, synth, ctx, "rmat20", 1 << 20, lambda: synth.rmat_pairs(20, 16, 0.57, 0.19, 0.19, seed=1))
    out = {"metric": "95 % interval coverage over 100 seeds, R-MAT 20", "graph": gi, "eps": args.eps, "queries": {}}
    for q in ("4-clique", "5-clique"):
        p = S.sgpm_pattern_create(ctx, *synth.pattern(q))
        t0 = time.perf_counter()
        exact = S.sgpm_exact_count(ctx, g, p)
        te = time.perf_counter() - t0
        log(f"coverage {q}: exact {exact} in {te:.2f} s")
        cover, ns, errs = 0, [], []
        for seed in range(100):
            r, _ = S.sgpm_estimate(ctx, g, p, S.sgpm_options_default(eps=args.eps, seed=1000 + seed))
            cover += int(r.ci_lo <= exact <= r.ci_hi)
            ns.append(int(r.n_samples))
            errs.append(abs(r.estimate - exact) / exact)
        out["queries"][q] = {"exact": exact, "exact_count_s": te, "coverage": cover / 100,
                             "n_stop": sorted(set(ns)), "mean_rel_err": sum(errs) / len(errs),
                             "max_rel_err": max(errs)}
        log(f"coverage {q}: {out['queries'][q]}")
    return out


def torch_sync():
    import torch
    torch.cuda.synchronize()


WORKLOADS = {"c1": workload_c1, "c3": workload_c3, "c4": workload_c4, "c5": workload_c5,
             "coverage": workload_coverage}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--eps", type=float, default=0.01)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-probes", action="store_true", help="skip the measured copy/gather rooflines")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-uniform leg")
    ap.add_argument("--no-c4", action="store_true", help="skip the R-MAT 24 learned-vs-uniform leg")
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "coverage"],
                    help="c1: ER triangle throughput; "
                         "c2 (default): R-MAT 20 4-/5-clique, the benchmark line; c3: 24 motif queries on three "
                         "Chung-Lu graphs, batch vs solo; c4: R-MAT 24 5-clique, learned vs uniform; c5: R-MAT 26 "
                         "6-clique, 5-cycle, diamond in loose (hybrid) mode; coverage: exact counts and the 95 %% "
                         "intervals of 100 seeds on R-MAT 20")
    ap.add_argument("--counters-run-gs", action="store_true",
                    help="for counter runs: the 256 MiB calibration copy, then one exact count of the 4-clique, "
                         "5-clique and diamond on R-MAT 20 colour-sparsified with c = 16 (seed 11, colouring 0)")
    ap.add_argument("--counters-run", action="store_true",
                    help="short run for hardware counters: one 256 MiB copy, then one 4M-sample window per query")
    ap.add_argument("--counters-learned", action="store_true",
                    help="with --counters-run: also train the MLP proposal and run one 4M-sample learned window "
                         "per query")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding is a "
              "design note, not built.", file=sys.stderr)
        sys.exit(2)

    from paper_2405_03488_amd import sgpm as S
    from paper_2405_03488_amd import synth

    if S.lib().sgpm_device_count() < 1:
        log("no HIP device visible")
        sys.exit(1)
    import torch  # device memory / stream plumbing only
    torch.cuda.init()
    if args.workload != "c2":
        print(json.dumps(WORKLOADS[args.workload](S, synth, args)), flush=True)
        return

    t0 = time.time()
    scale = args.scale
    n = 1 << scale
    pairs = synth.rmat_pairs(scale, 16, 0.57, 0.19, 0.19, seed=1)
    off, nbr = synth.pairs_to_csr(n, pairs)
    ctx = S.sgpm_create(0)
    g = S.sgpm_graph_from_csr(ctx, n, off, nbr)
    gn, gm, maxdeg, _ = S.sgpm_graph_stats(g)
    log(f"graph rmat{scale}: n={gn} m={gm} maxdeg={maxdeg} built in {time.time() - t0:.1f}s")

    queries = ["4-clique", "5-clique"]
    pats = {q: S.sgpm_pattern_create(ctx, *synth.pattern(q)) for q in queries}

    if args.counters_run_gs:
        S.sgpm_probe_copy(ctx, 256 << 20, 1)
        sp = S.sgpm_gs_sparsify(ctx, g, 16, 11, 0)
        for q in ("4-clique", "5-clique", "diamond"):
            pq = pats[q] if q in pats else S.sgpm_pattern_create(ctx, *synth.pattern(q))
            tc = time.perf_counter()
            cnt = S.sgpm_exact_count(ctx, sp, pq)
            log(f"{q}: exact count {cnt} on the sparsified graph in {1e3 * (time.perf_counter() - tc):.2f} ms")
        S.sgpm_graph_free(sp)
        return

    if args.counters_run:
        S.sgpm_probe_copy(ctx, 256 << 20, 1)
        for q in queries:
            o = S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=4 << 20, seed=1000, checksum=1,
                                       lanes_per_sample=64)
            r, _ = S.sgpm_estimate(ctx, g, pats[q], o)
            log(f"{q}: {r.n_samples} samples, kernel {r.seconds_kernel * 1e3:.3f} ms over {r.launches} launch(es)")
        if args.counters_learned:
            model = S.sgpm_model_train(ctx, g, [pats[q] for q in queries])
            for q in queries:
                o = S.sgpm_options_default(mode=S.MODE_FIXED_N, fixed_n=4 << 20, seed=1000, checksum=1,
                                           proposal=model.value)
                r, _ = S.sgpm_estimate(ctx, g, pats[q], o)
                log(f"{q} learned: {r.n_samples} samples, kernel {r.seconds_kernel * 1e3:.3f} ms")
            S.sgpm_model_free(model)
        return

    def opts_for(q, seed, lanes):
        return S.sgpm_options_default(eps=args.eps, confidence=0.95, seed=seed, checksum=1, lanes_per_sample=lanes,
                                      query_tag=0)

    # warmup: also picks the lane count per query (autotuner on the first window)
    lanes = {q: 0 for q in queries}
    warm_launches = 0
    for w in range(max(1, args.warmup)):
        for q in queries:
            o = opts_for(q, 900 + w, lanes[q])
            r, _ = S.sgpm_estimate(ctx, g, pats[q], o)
            lanes[q] = r.lanes_per_sample
            warm_launches += r.launches
            log(f"warmup {q}: n={r.n_samples} est={r.estimate:.6g} eps_hat={r.eps_hat:.4g} lanes={r.lanes_per_sample}"
                f" t={r.seconds_total:.4f}s")

    runs = []
    torch.cuda.synchronize()
    t_begin = time.perf_counter()
    for step in range(args.steps):
        for q in queries:
            seed = 1000 + step
            o = opts_for(q, seed, lanes[q])
            r, rc = S.sgpm_estimate(ctx, g, pats[q], o)
            runs.append({"q": q, "seed": seed, "r": r, "rc": rc, "opts": o})
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    wall = t_end - t_begin
    total_samples = sum(x["r"].n_samples for x in runs)
    kernel_s = sum(x["r"].seconds_kernel for x in runs)
    # device time with at least one sampling kernel running (estimates run one after another)
    busy_s = sum(x["r"].seconds_kernel_busy for x in runs)
    launches = sum(x["r"].launches for x in runs)

    # algorithmic bytes per sample, from the instrumented kernel on step 0's samples
    bps = {}
    for q in queries:
        o = opts_for(q, 1000, lanes[q])
        o.mode = S.MODE_FIXED_N
        o.fixed_n = int(next(x["r"].n_samples for x in runs if x["q"] == q))
        r, _ = S.sgpm_estimate(ctx, g, pats[q], o, counted=True)
        bps[q] = r.bytes / max(1, r.n_samples)
    alg_bytes = sum(bps[x["q"]] * x["r"].n_samples for x in runs)
    # per launch: exclusive time (the union of the launches' intervals / launches)
    achieved = alg_bytes / busy_s / 1e9 if busy_s > 0 else 0.0

    learned = None if args.no_learned else learned_leg(S, ctx, g, pats, queries, args.eps, args.steps, lanes)
    other = None if args.no_learned else other_legs(S, ctx, g, pats, queries, args.eps)
    c4 = None if args.no_learned or args.no_c4 else learned_c4_leg(S, synth, ctx, args.eps, max(3, args.steps))

    probes = None
    if not args.no_probes:
        footprint = (gn + 1) * 8 + 2 * gm * 4 + gm * 8  # offsets + rows + oriented edge pairs
        probes = {"hbm_copy_GBs": S.sgpm_probe_copy(ctx, 1 << 30, 5),
                  "working_set_bytes": footprint}
        for seg in (64, 256):
            probes[f"gather_{seg}B_GBs"] = S.sgpm_probe_gather(ctx, footprint, seg, 16)
        log(f"probes: {probes}")

    per_q = {}
    for q in queries:
        rs = [x["r"] for x in runs if x["q"] == q]
        per_q[q] = {"time_to_eps_s": float(np.mean([r.seconds_total for r in rs])),
                    "n_stop": [int(r.n_samples) for r in rs], "estimate": [float(r.estimate) for r in rs],
                    "eps_hat": [float(r.eps_hat) for r in rs], "hit_rate": float(np.mean([r.n_hits / r.n_samples
                                                                                          for r in rs])),
                    "converged": all(r.converged for r in rs), "lanes_per_sample": lanes[q],
                    "windows": [int(r.windows) for r in rs],
                    "device_span_s": float(np.mean([r.seconds_sampling for r in rs])),
                    "kernel_s": float(np.mean([r.seconds_kernel for r in rs])),
                    "kernel_busy_s": float(np.mean([r.seconds_kernel_busy for r in rs])),
                    "bytes_per_sample": bps[q]}

    # CPU leg: oracle baseline and verification of the timed runs
    cpu = None
    cpu_bytes = None
    verified = None
    if not args.no_cpu:
        from oracle import oracle as O
        tc = time.time()
        og = O.OGraph.from_raw_csr(n, off, nbr)
        log(f"oracle graph built in {time.time() - tc:.1f}s")
        # every timed run again in the oracle, same options: the stop point,
        # the exact sums and the checksum over all samples must be identical
        verified = True
        tv = time.perf_counter()
        cpu_tte = {}
        for x in runs:
            k, e = synth.pattern(x["q"])
            op = O.compile_plan(k, e)
            so = x["opts"]
            t_o = time.perf_counter()
            orr = O.run(og, op, O.make_opts(eps=so.eps, confidence=so.confidence, seed=so.seed, tag=so.query_tag,
                                            n_min=so.n_min, w_min=so.w_min, quantum=so.quantum,
                                            max_samples=so.max_samples, growth=so.window_growth))
            cpu_tte.setdefault(x["q"], []).append(time.perf_counter() - t_o)
            r = x["r"]
            if (orr.n, orr.S1, orr.S2, orr.hits, orr.checksum) != (r.n_samples, r.S1, r.S2, r.n_hits, r.checksum):
                verified = False
                log(f"verification failed: {x['q']} seed {x['seed']}")
        log(f"verified {len(runs)} timed runs against the oracle in {time.perf_counter() - tv:.1f}s")
        k, e = synth.pattern("4-clique")
        op = O.compile_plan(k, e)
        th = O.nthreads()
        cal = 200000
        tc = time.perf_counter()
        O.run(og, op, O.make_opts(fixed_n=cal, seed=5, threads=th))
        dt = time.perf_counter() - tc
        N = max(cal, int(cal * args.cpu_seconds / max(dt, 1e-6)))
        tc = time.perf_counter()
        orr = O.run(og, op, O.make_opts(fixed_n=N, seed=6, threads=th))
        dt = time.perf_counter() - tc
        cpu = {"value": N / dt, "unit": "samples/s", "cores": th, "kind": "oracle",
               "sample": f"4-clique NS-prune on the same rmat{scale} graph, fixed {N} samples (seed 6), "
                         f"{dt:.1f}s on {th} threads"}
        log(f"cpu oracle: {N / dt:.4g} samples/s ({N} samples, {dt:.1f}s, {th} threads)")
        # the same oracle on one core, on a sample of about a tenth of the time
        N1 = max(20000, int(N / max(1, th) / 10))
        tc = time.perf_counter()
        O.run(og, op, O.make_opts(fixed_n=N1, seed=7, threads=1))
        dt1 = time.perf_counter() - tc
        cpu["single_core"] = {"value": N1 / dt1, "unit": "samples/s", "cores": 1,
                              "sample": f"fixed {N1} samples (seed 7), {dt1:.1f}s on 1 thread"}
        cpu["host"] = {"nproc": os.cpu_count(), "cpu_model": host_cpu_model()}
        # the oracle's time to eps on the same windows (the verification reruns above:
        # same seeds and window schedule, hence the same stop points as the GPU)
        cpu["time_to_eps_s"] = {q: float(np.mean(v)) for q, v in cpu_tte.items()}
        cpu["time_to_eps_runs"] = {q: len(v) for q, v in cpu_tte.items()}
        cpu["time_to_eps_cores"] = O.nthreads()
        log(f"cpu oracle, one core: {N1 / dt1:.4g} samples/s ({N1} samples, {dt1:.1f}s)")
        # algorithmic bytes per sample (the measurement definition the roofline
        # uses), by the step at which the sample ended, from the oracle's records
        bdist = {}
        for q in queries:
            kq, eq = synth.pattern(q)
            opq = O.compile_plan(kq, eq)
            ends = {}
            allb = []
            minb = []
            for sid in range(20000):
                rec = O.sample(og, opq, 1, 0, sid)
                key = "hit" if rec.hit else f"ended at step {rec.fail_step}"
                ends.setdefault(key, []).append(int(rec.bytes))
                allb.append(int(rec.bytes))
                minb.append(int(rec.bytes_min))
            a = np.array(allb, dtype=np.float64)
            bdist[q] = {"definition": "8 first edge + 16 per opened row + 4 per entry of every merged row inside "
                                      "the step bounds",
                        "samples": len(allb), "mean": float(a.mean()), "p50": float(np.percentile(a, 50)),
                        "p90": float(np.percentile(a, 90)), "p99": float(np.percentile(a, 99)), "max": float(a.max()),
                        "mean_smallest_row_only": float(np.mean(minb)),
                        "by_end": {k2: {"samples": len(v), "mean": float(np.mean(v))} for k2, v in sorted(ends.items())}}
        cpu_bytes = bdist
        # the GS exact count's algorithmic bytes (every node of the search tree)
        # on the GS leg's two colourings, from the oracle, against the count
        # kernels' time in that leg
        if other is not None and other.get("gs"):
            gsr = {}
            for q in queries:
                kq, eq = synth.pattern(q)
                opq = O.compile_plan(kq, eq)
                t0 = time.perf_counter()
                reps = range(int(other["gs"][q]["colourings"]))
                gb = sum(O.gs_count_bytes(og, opq, 16, 5, r) for r in reps)
                # the same colourings counted by the oracle: S1 = sum of 16^(k-1) Y_r
                s1 = sum(O.gs_count(og, opq, 16, 5, r) * 16 ** (kq - 1) for r in reps)
                kt = other["gs"][q]["count_kernel_s"]
                gsr[q] = {"alg_bytes": gb, "count_kernel_s": kt, "achieved_GBs": gb / kt / 1e9 if kt > 0 else None,
                          "frac_of_hbm_peak": gb / kt / 1e9 / HBM_PEAK_GBS if kt > 0 else None,
                          "counts_equal_oracle": s1 == other["gs"][q]["S1"],
                          "oracle_s": time.perf_counter() - t0}
                log(f"gs count {q}: {gb} algorithmic bytes in {kt * 1e3:.2f} ms of count kernels; "
                    f"sums equal the oracle's: {s1 == other['gs'][q]['S1']}")
            other["gs_count_roofline"] = gsr

    value = total_samples / wall
    traffic = measured_traffic(runs, launches)
    avg_launch_s = busy_s / max(1, launches)
    gather = (probes or {}).get("gather_64B_GBs")
    line = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u128", "data": "synthetic",
        "config": {"workload": f"rmat{scale}-ef16 (a,b,c)=(.57,.19,.19) 4-clique+5-clique NS-prune strict "
                               f"eps={args.eps} conf=0.95", "n": gn, "m": gm, "queries": queries},
        "verified": verified,
        "time_to_eps_s": {q: per_q[q]["time_to_eps_s"] for q in queries},
        "queries": per_q,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     # the counted HBM traffic as a rate, and the algorithmic and traffic rates against the
                     # measured random 64-B gather rate over the same working set (the bound that applies)
                     "traffic_GBs": traffic / avg_launch_s / 1e9 if traffic else None,
                     "frac_of_gather_probe": achieved / gather if gather else None,
                     "traffic_frac_of_gather_probe": traffic / avg_launch_s / 1e9 / gather
                     if (traffic and gather) else None,
                     "kernel": sorted({"ns_wave_kernel" if lanes[q] == 64 else f"ns_window_kernel<{lanes[q]}>"
                                       for q in queries}),
                     "frac_smallest_row_bytes": (achieved / HBM_PEAK_GBS * sum(
                         cpu_bytes[q]["mean_smallest_row_only"] / cpu_bytes[q]["mean"] for q in queries) / len(queries))
                     if cpu_bytes else None,
                     "launches": launches,
                     "avg_launch_ms": busy_s / max(1, launches) * 1e3,
                     "avg_launch_ms_events_raw": kernel_s / max(1, launches) * 1e3,
                     "kernel_busy_ms_per_step": busy_s / args.steps * 1e3,
                     "sampling_launches_before_timed": warm_launches,
                     "alg_bytes_per_launch": alg_bytes / max(1, launches),
                     "measured": probes},
        "cpu_baseline": cpu,
        "bytes_per_sample": cpu_bytes,
        "learned_vs_uniform": learned,
        "learned_vs_uniform_c4": c4,
        "gs_hybrid_mlp": other,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
