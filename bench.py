#!/usr/bin/env python3
"""Benchmark: one clustering path of the convex clustering model on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input
already resident in HBM: the exact k-NN Gaussian weight graph
(ccm_build_knn_graph) followed by the warm-started SSNAL path over the gamma
grid to relative KKT <= 1e-6 (ccm_solve_path: edge gather, per-edge
projection, atomic-free B^T scatter, Newton-CG matvecs, line search, KKT
tests, cluster labels).  The reported value is the wall time of that step.

Default workload: n = 10,000 points in d = 64 drawn from 10 Gaussians
(sigma 1, centres N(0, 25 I)), k = 10, phi = 1 / median k-NN distance,
q = 2, 20 gammas log-spaced in [1e-3, 1e2].

The roofline object reports the Newton/CG matvec (the dominant kernel):
algorithmic bytes of the launches that did work in the timed steps divided
by their summed HIP-event durations (recorded by the library on its launch
stream).  The cpu_baseline object times the oracle (CPU, FP64) on a bounded
sample of the same workload and scales it to one path.

The same JSON line also reports the growth forms beside the plain path:
"adjoint" (n = 20000, d = 32: tight forward solve + VJP) and "batched" (512
instances of uneven n, d and q, 10 gammas each, one batched call).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure

WORKLOADS = {
    "mixture64_n10000": dict(gen="mixture64", kw=dict(), k=10, phi=0.0, q=2.0,
                             gammas=(-3.0, 2.0, 20), tol=1e-6,
                             desc="n=10000 d=64 10 Gaussians (sigma 1, centres N(0,25I)), "
                                  "k=10 Gaussian weights phi=1/median, q=2, 20 gammas "
                                  "log-spaced [1e-3,1e2], SSNAL to KKT 1e-6"),
    "blobs2d_n200": dict(gen="blobs2d", kw=dict(), k=10, phi=0.5, q=2.0,
                         gammas=(-3.0, 1.0, 10), tol=1e-6,
                         desc="n=200 d=2 4 blobs, k=10 w=exp(-0.5 d^2), q=2, 10 gammas "
                              "[1e-3,1e1], SSNAL to KKT 1e-6"),
    "images784_n100000": dict(gen="images784", kw=dict(), k=10, phi=0.0, q=2.0,
                              gammas=(-3.0, 1.0, 15), tol=1e-6, codes=1.0 / 255.0,
                              desc="n=100000 d=784 10 image classes quantised to k/255, k=10 "
                                   "graph from exact integer distances of the 8-bit codes "
                                   "(int8 MFMA), q=2, 15 gammas [1e-3,1e1], SSNAL to KKT 1e-6"),
}

METRIC = "path wall-time @KKT 1e-6 + edge-op HBM GB/s %peak; plain vs batched/adjoint"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_points(wl):
    """(A, K): the points, and their 8-bit codes when the workload's graph is
    built from them (else None)."""
    import synthdata
    gen = getattr(synthdata, wl["gen"])
    out = gen(**wl["kw"])
    return out[0], (out[2] if wl.get("codes") else None)


def traffic_record(kernel_key):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    runs, valid only while the kernel source is unchanged."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel_key)
    except Exception:
        return None
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if h != rec["source_sha256"]:
        return None
    return rec


def cpu_baseline(A_np, K_np, wl, graph, budget_s=20.0):
    """The oracle on a bounded sample: k-NN rows and an evenly spaced subset
    of the gammas (each warm-started from the previous sampled gamma), scaled
    to one full step.  The solve sample runs on `graph` (the step's own graph,
    copied to the host; building it is not part of the sample)."""
    import oracle
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(1)
    except Exception:
        lim = None
    n = A_np.shape[0]
    k = wl["k"]
    # k-NN: a sample of query rows, scaled by n / rows
    nrows = 200 if n * A_np.shape[1] <= 2e7 else 8
    rows = np.arange(0, n, max(1, n // nrows))
    t0 = time.perf_counter()
    if K_np is not None:
        oracle.knn_brute_u8(K_np, k, rows=rows, block=1)
    else:
        oracle.knn_brute(A_np, k, rows=rows)
    t_knn = (time.perf_counter() - t0) * n / len(rows)
    src, dst, w = graph
    lo, hi, cnt = wl["gammas"]
    gam = np.logspace(lo, hi, int(cnt))
    stride = 5 if cnt >= 10 else 1
    sample = gam[::stride]
    X = U = None
    t_solve = 0.0
    done = 0
    for g in sample:
        t0 = time.perf_counter()
        X, U, _, info = oracle.ssnal(A_np, src, dst, w, g, wl["q"], wl["tol"], X0=X, U0=U)
        t_solve += time.perf_counter() - t0
        done += 1
        if t_solve > budget_s:
            break
    per_gamma = t_solve / max(done, 1)
    value = t_knn + per_gamma * cnt
    if lim is not None:
        lim.unregister() if hasattr(lim, "unregister") else None
    return dict(value=round(value, 3), unit="s", cores=1, kind="oracle",
                sample=(f"oracle k-NN on {len(rows)} of {n} query rows (x{n/len(rows):.0f}) + "
                        f"SSNAL on {done} of {cnt} gammas (every {stride}th, warm-started from "
                        f"the previous sampled gamma; mean per gamma x{cnt}); single thread"),
                measured_s=round(t_knn * len(rows) / n + t_solve, 3))


def batched_leg(ccm, torch, count, budget_s):
    """512 independent instances (uneven n, d, q), 10 gammas each, one call."""
    import synthdata
    insts = synthdata.instances(count=count)
    dev = []
    for it in insts:
        A = torch.from_numpy(it["A"]).cuda()
        src, dst, w, _ = ccm.ccm_build_knn_graph(A, 10, 0.0)
        dev.append(dict(A=A, src=src, dst=dst, w=w, q=it["q"]))
    torch.cuda.synchronize()
    g = np.logspace(-3, 1, 10)
    o = ccm.ccm_default_options(time_budget_s=budget_s)
    t0 = time.perf_counter()
    res = ccm.ccm_solve_path_batched(dev, g, 1e-6, opts=o)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = np.array([r["status"] for r in res])              # [instances, gammas]
    kk = np.array([r["kkt"][:, :3].max(axis=1) for r in res])  # per (instance, gamma)
    conv = int((st == 0).sum())
    return {"workload": f"instances{count}: n~U[100,5000], d in {{2,8,32,128}}, q in {{1,2,inf}}, "
                        "k=10, 10 gammas [1e-3,1e1], SSNAL to per-instance KKT 1e-6",
            "instances": count, "sum_n": int(sum(i["n"] for i in insts)),
            "sum_m": int(sum(int(x["src"].numel()) for x in dev)),
            "seconds": round(el, 3), "instance_paths_per_s": round(count / el, 2),
            "converged_pairs": conv, "total_pairs": int(st.size),
            "max_kkt_converged": float(kk[st == 0].max()) if conv else None,
            "status_counts": [int(c) for c in np.bincount(st.ravel(), minlength=4)],
            "time_budget_s": budget_s}


def adjoint_leg(ccm, torch):
    """n = 20000, d = 32, 8 blobs, q = 2, gamma = 0.5: tight forward solve +
    VJP of L = sum ||x_i - t_i||^2 with respect to A, log w and gamma."""
    import synthdata
    A_np, _, T_np = synthdata.mixture32()
    A = torch.from_numpy(A_np).cuda()
    T = torch.from_numpy(T_np).cuda()
    src, dst, w, _ = ccm.ccm_build_knn_graph(A, 10, 0.0)

    def run():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ccm.ccm_solve_path(A, src, dst, w, [0.5], 2.0, 1e-10)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        X = out["X"][0]
        dA, dlw, dg, it = ccm.ccm_path_vjp(A, src, dst, w, 0.5, X, out["labels"][0],
                                           2 * (X - T), tol=1e-12)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return out, t1 - t0, t2 - t1, dg, it

    # the first call in a process also loads the kernels' code objects (a
    # one-time cost, reported apart); the timed figures are the second call
    _, f0, v0, _, _ = run()
    out, f1, v1, dg, it = run()
    return {"workload": "mixture32_n20000: n=20000 d=32 8 Gaussians, k=10, q=2, gamma=0.5, "
                        "L=sum||x_i-t_i||^2",
            "m": int(src.numel()), "forward_seconds": round(f1, 4),
            "forward_kkt": float(out["kkt"][0][:3].max()), "clusters": int(out["n_clusters"][0]),
            "vjp_seconds": round(v1, 4), "vjp_cg_iterations": int(it),
            "first_call_seconds": {"forward": round(f0, 4), "vjp": round(v0, 4)},
            "dL_dgamma": dg}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mixture64_n10000", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-instances leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--batched-count", type=int, default=512)
    ap.add_argument("--batched-budget", type=float, default=90.0,
                    help="wall-clock budget (s) of each (q, d) group of the batched leg")
    ap.add_argument("--locality", type=int, default=-1, choices=(-1, 0, 1),
                    help="vertex processing order of the library (-1: its default)")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without HIP events around the matvec launches (roofline then "
                         "omitted)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the path solver is "
                                   "a single-device program (multi-GPU sharding is a design "
                                   "note only)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_2501_15964_amd as ccm

    wl = WORKLOADS[args.workload]
    A_np, K_np = make_points(wl)
    n, d = A_np.shape
    lo, hi, cnt = wl["gammas"]
    gammas = np.logspace(lo, hi, int(cnt))
    dev = torch.device("cuda:0")
    A = torch.from_numpy(A_np).to(dev)
    K = torch.from_numpy(K_np).to(dev) if K_np is not None else None
    torch.cuda.synchronize()
    # timed steps: HIP events around the Newton/CG matvec launches only (profile
    # level 2), which the roofline figure needs; one extra untimed step with
    # every kernel class timed (level 1) gives the per-class breakdown
    opts = ccm.ccm_default_options(profile=0 if args.no_profile else 2, locality=args.locality)
    opts_all = ccm.ccm_default_options(profile=1, locality=args.locality)

    def step(o=opts):
        t0 = time.perf_counter()
        if K is not None:
            src, dst, w, phi = ccm.ccm_build_knn_graph_u8(K, wl["codes"], wl["k"], wl["phi"])
        else:
            src, dst, w, phi = ccm.ccm_build_knn_graph(A, wl["k"], wl["phi"])
        t1 = time.perf_counter()
        out = ccm.ccm_solve_path(A, src, dst, w, gammas, wl["q"], wl["tol"], opts=o)
        t2 = time.perf_counter()
        return out, (t1 - t0), (t2 - t1), int(src.numel()), phi, (src, dst, w)

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(step())
        log(f"step {i + 1}/{args.steps}: {results[-1][1] + results[-1][2]:.3f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1000.0 * elapsed / args.steps

    out, _, _, m, phi, graph_dev = results[-1]
    kkt_max = float(np.max(out["kkt"][:, :3]))
    status = [int(s) for s in out["status"]]
    knn_ms = 1000.0 * float(np.mean([r[1] for r in results]))
    path_ms = 1000.0 * float(np.mean([r[2] for r in results]))

    roofline = None
    kern = None
    if not args.no_profile:
        mv_ms = mv_bytes = 0.0
        mv_calls = 0
        for r in results:
            for st in r[0]["stats"]:
                mv_ms += st["kern_ms"][2]
                mv_calls += st["kern_calls"][2]
                mv_bytes += st["matvec_bytes"]
        # per-class breakdown from one extra, untimed step with every class timed
        extra = step(opts_all)
        cls_ms = np.zeros(5)
        cls_calls = np.zeros(5, dtype=np.int64)
        for st in extra[0]["stats"]:
            cls_ms += np.array(st["kern_ms"])
            cls_calls += np.array(st["kern_calls"])
        if mv_ms > 0 and mv_calls > 0:
            avg_s = mv_ms / 1000.0 / mv_calls
            bytes_per_launch = mv_bytes / mv_calls
            achieved = bytes_per_launch / avg_s / 1e9
            rec = traffic_record(f"k_matvec_q2/{args.workload}")
            roofline = {"bound": "hbm", "kernel": "k_matvec (Newton/CG matvec, q=2)",
                        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": (rec["bytes_per_launch"] if rec else None),
                        "avg_launch_us": round(avg_s * 1e6, 2),
                        "launches": int(mv_calls),
                        "algorithmic_bytes_per_launch": round(bytes_per_launch)}
        names = ["edge", "scatter", "matvec", "cg_update", "other"]
        kern = {names[c]: {"ms": round(float(cls_ms[c]), 3), "launches": int(cls_calls[c])}
                for c in range(5)}
        kern["note"] = "one untimed step with every kernel class timed (HIP events)"

    # achievable copy bandwidth of the same device (calibration, untimed)
    buf_a = torch.empty(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
    buf_b = torch.empty_like(buf_a)
    ms_copy = ccm.ccm_stream_copy(buf_a, buf_b, buf_a.numel() * 8, repeats=10)
    copy_gbs = 2 * buf_a.numel() * 8 / (ms_copy / 1e3) / 1e9
    del buf_a, buf_b

    rec = {
        "metric": METRIC,
        "value": round(ms_per_step / 1000.0, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "desc": wl["desc"], "n": n, "d": d,
                   "k": wl["k"], "m": m, "phi": phi, "q": wl["q"], "n_gamma": int(cnt),
                   "tol": wl["tol"], "method": "ssnal", "parallelism": "single-gpu"},
        "phases_ms": {"knn_graph": round(knn_ms, 2), "path": round(path_ms, 2)},
        "max_kkt": kkt_max,
        "status": status,
        "n_clusters": [int(c) for c in out["n_clusters"]],
        "iterations": {"newton": int(sum(s["newton"] for s in out["stats"])),
                       "cg": int(sum(s["cg"] for s in out["stats"])),
                       "outer": int(sum(s["outer"] for s in out["stats"]))},
        "roofline": roofline,
        "kernels_per_step": kern,
        "copy_kernel_gbs": round(copy_gbs, 1),
        "cpu_baseline": None,
    }
    if not args.no_adjoint:
        log("adjoint leg ...")
        rec["adjoint"] = adjoint_leg(ccm, torch)
    if not args.no_batched:
        log("batched leg ...")
        rec["batched"] = batched_leg(ccm, torch, args.batched_count, args.batched_budget)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample) ...")
        graph = tuple(t.cpu().numpy() for t in graph_dev)
        rec["cpu_baseline"] = cpu_baseline(A_np, K_np, wl, graph)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
