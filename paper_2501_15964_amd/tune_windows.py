"""Window tuner for the vertex kernels (run on the GPU; writes the table the
library is compiled with).

The vertex kernels (B^T, the fused edge pass, the Newton matvec) give each
workgroup a window of whole vertices holding about GPB x chunk incidences,
where GPB is the number of row groups of a workgroup and chunk the
incidences per row group.  The chunk trades the LDS fix-up of vertices cut
between row groups and the tail of the launch against the incidence data
loaded per round.  For every row layout of the library (a range of row
widths d) and every q this script times the Newton/CG matvec over a sweep of
chunks on a synthetic k-NN graph (10 Gaussian blobs, k = 10, Gaussian
weights, about 80 M row values, i.e. n = 1e5 at d = 784, so that the rows
do not fit in the last-level cache; at most 2e5 points), with the matvec
launches timed by the library's own HIP events (ccm_options.profile = 2),
and writes the fastest chunk of each (layout, q) into
csrc/tuned_windows.hpp.  The table is then
compiled into the library, so a run never depends on timing noise: the
chunk changes the summation order of cut vertices, and the library's
results are bit-reproducible for a given build.

Usage: python -m paper_2501_15964_amd.tune_windows [--layouts 0,1,..]
[--header FILE] [--out FILE.md] [--dry-run], then rebuild the library.
Layouts not swept keep the chunks the header already holds.
"""
from __future__ import annotations

import argparse
import os
import re
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HEADER = os.path.join(HERE, "csrc", "tuned_windows.hpp")

# one representative width per row layout, in dispatch_row's order
LAYOUT_D = [2, 4, 8, 16, 32, 64, 128, 256, 512, 768, 784, 1024]
LAYOUT_NAME = ["d<=2", "d<=4", "d<=8", "d<=16", "d<=32", "d<=64", "d<=128", "d<=256",
               "d<=512", "d<=768", "d<=832", "d<=1024"]
CHUNKS = [2, 4, 8, 16, 32, 64, 128]
QS = [(1.0, "q=1"), (2.0, "q=2"), (float("inf"), "q=inf")]


def matvec_us(ccm, A, graph, q, chunk, gammas, budget_s):
    """Average Newton matvec launch (us) over a path solve with this chunk.
    The solve stops at its time budget if it has not converged by then: the
    launches it made are as good a sample as those of a converged solve."""
    src, dst, w = graph
    o = ccm.ccm_default_options(profile=2, window_chunk=chunk, time_budget_s=budget_s)
    out = ccm.ccm_solve_path(A, src, dst, w, gammas, q, 1e-6, opts=o)
    ms = sum(s["kern_ms"][2] for s in out["stats"])
    calls = sum(s["kern_calls"][2] for s in out["stats"])
    cg = sum(s["cg"] for s in out["stats"])
    return 1000.0 * ms / max(calls, 1), cg, [int(v) for v in out["status"]]


def read_header(path):
    """The (layout, q) -> chunk table a header holds."""
    text = open(path).read()
    body = text[text.index("kTunedChunk"):]
    vals = [int(v) for v in re.findall(r"\{\s*(\d+),\s*(\d+),\s*(\d+)\s*\}", body)
            for v in v]
    if len(vals) != 3 * len(LAYOUT_D):
        raise ValueError(f"{path}: expected {len(LAYOUT_D)} rows of 3 chunks")
    return {(i // 3, i % 3): v for i, v in enumerate(vals)}


def write_header(table, path):
    rows = []
    for li in range(len(LAYOUT_D)):
        rows.append("{" + ", ".join(str(table[(li, qi)]) for qi in range(3)) + "}")
    body = ",\n    ".join(", ".join(rows[i:i + 4]) for i in range(0, len(rows), 4))
    text = f"""// Window chunk (incidences per row group of a window) for each row layout
// and q, as picked by the project's window tuner (tune_windows.py in the
// package: it times the Newton matvec over a sweep of chunks on synthetic
// k-NN graphs and rewrites this table).  Rows: the row layouts of
// dispatch_row in order (d <= 2, 4, 8, 16, 32, 64, 128, 256, 512, 768, 832,
// 1024); columns: q = 1, 2, inf.
#pragma once

namespace ccm {{

constexpr int kTunedLayouts = {len(LAYOUT_D)};
constexpr int kTunedChunk[kTunedLayouts][3] = {{
    {body},
}};

}}  // namespace ccm
"""
    open(path, "w").write(text)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="also write the timing table (markdown) here")
    ap.add_argument("--dry-run", action="store_true", help="time only, leave the header alone")
    ap.add_argument("--values", type=float, default=8e7, help="row values n d per graph")
    ap.add_argument("--budget", type=float, default=2.0, help="seconds per path solve")
    ap.add_argument("--repeats", type=int, default=1, help="runs per chunk (the fastest counts)")
    ap.add_argument("--chunks", default=None, help="comma-separated chunks to sweep")
    ap.add_argument("--layouts", default=None, help="comma-separated layout indices to sweep")
    ap.add_argument("--header", default=HEADER, help="header to write (default: the package's)")
    args = ap.parse_args()
    sweep = (range(len(LAYOUT_D)) if args.layouts is None
             else [int(v) for v in args.layouts.split(",")])
    chunks = CHUNKS if args.chunks is None else [int(v) for v in args.chunks.split(",")]
    sys.path.insert(0, ROOT)
    import torch
    import synthdata
    import paper_2501_15964_amd as ccm

    gammas = [1e-2, 1e-1]
    table = read_header(HEADER)
    lines = ["| layout | q | " + " | ".join(f"chunk {c} (us)" for c in chunks) + " | picked |",
             "|---|---|" + "---:|" * len(chunks) + "---:|"]
    for li in sweep:
        d = LAYOUT_D[li]
        n_per = int(min(20000, max(200, args.values / d / 10)))
        A_np, _ = synthdata.mixture64(n_per=n_per, d=d, n_blobs=10, seed=7000 + d)
        A = torch.from_numpy(A_np).cuda()
        graph = ccm.ccm_build_knn_graph(A, 10, 0.0)[:3]
        print(f"d={d}: n = {A_np.shape[0]}, m = {graph[0].numel()}", flush=True)
        for qi, (q, qname) in enumerate(QS):
            t0 = time.perf_counter()
            times = []
            for c in chunks:
                runs = [matvec_us(ccm, A, graph, q, c, gammas, args.budget)
                        for _ in range(args.repeats)]
                times.append(min(r[0] for r in runs))
                print(f"  d={d} {qname} chunk {c}: {times[-1]:.1f} us "
                      f"(cg iterations {runs[0][1]}, status {runs[0][2]})", flush=True)
            best = chunks[int(np.argmin(times))]
            table[(li, qi)] = best
            lines.append(f"| {LAYOUT_NAME[li]} (d = {d}, n = {A_np.shape[0]}) | {qname} | " +
                         " | ".join(f"{t:.1f}" for t in times) + f" | {best} |")
            print(lines[-1], f"({time.perf_counter() - t0:.1f} s)", flush=True)
        del A, graph
        torch.cuda.empty_cache()
        # after every layout, so that a partial sweep keeps what it measured
        if not args.dry_run:
            write_header(table, args.header)
        if args.out:
            open(args.out, "w").write("\n".join(lines) + "\n")
    if not args.dry_run:
        print(f"wrote {args.header}; rebuild the library", flush=True)


if __name__ == "__main__":
    main()
