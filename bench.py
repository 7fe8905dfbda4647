"""Benchmark: overlapped RBF-FD differentiation-matrix build on one MI355X.

One step = one whole DM build from device-resident nodes to device-resident
CSR: stencils (kNN), greedy overlapped covering, per-stencil saddle solves,
CSR scatter.  Workload: 3D unit ball, N = 1,000,000 nodes (scrambled Halton
interior + Fibonacci shell), PHS r^5, polynomial degree 3 (M = 20), stencil
n = 50, delta = 0.3, Laplacian at every node, FP64.

Prints one JSON line: weights/s (nnz / build time), stencils/s, phase times,
p50/p99 build latency, the FP64 roofline fraction of the weights kernel and
the CPU oracle's rate on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64 (256 CUs x 2.4 GHz x 128)
HBM_PEAK_GBS = 8000.0

# The weights kernel's HBM traffic comes from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs summarised in this file, together with the SHA-256 of the
# kernel sources they were taken on; a stale summary reports null.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "weights_reg_ball1M_traffic.md")
KERNEL_SOURCES = ["paper_1606_03135_amd/csrc/weights_reg.hip",
                  "paper_1606_03135_amd/csrc/weights_common.hpp"]
COPY_BYTES = 1 << 30


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the weights kernel, or None if the summary is
    missing or was taken on other kernel sources."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    fields = dict(re.findall(r"^- (\w+): `?([0-9a-f.e+]+)`?\s*$", text, re.M))
    if fields.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def lu_flops(K, p):
    """Algorithmic flops of one stencil: partial-pivot LU of the K x K
    saddle matrix plus forward/back substitution for p right-hand sides."""
    return (2.0 * K ** 3 / 3.0 - K ** 2 / 2.0 - K / 6.0) + p * (2.0 * K * K - K)


def cpu_baseline(n, m, l, delta, n_sample):
    import nodesets
    import oracle
    threads = min(16, len(os.sched_getaffinity(0)))
    x = nodesets.ball(n_sample, 2)["x"]
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    t0 = time.perf_counter()
    r = oracle.build_dm(x, n, m, l, delta, nthreads=threads,
                        knn_method="grid")
    dt = time.perf_counter() - t0
    nnz = len(r["val"])
    return {"value": nnz / dt, "unit": "weights/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"oracle build_dm (grid kNN, sequential covering, "
                       f"OpenMP weights) on the 3D ball with N={n_sample} "
                       f"nodes, same n/m/l/delta: {dt:.2f} s, nnz={nnz}")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--N", type=int, default=1_000_000)
    ap.add_argument("--cpu-sample", type=int, default=1_000_000,
                    help="nodes of the ball the oracle builds (default: the "
                         "whole workload)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run a plain device copy of "
                         "known size (to scale HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU "
              "path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import nodesets
    import paper_1606_03135_amd as orbf

    n, m, l, delta = 50, 5, 3, 0.3
    M = math.comb(l + 3, 3)
    K = n + M
    x = nodesets.ball(args.N, 2)["x"]
    N = len(x)
    dev = torch.device("cuda:0")
    xd = torch.from_numpy(x).to(dev)
    ctx = orbf.Context(0)

    def step():
        return orbf.build_dm(xd, n, m, l, delta, ctx=ctx, sync=True)

    for _ in range(args.warmup):
        r = step()
    r = step() if args.warmup == 0 else r
    nc = int(r["n_centers"].item())
    p = r["p"][:nc].cpu().numpy().astype(np.float64)
    flops_launch = float(np.sum(lu_flops(K, p)))
    nnz = int(r["row_ptr"][-1].item())

    torch.cuda.synchronize()
    lat, wk, phases = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        step()
        lat.append(time.perf_counter() - s0)
        pt = ctx.phase_times()
        phases.append(pt[:4])
        wk.append(pt[4])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    ms_step = 1e3 * elapsed / args.steps
    value = nnz * args.steps / elapsed
    wk_ms = float(np.mean(wk))
    achieved = flops_launch / (wk_ms * 1e-3) / 1e12
    ph = np.mean(np.array(phases), axis=0)
    knn_bytes = N * 3 * 8 + N * n * 4 + N * 8
    csr_bytes = nnz * 12 + (N + 1) * 8
    out = {
        "metric": "RBF-FD weights/sec building 3D Laplacian DM (N=1M); "
                  "p50/p99 request latency",
        "value": value,
        "unit": "weights/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D unit ball N={N} (scrambled Halton + "
                               f"Fibonacci shell), PHS r^5, l=3 (M=20), "
                               f"n=50, delta=0.3, Laplacian, FP64",
                   "N": N, "n": n, "m": m, "l": l, "delta": delta,
                   "parallelism": "single GPU"},
        "stencils_per_s": nc * args.steps / elapsed,
        "n_centers": nc,
        "nnz": nnz,
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                       "p99": 1e3 * float(np.percentile(lat, 99))},
        "phase_ms": {"knn": ph[0], "cover": ph[1], "weights": ph[2],
                     "csr": ph[3]},
        "hbm_gbs": {"knn": knn_bytes / (ph[0] * 1e-3) / 1e9,
                    "csr": csr_bytes / (ph[3] * 1e-3) / 1e9},
        "roofline": {"bound": "alu", "kernel": "weights_reg_kernel<9,2>",
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(),
                     "flops_per_launch": flops_launch,
                     "launch_ms": wk_ms},
    }
    if args.copy_calibration:
        # plain elementwise copy: reads and writes COPY_BYTES each
        a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        a.fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = COPY_BYTES
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, m, l, delta, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
