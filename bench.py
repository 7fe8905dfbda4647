"""Benchmark: overlapped RBF-FD differentiation-matrix build on one MI355X.

Default workload (the headline): one step = one whole DM build from
device-resident nodes to device-resident CSR (stencils, greedy overlapped
covering, per-stencil saddle solves, CSR) of the 3D unit ball with
N = 1,000,000 nodes (scrambled Halton interior + Fibonacci shell), PHS r^5,
polynomial degree 3 (M = 20), stencil n = 50, delta = 0.3, Laplacian at
every node, FP64.  Prints one JSON line: weights/s (nnz / build time),
stencils/s, phase times, p50/p99 build latency, the FP64 roofline fraction
of the weights kernel, the FP32 + FP64-refinement variant of the same build
with its weight error, and the CPU oracle's rate on the same workload.
After the timed builds, the built DM's consumers are timed on their own:
its Gershgorin disks, y = L x, one backward-Euler step (I - dt L) u1 = u0
with Dirichlet rows on the sphere, solved by BiCGSTAB, and BDF4 steps of
the same problem (after one step each of BDF1-3).

Unless --quick, the same JSON line also carries the other measured
workloads, each timed after the headline:
  - w1_square: the jittered 45 x 45 square (2,025 nodes), r^3, l = 2,
    n = 12, delta = 1 (standard RBF-FD), microseconds per build;
  - w2_disk: the unit disk, 99,400 interior + 600 boundary nodes, r^5,
    l = 4, n = 31, delta = 0.5, Lebesgue threshold 5 on the Laplacian rows,
    normal-derivative boundary rows, in the shuffled and the Poisson-disk
    generation order, with phase times;
  - delta1_gpu: the headline ball at delta = 1 (standard RBF-FD), and the
    speedup of the overlapped build over it;
  - batched: the 512-set batch below (FP32 + refinement and FP64, with the
    FP64 peak fraction of the summed per-set flops);
  - serving: the request stream below, FP64 and FP32 + refinement;
  - cpu_baseline: besides the oracle's rate on the whole workload (all
    threads of the job's CPU share), single-thread phase times on a
    100k-node sample and the oracle's delta = 1 build of the whole ball.

--workload batched: 512 mixed node sets (N log-uniform in [1e3, 2e5], 2D/3D,
l in {2,3,4}, n in [2M+1, 3M], delta in {0.2, 0.5, 1}) in one batched call,
FP32 + refinement (and FP64 beside it); repeated batches replay a HIP graph.

--workload serving: Poisson stream of DM-build requests (N lognormal,
median 2e4, clipped to [5e3, 5e5]; 2D/3D; l in {2,3,4}; delta ~ U[0.2, 1];
n = 2M+1) into the request engine; saturation throughput mu from a closed
loop, then open-loop runs at 0.5 mu and 0.8 mu with p50/p99 latency.
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
KERNEL_SOURCES = ["paper_1606_03135_amd/csrc/weights_reg_kernel.hpp",
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


OPS = {"laplacian": ("OP_LAPLACIAN", "Laplacian"), "dx": ("OP_DX", "d/dx"),
       "dy": ("OP_DY", "d/dy"), "dz": ("OP_DZ", "d/dz"),
       "identity": ("OP_IDENTITY", "identity")}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_threads():
    """Threads the oracle may use: the job's CPU share (its affinity mask,
    capped by OMP_NUM_THREADS where the environment sets it)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return n


def cpu_baseline(n, m, l, delta, n_sample, op="laplacian", extras=True):
    """The oracle as it stands, timed on the host: the whole workload on
    every thread of the job's share; with ``extras``, single-thread phase
    times on a 100k-node sample of the same ball and the delta = 1
    (standard RBF-FD) build of the whole ball on all threads."""
    import nodesets
    import oracle
    threads = host_threads()
    x = nodesets.ball(n_sample, 2)["x"]
    t0 = time.perf_counter()
    r = oracle.build_dm(x, n, m, l, delta, nthreads=threads,
                        knn_method="grid", op=getattr(oracle, OPS[op][0]))
    dt = time.perf_counter() - t0
    nnz = len(r["val"])
    out = {"value": nnz / dt, "unit": "weights/s", "cores": threads,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": (f"oracle build_dm (grid kNN, sequential covering, "
                      f"OpenMP weights) on the 3D ball with N={n_sample} "
                      f"nodes, same n/m/l/delta: {dt:.2f} s, nnz={nnz}")}
    if not extras or op != "laplacian":
        return out
    # single thread, per phase, on a 100k-node ball
    xs = nodesets.ball(100_000, 2)["x"]
    t0 = time.perf_counter()
    idx, rho2 = oracle.knn(xs, n, "grid")
    t1 = time.perf_counter()
    oracle.cover(xs, idx, rho2, delta)
    t2 = time.perf_counter()
    rr = oracle.overlapped_rows(xs, idx, rho2, m, l, delta, nthreads=1)
    t3 = time.perf_counter()
    rp, col, val = oracle.csr(idx, rr["owner"], rr["W"])
    t4 = time.perf_counter()
    out["single_thread_phases_s"] = {
        "sample": "3D ball, N=100000, same n/m/l/delta, one thread",
        "knn": t1 - t0, "cover": t2 - t1,
        "weights": (t3 - t2) - (t2 - t1),  # overlapped_rows also covers
        "csr": t4 - t3, "weights_per_s": len(val) / (t4 - t0 - (t2 - t1))}
    # standard RBF-FD (delta = 1) on the whole ball, same threads: the
    # paper's comparison (Sec. 4.3 speedup model, Sec. 7.2.2 results)
    t0 = time.perf_counter()
    r1 = oracle.overlapped_rows(x, r["knn"], r["rho2"], m, l, 1.0,
                                nthreads=threads)
    d1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.overlapped_rows(x, r["knn"], r["rho2"], m, l, delta,
                           nthreads=threads)
    dd = time.perf_counter() - t0
    out["delta1"] = {"covering_and_weights_s": d1,
                     "same_at_delta_s": dd, "speedup": d1 / dd,
                     "n_centers_delta1": int(len(r1["centers"])),
                     "n_centers": int(len(r["centers"]))}
    return out


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_flops(r, K):
    nc = int(r["n_centers"].item())
    p = np.bincount(r["owner"].cpu().numpy().clip(0))[
        r["centers"][:nc].cpu().numpy()].astype(np.float64)
    return float(np.sum(lu_flops(K, p))), nc


def bench_ball(args, torch, orbf, nodesets):
    n, m, l, delta = 50, 5, 3, 0.3
    M = math.comb(l + 3, 3)
    K = n + M
    x = nodesets.ball(args.N, 2)["x"]
    N = len(x)
    dev = torch.device("cuda:0")
    xd = torch.from_numpy(x).to(dev)
    ctx = orbf.Context(0)

    op = getattr(orbf, OPS[args.op][0])
    opname = OPS[args.op][1]

    def run(prec, steps, warmup):
        def step():
            return orbf.build_dm(xd, n, m, l, delta, ctx=ctx, sync=True,
                                 prec=prec, op=op)
        r = None
        for _ in range(max(warmup, 1)):
            r = step()
        torch.cuda.synchronize()
        lat, wk, phases = [], [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            r = step()
            lat.append(time.perf_counter() - s0)
            pt = ctx.phase_times()
            phases.append(pt[:4])
            wk.append(pt[4])
        torch.cuda.synchronize()
        return r, lat, wk, phases, time.perf_counter() - t0

    r, lat, wk, phases, elapsed = run(orbf.PREC_FP64, args.steps,
                                      args.warmup)
    _log(f"FP64: {1e3 * elapsed / args.steps:.2f} ms per build")
    flops_launch, nc = build_flops(r, K)
    nnz = int(r["row_ptr"][-1].item())
    ms_step = 1e3 * elapsed / args.steps
    value = nnz * args.steps / elapsed
    wk_ms = float(np.mean(wk))
    achieved = flops_launch / (wk_ms * 1e-3) / 1e12
    ph = np.mean(np.array(phases), axis=0)
    knn_bytes = N * 3 * 8 + N * n * 4 + N * 8
    csr_bytes = nnz * 12 + (N + 1) * 8
    out = {
        "metric": f"RBF-FD weights/sec building 3D {opname} DM (N=1M); "
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
                               f"n=50, delta=0.3, {opname}, FP64",
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
        # the weights kernel runs as three launches, one per pass width
        # (8, 16, 24 right-hand sides: weights_reg_kernel<9, PL, false>,
        # PL = 3, 2, 1), after a 4 us classification; launch_ms spans all
        # of them on the context's stream
        "roofline": {"bound": "alu",
                     "kernel": "weights_reg_kernel<9,{3,2,1},false>",
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(),
                     "flops_per_launch": flops_launch,
                     "launch_ms": wk_ms},
    }
    # Gershgorin disks of the built DM (Sec. 4.2.1): a diagnostic pass over
    # the CSR, timed on its own after the builds
    e0, e1 = torch.cuda.Event(enable_timing=True), \
        torch.cuda.Event(enable_timing=True)
    orbf.gershgorin(ctx, r["row_ptr"], r["col"], r["val"])
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        _, _, gs = orbf.gershgorin(ctx, r["row_ptr"], r["col"], r["val"])
    e1.record()
    torch.cuda.synchronize()
    gms = e0.elapsed_time(e1) / 10
    gs = gs.cpu().numpy()
    out["gershgorin"] = {"ms": gms, "max_right_edge": float(gs[0]),
                         "min_left_edge": float(gs[1]),
                         "rows_reaching_positive_re": int(gs[2]),
                         "hbm_gbs": (nnz * 12 + (N + 1) * 8) / (gms * 1e-3)
                         / 1e9}
    # y = L x with the built DM: the product its consumers (time stepping,
    # Krylov solves) are made of, timed on its own after the builds
    xv = torch.rand(N, dtype=torch.float64, device=dev)
    yv = orbf.spmv(ctx, r["row_ptr"], r["col"], r["val"], xv)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(20):
        orbf.spmv(ctx, r["row_ptr"], r["col"], r["val"], xv, yv)
    e1.record()
    torch.cuda.synchronize()
    sms = e0.elapsed_time(e1) / 20
    out["spmv"] = {"ms": sms, "hbm_gbs": (nnz * 12 + (N + 1) * 8 + N * 16)
                   / (sms * 1e-3) / 1e9}
    # one backward-Euler step of u_t = Laplacian u with the built DM
    # (Sec. 5): (I - dt L) u1 = u0 inside, u1 = 0 on the unit sphere's
    # nodes, dt = 1e-5, from a Gaussian bump, solved to 1e-10 by BiCGSTAB
    kind = torch.from_numpy(
        (np.sqrt((x * x).sum(1)) < 1.0 - 1e-12).astype(np.uint8)).to(dev)
    u0 = torch.from_numpy(np.exp(-4.0 * (x * x).sum(1))).to(dev)
    b = u0 * kind.to(torch.float64)
    orbf.solve_implicit(ctx, r["row_ptr"], r["col"], r["val"], b,
                        beta=-1e-5, row_kind=kind, x0=u0, tol=1e-10,
                        max_iter=10)  # warm: scratch and pinned scalars
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, its, res = orbf.solve_implicit(ctx, r["row_ptr"], r["col"], r["val"],
                                      b, beta=-1e-5, row_kind=kind, x0=u0,
                                      tol=1e-10, max_iter=1000)
    torch.cuda.synchronize()
    ims = 1e3 * (time.perf_counter() - t0)
    out["implicit_step"] = {"ms": ims, "iterations": its, "relres": res,
                            "ms_per_iteration": ims / max(its, 1),
                            "dt": 1e-5, "tol": 1e-10,
                            "dirichlet_rows": int(N - kind.sum().item())}
    # BDF4 time stepping with the same DM and boundary (Sec. 5): one step
    # each of BDF1-3, then BDF4 steps; the timed steps are BDF4
    hist = [u0]
    for _ in range(3):
        un, _, _ = orbf.bdf_step(ctx, r["row_ptr"], r["col"], r["val"], hist,
                                 1e-5, row_kind=kind, tol=1e-10)
        hist = [un] + hist[:3]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bits = 0
    for _ in range(5):
        un, it, _ = orbf.bdf_step(ctx, r["row_ptr"], r["col"], r["val"], hist,
                                  1e-5, row_kind=kind, tol=1e-10)
        hist = [un] + hist[:3]
        bits += it
    torch.cuda.synchronize()
    bms = 1e3 * (time.perf_counter() - t0) / 5
    out["bdf4_step"] = {"ms": bms, "iterations_mean": bits / 5, "dt": 1e-5,
                        "tol": 1e-10}
    if not args.no_fp32:
        W64 = r["W"].clone()
        steps32 = max(3, args.steps // 5)
        r32, lat32, wk32, _, el32 = run(orbf.PREC_FP32_IR, steps32, 1)
        rel = ((W64 - r32["W"]).abs().amax(1) /
               W64.abs().amax(1)).max().item()
        st = r32["ir_steps"].cpu().numpy()
        ok = st >= 0
        out["fp32_ir"] = {
            "value": nnz * steps32 / el32, "unit": "weights/s",
            "steps": steps32, "ms_per_step": 1e3 * el32 / steps32,
            "weights_kernel_ms": float(np.mean(wk32)),
            "achieved_tflops": flops_launch / (np.mean(wk32) * 1e-3) / 1e12,
            "max_row_rel_err_vs_fp64": rel,
            "corrections_mean": float(st[ok].mean()) if ok.any() else None,
            "corrections_max": int(st.max()),
            "fp64_fallback_rows": float((~ok).mean())}
        del W64, r32
    # what this device reaches on the two units the roofline is priced
    # against, next to the published peaks: the FP64 FMA rate of
    # independent dependency chains on every SIMD, and a plain elementwise
    # copy of COPY_BYTES (read + write), both timed after the builds
    fma = ctx.measure_fp64_fma()
    a = torch.full((COPY_BYTES // 8,), 1.0, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    e0.record()
    for _ in range(5):
        torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    cms = e0.elapsed_time(e1) / 5
    out["measured_peaks"] = {
        "fp64_fma_tflops": fma,
        "fp64_fma_frac_of_published": fma / FP64_PEAK_TFLOPS,
        "copy_gbs": 2 * COPY_BYTES / (cms * 1e-3) / 1e9,
        "copy_frac_of_published": 2 * COPY_BYTES / (cms * 1e-3) / 1e9
        / HBM_PEAK_GBS,
        "roofline_frac_vs_measured_fma": achieved / fma}
    del a, b
    if args.copy_calibration:
        # plain elementwise copy: reads and writes COPY_BYTES each
        a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        a.fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = COPY_BYTES
    if not args.quick:
        d1 = bench_delta1(torch, orbf, xd, n, m, l)
        d1["speedup_of_delta"] = d1["ms_per_build"] / ms_step
        out["delta1_gpu"] = d1
        _log(f"delta = 1: {d1['ms_per_build']:.2f} ms per build")
    del r
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, m, l, delta, args.cpu_sample,
                                           args.op, extras=not args.quick)
    return out


def _ev(torch):
    return torch.cuda.Event(enable_timing=True)


def bench_w1(torch, orbf, nodesets, reps=30):
    """Jittered 45 x 45 square (2,025 nodes), r^3, l = 2, n = 12, delta = 1
    (standard RBF-FD), Laplacian, FP64: a latency-bound build, reported in
    microseconds (median over ``reps`` builds after warm-up)."""
    x = nodesets.square(45, 0)
    xd = torch.from_numpy(x).to("cuda:0")
    ctx = orbf.Context(0)
    for _ in range(5):
        orbf.build_dm(xd, 12, 3, 2, 1.0, ctx=ctx)
    wall, span = [], []
    for _ in range(reps):
        e0, e1 = _ev(torch), _ev(torch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        r = orbf.build_dm(xd, 12, 3, 2, 1.0, ctx=ctx, sync=False)
        e1.record()
        ctx.sync()
        wall.append(time.perf_counter() - t0)
        span.append(e0.elapsed_time(e1))
    nnz = int(r["row_ptr"][-1].item())
    # the same build repeated through the batched entry point with one set:
    # captured in a HIP graph on its second call and replayed after
    sets = [dict(xyz=xd, n=12, m=3, l=2, delta=1.0)]
    outs = orbf.build_dm_batched(ctx, sets)
    for _ in range(3):
        orbf.build_dm_batched(ctx, sets, outputs=outs)
    torch.cuda.synchronize()
    replay = []
    for _ in range(reps):
        t0 = time.perf_counter()
        orbf.build_dm_batched(ctx, sets, outputs=outs)
        torch.cuda.synchronize()
        replay.append(time.perf_counter() - t0)
    return {"workload": "2D square N=2025 (jittered 45x45), r^3, l=2, n=12, "
                        "delta=1, Laplacian, FP64",
            "builds": reps, "nnz": nnz,
            "us_median": 1e6 * float(np.median(wall)),
            "us_p90": 1e6 * float(np.percentile(wall, 90)),
            "device_span_us_median": 1e3 * float(np.median(span)),
            "weights_per_s": nnz / float(np.median(wall)),
            "graph_replay_us_median": 1e6 * float(np.median(replay)),
            "graph_replay_us_p90": 1e6 * float(np.percentile(replay, 90))}


def bench_w2(torch, orbf, nodesets, reps=10):
    """Unit disk, 99,400 interior + 600 boundary nodes, r^5, l = 4, n = 31,
    delta = 0.5, Lebesgue threshold tau = 5 on the Laplacian rows, normal
    derivative rows at the boundary, FP64; in the shuffled order and in
    the Poisson-disk generation order.  Phases timed with events between
    the entry points: kNN, interior rows (the Lebesgue covering and its
    solves), boundary rows, CSR."""
    dev = torch.device("cuda:0")
    res = {"workload": "2D disk 99400 interior + 600 boundary, r^5, l=4, "
                       "n=31, delta=0.5, tau=5, Laplacian + Neumann rows, "
                       "FP64"}
    for order in ("shuffled", "generation"):
        D = nodesets.disk(99400, 600, 1, order=order)
        xd = torch.from_numpy(D["x"]).to(dev)
        el = torch.from_numpy(D["eligible"]).to(dev)
        bd = torch.from_numpy(D["boundary"]).to(dev)
        nr = torch.from_numpy(D["normals"]).to(dev)
        N = xd.shape[0]
        ctx = orbf.Context(0)

        def once():
            ev = [_ev(torch) for _ in range(5)]
            ev[0].record()
            knn, rho2 = orbf.build_nodes_knn(ctx, xd, 31)
            ev[1].record()
            centers = torch.empty(N, dtype=torch.int32, device=dev)
            nc = torch.zeros(1, dtype=torch.int64, device=dev)
            owner = torch.empty(N, dtype=torch.int32, device=dev)
            lam = torch.zeros(N, dtype=torch.float64, device=dev)
            W = orbf.compute_weights(ctx, orbf.OP_LAPLACIAN, 5, 4, 31, 0.5,
                                     xd, knn, rho2, centers=centers,
                                     n_centers=nc, owner=owner, eligible=el,
                                     tau=5.0, lebesgue=lam)
            ev[2].record()
            orbf.compute_weights(ctx, orbf.OP_NEUMANN, 5, 4, 31, 1.0, xd,
                                 knn, rho2, rows=bd, normals=nr, owner=owner,
                                 W=W, lebesgue=lam)
            ev[3].record()
            rp, _, _ = orbf.assemble_csr(ctx, knn, owner, W)
            ev[4].record()
            ctx.sync()
            return [ev[i].elapsed_time(ev[i + 1]) for i in range(4)], rp, nc

        for _ in range(3):
            once()
        ph = []
        for _ in range(reps):
            t, rp, nc = once()
            ph.append(t)
        ph = np.array(ph)
        tot = ph.sum(1)
        nnz = int(rp[-1].item())
        res[order] = {"ms_median": float(np.median(tot)),
                      "weights_per_s": nnz / (float(np.median(tot)) * 1e-3),
                      "nnz": nnz, "n_centers": int(nc.item()),
                      "phase_ms": dict(zip(("knn", "interior_rows",
                                            "boundary_rows", "csr"),
                                           np.median(ph, 0).tolist()))}
        del ctx
    return res


def bench_delta1(torch, orbf, xd, n, m, l, reps=3):
    """The same ball with delta = 1 (standard RBF-FD: every node its own
    stencil), for the speedup of the overlapped build (Sec. 4.3 model,
    Sec. 7.2.2)."""
    ctx = orbf.Context(0)
    r = orbf.build_dm(xd, n, m, l, 1.0, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = orbf.build_dm(xd, n, m, l, 1.0, ctx=ctx)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    return {"ms_per_build": ms, "n_centers": int(r["n_centers"].item()),
            "weights_ms": float(ctx.phase_times()[2])}


def bench_batched(args, torch, orbf, nodesets):
    specs = nodesets.batch_specs(args.sets, 4)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    xs = [torch.from_numpy(nodesets.make_set(s)).to(dev) for s in specs]
    gen_s = time.perf_counter() - t0
    _log(f"{len(specs)} node sets generated in {gen_s:.1f} s")
    ctx = orbf.Context(0)
    tuned = None
    if not args.no_tune:
        from paper_1606_03135_amd import tune
        rep, tune_s = tune.tune_sets(
            ctx, [dict(xyz=x, n=s["n"], m=s["m"], l=s["l"], delta=s["delta"])
                  for s, x in zip(specs, xs)], reps=2)
        picks = {}
        for r in rep:
            picks[r["pick"]] = picks.get(r["pick"], 0) + 1
        tuned = {"classes": len(rep), "picks": picks, "tune_s": tune_s}
        _log(f"tuned {len(rep)} (K, p-class) classes in {tune_s:.1f} s: "
             f"{picks}")

    def sets_for(prec):
        return [dict(xyz=x, n=s["n"], m=s["m"], l=s["l"], delta=s["delta"],
                     prec=prec) for s, x in zip(specs, xs)]

    def run(prec, steps, warmup):
        sets = sets_for(prec)
        outs = orbf.build_dm_batched(ctx, sets)
        _log(f"prec {prec}: first batch done")
        for _ in range(max(warmup, 2)):  # second call captures the graph
            orbf.build_dm_batched(ctx, sets, outputs=outs)
        _log(f"prec {prec}: warm-up done")
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for _ in range(steps):
            s0 = time.perf_counter()
            orbf.build_dm_batched(ctx, sets, outputs=outs)
            lat.append(time.perf_counter() - s0)
        torch.cuda.synchronize()
        return outs, lat, time.perf_counter() - t0

    o32, lat32, el32 = run(orbf.PREC_FP32_IR, args.steps, args.warmup)
    nnz = sum(int(o["row_ptr"][-1].item()) for o in o32)
    ncent = sum(int(o["n_centers"].item()) for o in o32)
    # algorithmic flops of the batch: per set, an LU of its K x K system
    # per stencil plus one substitution pair per kept row
    flops = 0.0
    for s, o in zip(specs, o32):
        nc = int(o["n_centers"].item())
        own = o["owner"].cpu().numpy()
        p = np.bincount(own[own >= 0], minlength=len(own))[
            o["centers"][:nc].cpu().numpy()].astype(np.float64)
        flops += float(np.sum(lu_flops(s["n"] + s["M"], p)))
    W32 = [o["W"].clone() for o in o32]
    st = np.concatenate([o["ir_steps"].cpu().numpy() for o in o32])
    del o32
    o64, lat64, el64 = run(orbf.PREC_FP64, args.steps, args.warmup)
    rel = max(((a["W"] - b).abs().amax(1) / a["W"].abs().amax(1)).max().item()
              for a, b in zip(o64, W32))
    ok = st >= 0
    Ks = [s["n"] + s["M"] for s in specs]
    return {
        "metric": "RBF-FD weights/sec, batched DM build of 512 mixed node "
                  "sets (FP32 LU + FP64 refinement)",
        "value": nnz * args.steps / el32, "unit": "weights/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * el32 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64ir",
        "data": "synthetic",
        "config": {"workload": f"{len(specs)} node sets, N log-uniform "
                               f"[1e3, 2e5] (sum {sum(x.shape[0] for x in xs)}"
                               f"), 2D jittered grids / 3D balls, l in "
                               f"{{2,3,4}}, n in [2M+1, 3M], delta in "
                               f"{{0.2,0.5,1.0}}, Laplacian",
                   "K_range": [min(Ks), max(Ks)], "workers": 4,
                   "parallelism": "single GPU"},
        "nnz": nnz, "n_centers": ncent,
        "stencils_per_s": ncent * args.steps / el32,
        "fp64": {"value": nnz * args.steps / el64, "unit": "weights/s",
                 "ms_per_step": 1e3 * el64 / args.steps,
                 "fp64_peak_frac": flops * args.steps / el64 / 1e12
                 / FP64_PEAK_TFLOPS},
        "flops_per_batch": flops,
        "fp64_peak_frac": flops * args.steps / el32 / 1e12 / FP64_PEAK_TFLOPS,
        "max_row_rel_err_vs_fp64": rel,
        "corrections_mean": float(st[ok].mean()) if ok.any() else None,
        "fp64_rows": float((~ok).mean()),
        "node_generation_s": gen_s,
        "autotuned": tuned,
    }


def bench_serving(args, torch, orbf, nodesets):
    dev = torch.device("cuda:0")
    pool = nodesets.request_specs(args.pool, 1.0, 5)
    t0 = time.perf_counter()
    xs = [torch.from_numpy(nodesets.make_set(s)).to(dev) for s in pool]
    gen_s = time.perf_counter() - t0
    _log(f"{len(pool)} node sets generated in {gen_s:.1f} s")
    rng = np.random.Generator(np.random.PCG64(6))
    arena = max(orbf.lib().orbf_request_bytes(x.shape[0], x.shape[1],
                                              s["n"], 0)
                for s, x in zip(pool, xs)) * 4 * args.slots
    scratch = max(orbf.workspace_size(x.shape[0], x.shape[1], s["n"], s["l"])
                  for s, x in zip(pool, xs))
    srv = orbf.Server(0, slots=args.slots, arena=arena, slot_scratch=scratch)

    def run(count, rate, prec=0):
        """rate None: closed loop (all arrive at once)."""
        picks = rng.integers(0, len(pool), count)
        gaps = (rng.exponential(1.0 / rate, count) if rate
                else np.zeros(count))
        arrive = np.cumsum(gaps)
        lat, nnz = [], 0
        start = srv.now() + 0.01
        i = done = 0
        while done < count:
            now = srv.now()
            while i < count and start + arrive[i] <= now:
                k = picks[i]
                s = pool[k]
                srv.submit(xs[k], s["n"], s["m"], s["l"], s["delta"],
                           prec=prec, t_arrival=start + arrive[i])
                i += 1
            for t in srv.poll():
                info = srv.result(t)
                assert info["status"] == 0, info
                lat.append(info["t_done"] - info["t_arrival"])
                nnz += info["N"] * info["n"]
                srv.release(t)
                done += 1
        span = srv.now() - start
        _log(f"{count} requests at rate {rate}: {count / span:.1f} req/s")
        lat = np.array(lat)
        return {"requests": count,
                "offered_rps": rate, "achieved_rps": count / span,
                "weights_per_s": nnz / span,
                "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                "p99_ms": 1e3 * float(np.percentile(lat, 99))}

    by_prec = {}
    for prec, name in ((0, "fp64"), (1, "fp32_ir")):
        run(min(64, args.requests), None, prec)  # warm-up
        sat = run(args.requests, None, prec)
        mu = sat["achieved_rps"]
        loads = {"saturation": sat}
        for f in (0.5, 0.8):
            loads[f"{f}mu"] = run(args.requests, f * mu, prec)
        by_prec[name] = loads
    srv.close()
    loads = by_prec["fp64"]
    main_load = loads["0.5mu"]
    return {
        "metric": "DM-build serving: p50/p99 request latency and weights/s "
                  "under Poisson arrivals",
        "value": main_load["weights_per_s"], "unit": "weights/s",
        "n_gpus": 1, "steps": args.requests, "warmup": 64,
        "ms_per_step": 1e3 / main_load["achieved_rps"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"Poisson stream, {args.pool} distinct node "
                               f"sets (N lognormal median 2e4 sigma 1, "
                               f"clipped [5e3, 5e5], 2D/3D, l in {{2,3,4}}, "
                               f"delta U[0.2,1], n=2M+1), {args.slots} slots",
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": main_load["p50_ms"], "p99": main_load["p99_ms"]},
        "loads": loads, "fp32_ir_loads": by_prec["fp32_ir"],
        "node_generation_s": gen_s,
    }


def weights_only(args, torch, orbf, nodesets):
    """The headline ball's weights phase alone, twice, in one precision:
    the launches a counter run (rocprofv3 --pmc) attributes to the weights
    kernels, without the rest of the bench."""
    n, m, l, delta = 50, 5, 3, 0.3
    x = nodesets.ball(args.N, 2)["x"]
    xd = torch.from_numpy(x).to("cuda:0")
    ctx = orbf.Context(0)
    knn, rho2 = orbf.build_nodes_knn(ctx, xd, n)
    centers, nc, owner, _ = orbf.select_overlapped_stencils(ctx, xd, knn,
                                                            rho2, delta)
    W = torch.empty((len(x), n), dtype=torch.float64, device="cuda:0")
    prec = orbf.PREC_FP32_IR if args.weights_only == "fp32" else \
        orbf.PREC_FP64
    st = torch.empty(len(x), dtype=torch.int32, device="cuda:0")
    for _ in range(2):
        orbf.compute_weights(ctx, orbf.OP_LAPLACIAN, m, l, n, delta, xd, knn,
                             rho2, centers=centers, n_centers=nc,
                             owner=owner, W=W, prec=prec,
                             ir_steps=st if prec == orbf.PREC_FP32_IR
                             else None)
    ctx.sync()
    _log(f"weights only, {args.weights_only}: {int(nc.item())} stencils, "
         "two builds")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ball",
                    choices=["ball", "batched", "serving"])
    ap.add_argument("--N", type=int, default=1_000_000)
    ap.add_argument("--op", default="laplacian", choices=sorted(OPS),
                    help="operator of the ball workload's DM (the headline "
                         "is the Laplacian)")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000,
                    help="nodes of the ball the oracle builds (default: the "
                         "whole workload)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched: skip the schedule autotuner")
    ap.add_argument("--sets", type=int, default=512)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--pool", type=int, default=128)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--quick", action="store_true",
                    help="ball workload only: skip the W1/W2/delta=1/batched/"
                         "serving sub-records and the oracle's extra legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run a plain device copy of "
                         "known size (to scale HBM byte counters)")
    ap.add_argument("--weights-only", choices=["fp64", "fp32"],
                    help="for counter runs: build the ball's stencils and "
                         "covering, then run only the weights entry point "
                         "twice in this precision, and print no JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU "
              "path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import nodesets
    import paper_1606_03135_amd as orbf

    if args.weights_only:
        weights_only(args, torch, orbf, nodesets)
        return
    fn = {"ball": bench_ball, "batched": bench_batched,
          "serving": bench_serving}[args.workload]
    out = fn(args, torch, orbf, nodesets)
    if args.workload == "ball" and not args.quick and args.op == "laplacian":
        # the other workloads, timed after the headline
        torch.cuda.empty_cache()
        out["w1_square"] = bench_w1(torch, orbf, nodesets)
        _log(f"W1: {out['w1_square']['us_median']:.0f} us per build")
        out["w2_disk"] = bench_w2(torch, orbf, nodesets)
        _log("W2: shuffled {:.2f} ms, generation order {:.2f} ms".format(
            out["w2_disk"]["shuffled"]["ms_median"],
            out["w2_disk"]["generation"]["ms_median"]))
        torch.cuda.empty_cache()
        b = bench_batched(argparse.Namespace(
            sets=512, steps=2, warmup=2, no_tune=False), torch, orbf,
            nodesets)
        out["batched"] = {k: b[k] for k in (
            "value", "unit", "ms_per_step", "fp64", "fp64_peak_frac",
            "flops_per_batch", "nnz", "n_centers", "max_row_rel_err_vs_fp64",
            "corrections_mean", "fp64_rows", "autotuned", "dtype")}
        out["batched"]["workload"] = b["config"]["workload"]
        torch.cuda.empty_cache()
        sv = bench_serving(argparse.Namespace(
            pool=128, slots=4, requests=2000), torch, orbf, nodesets)
        out["serving"] = {"workload": sv["config"]["workload"],
                          "fp64": sv["loads"], "fp32_ir": sv["fp32_ir_loads"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
