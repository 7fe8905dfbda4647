"""Autotuner of the weights kernel schedules (``orbf_set_schedule``).

Stencils of one system size K = n + M can be solved by a one-wavefront
kernel with 16 or 8 right-hand sides per pass, or with 8, 16 or 24 chosen
per stencil from its retained rows ("split"; K <= 72), by a four-
wavefront workgroup kernel (K <= 144), or by the one-wavefront blocked
elimination on the FP64 matrix cores ("matrix"; 32 < K <= 80).  Which is fastest depends on K and on
how many rows a stencil keeps (p-class: n (1 - delta)^d above 8 or not).
The tuner times each candidate on the largest node set of each (K, p-class)
present in a workload, with HIP events around the weights kernel, and keeps
the fastest in the context's table; the table can be saved as JSON and
loaded into another context.
"""
import json
import math
import time

import paper_1606_03135_amd as orbf

SCHEDULES = {"wave16": 0, "wave8": 1, "group16": 2, "split": 3,
             "matrix": 4}
NAMES = {v: k for k, v in SCHEDULES.items()}


def _candidates(K):
    out = []
    if K <= 72:
        out = ["split", "wave16", "wave8", "group16"]
    elif K <= 144:
        out = ["group16"]
    if 32 < K <= 80:
        out.append("matrix")
    return out


def pclass(n, d, delta):
    return 1 if n * (1.0 - delta) ** d > 8.0 else 0


def _lib():
    import ctypes
    L = orbf.lib()
    if not hasattr(L, "_sched_ready"):
        L.orbf_set_schedule.argtypes = [ctypes.c_void_p, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int]
        L.orbf_set_schedule.restype = ctypes.c_int
        L.orbf_get_schedules.argtypes = [ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)]
        L.orbf_get_schedules.restype = ctypes.c_int
        L._sched_ready = True
    return L


def set_schedule(ctx, K, pc, name):
    code = -1 if name is None else SCHEDULES[name]
    ctx.check(_lib().orbf_set_schedule(ctx._h, int(K), int(pc), code))


def get_schedules(ctx):
    import ctypes
    cap = 512
    buf = (ctypes.c_int32 * (3 * cap))()
    cnt = ctypes.c_int()
    ctx.check(_lib().orbf_get_schedules(ctx._h, buf, cap, ctypes.byref(cnt)))
    return [(buf[3 * i], buf[3 * i + 1], NAMES[buf[3 * i + 2]])
            for i in range(min(cnt.value, cap))]


def tune_sets(ctx, sets, reps=3, log=None):
    """Tune every (K, p-class) of ``sets`` (dicts as for build_dm_batched:
    xyz, n, m, l, delta).  Returns a list of dicts with the timings."""
    groups = {}
    for s in sets:
        d = s["xyz"].shape[1]
        K = s["n"] + math.comb(s["l"] + d, d)
        key = (K, pclass(s["n"], d, s["delta"]))
        if key not in groups or s["xyz"].shape[0] > groups[key]["xyz"].shape[0]:
            groups[key] = s
    report = []
    t0 = time.perf_counter()
    for (K, pc), s in sorted(groups.items()):
        cands = _candidates(K)
        if len(cands) < 2:
            continue
        times = {}
        for name in cands:
            set_schedule(ctx, K, pc, name)
            best = math.inf
            for _ in range(reps):
                orbf.build_dm(s["xyz"], s["n"], s["m"], s["l"], s["delta"],
                              ctx=ctx)
                best = min(best, ctx.phase_times()[4])
            times[name] = best
        pick = min(times, key=times.get)
        set_schedule(ctx, K, pc, pick)
        report.append(dict(K=K, pclass=pc, N=int(s["xyz"].shape[0]),
                           pick=pick, ms=times))
        if log:
            log(f"K={K} pclass={pc}: {pick} {times}")
    return report, time.perf_counter() - t0


def save(ctx, path):
    with open(path, "w") as f:
        json.dump([dict(K=K, pclass=pc, schedule=name)
                   for K, pc, name in get_schedules(ctx)], f, indent=1)


def load(ctx, path):
    with open(path) as f:
        for row in json.load(f):
            set_schedule(ctx, row["K"], row["pclass"], row["schedule"])
