"""Batched builds and the request engine, through the C ABI.

Every set or request runs the single-set kernels on a worker stream of its
own, so its outputs must equal, bit for bit, those of a single-set build of
the same input (and therefore the oracle's to the usual bars); graph replays
of a repeated batch must equal the eager run; a request's result must not
depend on what else is in flight.
"""
import math
import sys

import numpy as np
import pytest

import nodesets
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("knn", "rho2", "owner", "W", "row_ptr", "col", "val")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def orbf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1606_03135_amd as P
    P.lib()
    return P


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def small_specs(count, seed, nmax=12000):
    """Batch descriptions of the batched workload's kind, sizes capped so
    the oracle and single-set builds stay quick."""
    out = []
    for s in nodesets.batch_specs(count, seed):
        s = dict(s)
        if s["N"] > nmax:
            s["N"] = nmax if s["d"] == 3 else int(math.sqrt(nmax)) ** 2
        out.append(s)
    return out


def as_set(spec, x, prec=0):
    return dict(xyz=gpu(x), n=spec["n"], m=spec["m"], l=spec["l"],
                delta=spec["delta"], prec=prec)


def same(a, b, keys=KEYS):
    for k in keys:
        assert torch.equal(a[k], b[k]), k


def test_batched_equals_single_and_oracle(orbf):
    ctx = orbf.Context(0)
    specs = small_specs(24, 4)
    xs = [nodesets.make_set(s) for s in specs]
    sets = [as_set(s, x) for s, x in zip(specs, xs)]
    # one disk set with boundary rows and the Lebesgue test
    D = nodesets.disk(3000, 120, 1)
    sets.append(dict(xyz=gpu(D["x"]), n=31, m=5, l=4, delta=0.5, tau=5.0,
                     eligible=gpu(D["eligible"]), boundary=gpu(D["boundary"]),
                     normals=gpu(D["normals"])))
    _say(f"[gpu] batched {len(sets)} sets, N total "
         f"{sum(s['xyz'].shape[0] for s in sets)}")
    outs = orbf.build_dm_batched(ctx, sets)
    for i, (s, o) in enumerate(zip(sets, outs)):
        r = orbf.build_dm(s["xyz"], s["n"], s["m"], s["l"], s["delta"],
                          tau=s.get("tau", math.inf),
                          eligible=s.get("eligible"),
                          boundary=s.get("boundary"),
                          normals=s.get("normals"), ctx=ctx)
        same(o, r)
        assert int(o["n_centers"].item()) == int(r["n_centers"].item())
    # the oracle on a few sets (bit-exact structure, 1e-9 weights)
    for i in (0, 5, 11, len(sets) - 1):
        s = sets[i]
        x = s["xyz"].cpu().numpy()
        el = s.get("eligible")
        ref = oracle.build_dm(
            x, s["n"], s["m"], s["l"], s["delta"], tau=s.get("tau", math.inf),
            eligible=None if el is None else el.cpu().numpy(),
            boundary=None if s.get("boundary") is None
            else s["boundary"].cpu().numpy(),
            normals=None if s.get("normals") is None
            else s["normals"].cpu().numpy())
        o = outs[i]
        assert np.array_equal(o["knn"].cpu().numpy(), ref["knn"])
        assert np.array_equal(o["owner"].cpu().numpy(), ref["owner"])
        assert np.array_equal(o["col"].cpu().numpy(), ref["col"])
        own = ref["owner"] >= 0
        W = o["W"].cpu().numpy()[own]
        err = float((np.abs(W - ref["W"][own]).max(1) /
                     np.abs(ref["W"][own]).max(1)).max())
        _say(f"[gpu] batched set {i}: N={len(x)} d={x.shape[1]} "
             f"max row rel err {err:.2e}")
        assert err <= 1e-9


def test_batched_graph_replay(orbf):
    """The second identical call is captured, later ones replayed; every
    call must reproduce the eager result, with eager work in between."""
    ctx = orbf.Context(0)
    specs = small_specs(16, 7)
    sets = [as_set(s, nodesets.make_set(s)) for s in specs]
    outs = orbf.build_dm_batched(ctx, sets)
    ref = [{k: o[k].clone() for k in KEYS} for o in outs]
    for rep in range(4):
        for o in outs:
            for k in KEYS:
                o[k].zero_()
        torch.cuda.synchronize()
        orbf.build_dm_batched(ctx, sets, outputs=outs)
        _say(f"[gpu] graph replay {rep}")
        for o, r in zip(outs, ref):
            same(o, r)


def test_graph_replay_meets_a_deeper_covering(orbf):
    """A replayed graph launches the number of covering levels recorded when
    it was captured; one workgroup then runs whatever levels remain.  The
    batch is captured on Halton-ordered nodes (a shallow dependency DAG),
    then the same buffers are refilled with the nodes in lexicographic order
    (a deep one) and the graph replayed: the result must equal an eager
    build of the sorted nodes, and the oracle's covering."""
    ctx = orbf.Context(0)
    spec = dict(d=3, N=12000, n=50, m=5, l=3, delta=0.3)
    x = nodesets.ball(spec["N"], 2)["x"]
    xs = np.ascontiguousarray(x[np.lexsort((x[:, 2], x[:, 1], x[:, 0]))])
    sets = [as_set(spec, x)]
    outs = orbf.build_dm_batched(ctx, sets)
    for _ in range(2):  # captured, then replayed
        orbf.build_dm_batched(ctx, sets, outputs=outs)
    sets[0]["xyz"].copy_(gpu(xs))
    torch.cuda.synchronize()
    _say("[gpu] graph replay on lexicographically ordered nodes")
    orbf.build_dm_batched(ctx, sets, outputs=outs)
    ref = orbf.build_dm(gpu(xs), spec["n"], spec["m"], spec["l"],
                        spec["delta"], ctx=orbf.Context(0))
    same(outs[0], ref)
    idx, rho2 = oracle.knn(xs, spec["n"])
    owner, centers = oracle.cover(xs, idx, rho2, spec["delta"])
    assert np.array_equal(outs[0]["owner"].cpu().numpy(), owner)
    assert np.array_equal(ref["centers"].cpu().numpy()[:len(centers)],
                          centers)


def test_batched_fp32_refined(orbf):
    ctx = orbf.Context(0)
    specs = small_specs(12, 9)
    xs = [nodesets.make_set(s) for s in specs]
    a = orbf.build_dm_batched(ctx, [as_set(s, x) for s, x in zip(specs, xs)])
    b = orbf.build_dm_batched(ctx, [as_set(s, x, orbf.PREC_FP32_IR)
                                    for s, x in zip(specs, xs)])
    worst = 0.0
    for oa, ob in zip(a, b):
        assert torch.equal(oa["owner"], ob["owner"])
        assert torch.equal(oa["col"], ob["col"])
        rel = ((oa["W"] - ob["W"]).abs().amax(1) /
               oa["W"].abs().amax(1)).max().item()
        worst = max(worst, rel)
    _say(f"[gpu] batched fp32+ir vs fp64: max row rel diff {worst:.2e}")
    assert worst <= 1e-9


def _drain(srv, tickets, timeout_s=120.0):
    done = set()
    t0 = srv.now()
    while len(done) < len(tickets):
        done.update(srv.poll())
        assert srv.now() - t0 < timeout_s, "server did not finish"
    return done


def test_server_alone_equals_mix(orbf):
    """A request's outputs are the same alone and among others in flight,
    and equal a single-set build."""
    ctx = orbf.Context(0)
    specs = [dict(s, t=0.0) for s in small_specs(10, 11, nmax=30000)]
    xs = [gpu(nodesets.make_set(s)) for s in specs]
    probe = 3
    srv = orbf.Server(0, slots=4, arena=3 << 30, slot_scratch=256 << 20)
    t = srv.submit(xs[probe], specs[probe]["n"], specs[probe]["m"],
                   specs[probe]["l"], specs[probe]["delta"])
    _drain(srv, [t])
    alone = srv.fetch(t)
    assert srv.result(t)["status"] == 0
    srv.release(t)
    tickets = [srv.submit(x, s["n"], s["m"], s["l"], s["delta"])
               for s, x in zip(specs, xs)]
    _say(f"[gpu] server mix of {len(tickets)}: {srv.stats()}")
    _drain(srv, tickets)
    mixed = srv.fetch(tickets[probe])
    same(mixed, alone)
    for s, x, t in zip(specs, xs, tickets):
        info = srv.result(t)
        assert info["status"] == 0
        assert info["t_arrival"] <= info["t_admit"] <= info["t_done"]
        r = orbf.build_dm(x, s["n"], s["m"], s["l"], s["delta"], ctx=ctx)
        same(srv.fetch(t), r)
        assert info["n_centers"] == int(r["n_centers"].item())
        srv.release(t)
    assert srv.stats()["arena_used"] == 0
    srv.close()


def test_moving_nodes_rebuilt_each_step(orbf):
    """Dynamic domains (Sec. 8 motivates per-step rebuilds for moving
    nodes): a 20k-node ball that moves each step (rotation about z plus a
    small random drift) is rebuilt through the request engine every step.
    Every step's DM equals a direct build of the same nodes bit for bit, and
    the first step's stencils and covering equal the oracle's."""
    ctx = orbf.Context(0)
    x0 = nodesets.ball(20000, 2)["x"]
    rng = np.random.default_rng(5)
    n, m, l, delta = 50, 5, 3, 0.3
    srv = orbf.Server(0, slots=2, arena=2 << 30, slot_scratch=512 << 20)
    x = x0.copy()
    lat = []
    for step in range(6):
        th = 0.02 * step
        R = np.array([[np.cos(th), -np.sin(th), 0.0],
                      [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
        x = x0 @ R.T + 1e-4 * rng.standard_normal(x0.shape)
        xd = gpu(x)
        t = srv.submit(xd, n, m, l, delta)
        _drain(srv, [t])
        info = srv.result(t)
        assert info["status"] == 0
        lat.append(1e3 * (info["t_done"] - info["t_arrival"]))
        got = srv.fetch(t)
        ref = orbf.build_dm(xd, n, m, l, delta, ctx=ctx)
        same(got, ref)
        if step == 0:
            idx, rho2 = oracle.knn(x, n)
            owner, _ = oracle.cover(x, idx, rho2, delta)
            assert np.array_equal(got["knn"].cpu().numpy(), idx)
            assert np.array_equal(got["owner"].cpu().numpy(), owner)
        srv.release(t)
    _say(f"[gpu] moving 20k-node ball: rebuild latency per step (ms) "
         f"{['%.2f' % v for v in lat]}")
    srv.close()


def test_server_waits_for_device_written_coordinates(orbf):
    """Coordinates produced on the device, on a side stream that is still
    busy when the request is submitted: the request's slot stream waits for
    the event Server.submit records on the submitting stream, so the build
    sees the finished coordinates (a DM equal to a direct build of them)
    and never the zeros the buffer held before."""
    ctx = orbf.Context(0)
    x0 = gpu(nodesets.ball(20000, 2)["x"])
    n, m, l, delta = 50, 5, 3, 0.3
    srv = orbf.Server(0, slots=2, arena=2 << 30, slot_scratch=512 << 20)
    side = torch.cuda.Stream()
    tickets, coords = [], []
    for step in range(3):
        x = torch.zeros_like(x0)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            # a long product first, so the side stream is still busy at submit
            a = torch.randn(4096, 4096, dtype=torch.float64, device="cuda:0")
            for _ in range(4):
                a = a @ a
                a = a / a.abs().max()
            th = 0.05 * (step + 1)
            R = torch.tensor([[math.cos(th), -math.sin(th), 0.0],
                              [math.sin(th), math.cos(th), 0.0],
                              [0.0, 0.0, 1.0]], dtype=torch.float64,
                             device="cuda:0")
            x.copy_(x0 @ R.T + 0.0 * a[:1, :1])
            tickets.append(srv.submit(x, n, m, l, delta))
        coords.append(x)
    _drain(srv, tickets)
    torch.cuda.synchronize()
    for t, x in zip(tickets, coords):
        info = srv.result(t)
        assert info["status"] == 0
        got = srv.fetch(t)
        ref = orbf.build_dm(x, n, m, l, delta, ctx=ctx)
        same(got, ref)
        srv.release(t)
    srv.close()
    _say("[gpu] server built device-written coordinates after their event")


def test_server_budget_admission(orbf):
    """With an arena that holds about two requests at a time, requests wait
    for memory, the head is passed a bounded number of times, and every
    result is still right."""
    specs = [dict(s) for s in small_specs(8, 13, nmax=20000)]
    xs = [gpu(nodesets.make_set(s)) for s in specs]
    L = orbf.lib()
    need = max(L.orbf_request_bytes(x.shape[0], x.shape[1], s["n"], 0)
               for s, x in zip(specs, xs))
    ws = max(L.orbf_workspace_size(x.shape[0], x.shape[1], s["n"], s["l"], 0)
             for s, x in zip(specs, xs))
    arena = int(need * 2.3)  # the largest request fits, three do not
    ctx = orbf.Context(0)
    refs = [orbf.build_dm(x, s["n"], s["m"], s["l"], s["delta"], ctx=ctx)
            for s, x in zip(specs, xs)]
    srv = orbf.Server(0, slots=4, arena=arena, slot_scratch=ws)
    tickets = [srv.submit(x, s["n"], s["m"], s["l"], s["delta"])
               for s, x in zip(specs, xs)]
    index = {t: i for i, t in enumerate(tickets)}
    # a finished request holds its arena memory until released, so results
    # are consumed as they come
    done, waited = set(), 0
    t0 = srv.now()
    while len(done) < len(tickets):
        assert srv.now() - t0 < 60.0, f"stalled: {srv.stats()}"
        fin = srv.poll()
        st = srv.stats()
        assert st["arena_used"] <= st["arena_bytes"]
        waited = max(waited, st["waiting"])
        for t in fin:
            assert srv.result(t)["status"] == 0
            same(srv.fetch(t), refs[index[t]])
            srv.release(t)
            done.add(t)
    _say(f"[gpu] arena {arena >> 20} MiB: max waiting {waited}")
    assert waited > 0
    assert srv.stats()["arena_used"] == 0
    srv.close()


def test_server_and_batch_errors(orbf):
    srv = orbf.Server(0, slots=2, arena=48 << 20, slot_scratch=16 << 20)
    x = gpu(np.random.default_rng(0).random((500, 2)))
    with pytest.raises(orbf.OrbfError) as e:
        srv.submit(x, 8, 4, 2, 0.5)  # even PHS exponent
    assert e.value.code == orbf.EINVAL
    big = gpu(np.random.default_rng(1).random((400000, 3)))
    with pytest.raises(orbf.OrbfError) as e:
        srv.submit(big, 50, 5, 3, 0.3)  # outputs larger than the arena
    assert e.value.code == orbf.EBUDGET
    srv.close()
    ctx = orbf.Context(0)
    with pytest.raises(orbf.OrbfError) as e:
        orbf.build_dm_batched(ctx, [dict(xyz=x, n=8, m=3, l=2, delta=1.5)])
    assert e.value.code == orbf.EINVAL


def test_schedules_and_tuner(orbf):
    """Every schedule gives the oracle's weights (the two one-wavefront
    schedules bit for bit alike); the table rejects what a kernel cannot
    serve; the tuner picks one candidate per (K, p-class)."""
    from paper_1606_03135_amd import tune
    ctx = orbf.Context(0)
    x = nodesets.ball(6000, 2)["x"]
    xd = gpu(x)
    n, m, l, delta = 50, 5, 3, 0.3  # K = 70
    K = n + 20
    pc = tune.pclass(n, 3, delta)
    ref = oracle.build_dm(x, n, m, l, delta)
    own = ref["owner"] >= 0
    out = {}
    for name in ("wave16", "wave8", "group16", "matrix", "split"):
        tune.set_schedule(ctx, K, pc, name)
        r = orbf.build_dm(xd, n, m, l, delta, ctx=ctx)
        W = r["W"].cpu().numpy()
        err = float((np.abs(W[own] - ref["W"][own]).max(1) /
                     np.abs(ref["W"][own]).max(1)).max())
        _say(f"[gpu] schedule {name}: max row rel err {err:.2e}")
        assert err <= 1e-9
        out[name] = r["W"]
    assert torch.equal(out["wave16"], out["wave8"])
    assert torch.equal(out["wave16"], out["split"])
    assert (K, pc, "split") in tune.get_schedules(ctx)
    with pytest.raises(orbf.OrbfError):
        tune.set_schedule(ctx, 100, 0, "wave16")  # K > 72
    with pytest.raises(orbf.OrbfError):
        tune.set_schedule(ctx, 100, 0, "split")
    tune.set_schedule(ctx, K, pc, None)
    assert tune.get_schedules(ctx) == []
    specs = small_specs(6, 21, nmax=4000)
    sets = [as_set(s, nodesets.make_set(s)) for s in specs]
    rep, secs = tune.tune_sets(ctx, sets, reps=2)
    _say(f"[gpu] tuner: {len(rep)} classes in {secs:.1f} s")
    assert {(r["K"], r["pclass"]) for r in rep} == {
        (K_, p_) for K_, p_, _ in tune.get_schedules(ctx)}


@pytest.mark.parametrize("case", ["disk_K46", "ball_K60", "disk_K67_rows"])
def test_matrix_schedule_matches_oracle(orbf, case):
    """The matrix-core schedule (blocked elimination with FP64 matrix
    instructions) against the oracle at each tile count it instantiates
    (3, 4 and 5 row tiles of 16: K = 46, 60, 67), on covered rows and on
    explicit Neumann rows with normals; several right-hand-side passes
    where a stencil keeps more than 16 rows."""
    from paper_1606_03135_amd import tune
    ctx = orbf.Context(0)
    if case == "disk_K46":
        D = nodesets.disk(5000, 200, 3)
        x, n, m, l, delta = D["x"], 31, 5, 4, 0.2
    elif case == "ball_K60":
        x, n, m, l, delta = nodesets.ball(6000, 3)["x"], 40, 5, 3, 0.2
    else:
        D = nodesets.disk(4000, 160, 4, refine=True)
        x, n, m, l, delta = D["x"], 46, 5, 5, 0.5
    d = x.shape[1]
    M = math.comb(l + d, d)
    K = n + M
    pc = tune.pclass(n, d, delta)
    tune.set_schedule(ctx, K, pc, "matrix")
    tune.set_schedule(ctx, K, 0, "matrix")
    tune.set_schedule(ctx, K, 1, "matrix")
    if case == "disk_K67_rows":
        bd = D["boundary"]
        ref = oracle.build_dm(x, n, m, l, delta, eligible=D["eligible"],
                              boundary=bd, normals=D["normals"])
        r = orbf.build_dm(gpu(x), n, m, l, delta, eligible=gpu(D["eligible"]),
                          boundary=gpu(bd), normals=gpu(D["normals"]),
                          ctx=ctx)
    else:
        ref = oracle.build_dm(x, n, m, l, delta)
        r = orbf.build_dm(gpu(x), n, m, l, delta, ctx=ctx)
    assert np.array_equal(r["owner"].cpu().numpy(), ref["owner"])
    W = r["W"].cpu().numpy()
    own = ref["owner"] >= 0
    err = float((np.abs(W[own] - ref["W"][own]).max(1) /
                 np.abs(ref["W"][own]).max(1)).max())
    pmax = int(np.bincount(ref["owner"][own]).max())
    _say(f"[gpu] matrix schedule {case}: K={K}, up to {pmax} rows per "
         f"stencil, max row rel err {err:.2e}")
    assert err <= 1e-9
    with pytest.raises(orbf.OrbfError):
        tune.set_schedule(ctx, 81, 0, "matrix")  # beyond five row tiles


def test_split_schedule_without_cached_counts(orbf):
    """The split schedule takes each stencil's row count from the covering
    when handed its own centers/owner arrays, and counts them itself
    otherwise; both give the single-launch weights bit for bit, on a set
    whose stencils span all three pass widths."""
    from paper_1606_03135_amd import tune
    ctx = orbf.Context(0)
    x = gpu(nodesets.ball(20000, 5)["x"])
    n, m, l, delta = 50, 5, 3, 0.3
    knn, rho2 = orbf.build_nodes_knn(ctx, x, n)
    centers, nc, owner, p = orbf.select_overlapped_stencils(
        ctx, x, knn, rho2, delta)
    k = int(nc.item())
    pk = p[:k].cpu().numpy()
    _say(f"[gpu] split: {k} stencils, p<=8 {(pk <= 8).sum()}, "
         f"p<=16 {((pk > 8) & (pk <= 16)).sum()}, p>16 {(pk > 16).sum()}")
    assert (pk <= 8).any() and ((pk > 8) & (pk <= 16)).any() and (pk > 16).any()
    K, pc = n + 20, tune.pclass(n, 3, delta)

    def weights(name, c, nn, o):
        tune.set_schedule(ctx, K, pc, name)
        W = orbf.compute_weights(ctx, orbf.OP_LAPLACIAN, m, l, n, delta, x,
                                 knn, rho2, centers=c, n_centers=nn, owner=o)
        ctx.sync()
        return W.clone()

    one = weights("wave16", centers, nc, owner)
    cached = weights("split", centers, nc, owner)
    counted = weights("split", centers.clone(), nc.clone(), owner.clone())
    own = owner >= 0
    assert torch.equal(one[own], cached[own])
    assert torch.equal(one[own], counted[own])
