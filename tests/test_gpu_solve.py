"""Implicit time step with a DM on the GPU (orbf_solve_implicit, Sec. 5)
against the oracle's direct sparse solve of the same system.

The DMs are the oracle's own (built on the CPU and uploaded), so neither
the input nor the expected value comes from the HIP path.  Bars: the
solution within 1e-9 of the direct solve relative to its largest entry
(tol 1e-12 on the residual; the systems here have condition numbers of at
most a few thousand), and the true residual ||b - A x|| / ||b||, recomputed
on the CPU, below 1e-10.
"""
import ctypes
import sys

import numpy as np
import pytest

import nodesets
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def ctx(orbf):
    return orbf.Context(0)


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.fixture(scope="module")
def disk_dm():
    """2D disk, 3000 interior + 120 boundary nodes, n = 31, r^5, l = 4,
    delta = 0.5: Laplacian rows inside, normal-derivative rows on the
    boundary."""
    D = nodesets.disk(3000, 120, 1)
    ref = oracle.build_dm(D["x"], 31, 5, 4, 0.5, eligible=D["eligible"],
                          boundary=D["boundary"], normals=D["normals"])
    return D, ref


@pytest.fixture(scope="module")
def ball_dm():
    """3D ball, 6000 nodes, n = 50, r^5, l = 3, delta = 0.3 (Laplacian rows
    everywhere)."""
    x = nodesets.ball(6000, 2)["x"]
    return x, oracle.build_dm(x, 50, 5, 3, 0.3)


def _check(orbf, ctx, ref, b, kind, alpha, beta, x0=None, tag="",
           precond="none"):
    rp, col, val = ref["row_ptr"], ref["col"], ref["val"]
    want = oracle.solve_implicit(rp, col, val, b, kind, alpha, beta)
    x, it, res = orbf.solve_implicit(
        ctx, gpu(rp), gpu(col), gpu(val), gpu(b), alpha=alpha, beta=beta,
        row_kind=None if kind is None else gpu(kind),
        x0=None if x0 is None else gpu(x0), tol=1e-12, max_iter=2000,
        precond=precond)
    got = x.cpu().numpy()
    A = oracle.implicit_system(rp, col, val, kind, alpha, beta)
    true_res = np.linalg.norm(b - A @ got) / np.linalg.norm(b)
    err = np.abs(got - want).max() / np.abs(want).max()
    _say(f"[gpu] solve {tag} ({precond}): {it} iterations, "
         f"relres {res:.2e}, "
         f"true {true_res:.2e}, err vs direct {err:.2e}")
    assert res <= 1e-12
    assert true_res <= 1e-10
    assert err <= 1e-9
    return got, it, res


@pytest.mark.parametrize("precond", ["none", "jacobi"])
@pytest.mark.parametrize("bc,dt", [("dirichlet", 1e-3), ("dirichlet", 1e-2),
                                   ("neumann", 1e-3), ("neumann", 1e-4)])
def test_heat_step_on_disk(orbf, ctx, disk_dm, bc, dt, precond):
    """Backward Euler for u_t = Laplacian u on the disk: the paper's system
    with Dirichlet (boundary rows x_b = 0) or Neumann (the DM's
    normal-derivative rows = 0) data, from u0 = exp(-4 |x|^2)."""
    D, ref = disk_dm
    x = D["x"]
    N = len(x)
    kind = np.ones(N, np.uint8)
    kind[D["boundary"]] = 0 if bc == "dirichlet" else 2
    u0 = np.exp(-4.0 * (x ** 2).sum(1))
    b = u0.copy()
    b[kind != 1] = 0.0
    _check(orbf, ctx, ref, b, kind, 1.0, -dt, x0=u0, tag=f"disk {bc} {dt}",
           precond=precond)


def test_all_rows_shifted_ball(orbf, ctx, ball_dm):
    """row_kind NULL: A = alpha I + beta L on every row of a 3D ball DM."""
    x, ref = ball_dm
    b = np.cos(3 * x[:, 0]) * np.sin(2 * x[:, 1]) + x[:, 2]
    _check(orbf, ctx, ref, b, None, 2.0, -1e-4, tag="ball alpha=2")


def test_deterministic_and_zero_iterations(orbf, ctx, disk_dm):
    D, ref = disk_dm
    N = len(D["x"])
    kind = np.ones(N, np.uint8)
    kind[D["boundary"]] = 0
    rng = np.random.default_rng(4)
    b = rng.standard_normal(N)
    args = (gpu(ref["row_ptr"]), gpu(ref["col"]), gpu(ref["val"]), gpu(b))
    x1, it1, r1 = orbf.solve_implicit(ctx, *args, row_kind=gpu(kind),
                                      beta=-1e-3, tol=1e-11)
    x2, it2, r2 = orbf.solve_implicit(ctx, *args, row_kind=gpu(kind),
                                      beta=-1e-3, tol=1e-11)
    assert it1 == it2 and r1 == r2
    assert torch.equal(x1, x2)
    # max_iter = 0: x0 comes back unchanged with its own residual
    x0 = rng.standard_normal(N)
    x, it, res = orbf.solve_implicit(ctx, *args, row_kind=gpu(kind),
                                     beta=-1e-3, x0=gpu(x0), max_iter=0)
    assert it == 0
    assert np.array_equal(x.cpu().numpy(), x0)
    A = oracle.implicit_system(ref["row_ptr"], ref["col"], ref["val"], kind,
                               1.0, -1e-3)
    assert res == pytest.approx(np.linalg.norm(b - A @ x0) /
                                np.linalg.norm(b), rel=1e-12)
    # b = 0 from x0 = 0: the solution is 0 at once
    z, it, res = orbf.solve_implicit(ctx, args[0], args[1], args[2],
                                     gpu(np.zeros(N)), row_kind=gpu(kind))
    assert it == 0 and res == 0.0 and not z.any()


def test_solve_errors(orbf, ctx, disk_dm):
    _, ref = disk_dm
    rp, col, val = (gpu(ref["row_ptr"]), gpu(ref["col"]), gpu(ref["val"]))
    N = rp.numel() - 1
    b = torch.ones(N, dtype=torch.float64, device="cuda:0")
    L = orbf.lib()
    P = orbf._ptr
    it = ctypes.c_int(0)
    res = ctypes.c_double(0.0)
    common = (P(rp), P(col), P(val), None)

    def call(n, alpha, beta, bp, xp, tol, mi, pc=0):
        return L.orbf_solve_implicit(ctx._h, n, *common, alpha, beta, bp, xp,
                                     tol, mi, pc, ctypes.byref(it),
                                     ctypes.byref(res))

    x = torch.zeros_like(b)
    assert call(N, 1.0, -1e-3, P(b), P(b), 1e-10, 10) == orbf.EINVAL
    assert call(N, 1.0, -1e-3, P(b), P(x), -1.0, 10) == orbf.EINVAL
    assert call(N, 1.0, -1e-3, P(b), P(x), float("nan"), 10) == orbf.EINVAL
    assert call(N, 1.0, -1e-3, P(b), P(x), 1e-10, -1) == orbf.EINVAL
    assert call(N, float("inf"), -1e-3, P(b), P(x), 1e-10, 5) == orbf.EINVAL
    assert call(0, 1.0, -1e-3, P(b), P(x), 1e-10, 5) == orbf.EINVAL
    assert call(N, 1.0, -1e-3, None, P(x), 1e-10, 5) == orbf.EINVAL
    assert call(N, 1.0, -1e-3, P(b), P(x), 1e-10, 5, 2) == orbf.EINVAL
    with pytest.raises(ValueError):
        orbf.solve_implicit(ctx, rp, col, val, b[:-1])
