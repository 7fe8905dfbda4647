"""BDF time stepping with the DM on the GPU (orbf_bdf_rhs +
orbf_solve_implicit, Sec. 5: BDF4 started by BDF1-3).

- The library's coefficients equal the oracle's, which are derived from
  the formulas' definition and pinned to the BDF4 values the paper prints.
- One step of each order on an oracle-built disk DM (uploaded, so nothing
  expected comes from the HIP path) equals the oracle's step (direct sparse
  solve) within 1e-9 of its largest entry.
- End to end: the forced heat equation u_t = Lap u + f on the disk with
  Dirichlet data and the manufactured solution e^-t (1 + sin(pi x) cos(pi y)),
  BDF4 from BDF1-3, on GPU-built DMs (n = 31, l = 4, delta = 0.5): the RMS
  error at t = 0.05 falls at the order of the error estimate of Sec. 4.2.2,
  h^(l-1) = h^3.  The oracle's run of the same problem at dt = 1e-3
  measures 3.09 over 2k-12k nodes with RMS errors 6.5e-6, 1.2e-6 and
  4.4e-7, which the GPU reproduces to four digits; at 30k nodes that run
  reaches the time-stepping error floor (mostly the O(dt^2) BDF1 start), so
  the test steps at dt = 2.5e-4.
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


def exact(x, t):
    return np.exp(-t) * (1 + np.sin(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1]))


def forcing(x, t):
    s = np.sin(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])
    return np.exp(-t) * (-(1 + s) + 2 * np.pi ** 2 * s)


def test_bdf_coefficients_match_oracle(orbf):
    for k in range(1, 5):
        a, b = orbf.bdf_coefficients(k)
        ra, rb = oracle.bdf_coefficients(k)
        assert np.abs(np.array(a[:k]) - ra).max() <= 1e-14
        assert all(v == 0.0 for v in a[k:])
        assert abs(b - rb) <= 1e-14
    with pytest.raises(ValueError):
        orbf.bdf_coefficients(5)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_one_step_matches_oracle(orbf, ctx, k, bc):
    D = nodesets.disk(3000, 120, 1)
    x = D["x"]
    N = len(x)
    ref = oracle.build_dm(x, 31, 5, 4, 0.5, eligible=D["eligible"],
                          boundary=D["boundary"], normals=D["normals"])
    kind = np.ones(N, np.uint8)
    kind[D["boundary"]] = 0 if bc == "dirichlet" else 2
    rng = np.random.default_rng(10 + k)
    levels = [exact(x, -i * 1e-3) + 0.01 * rng.standard_normal(N)
              for i in range(k)]
    f = forcing(x, 1e-3)
    bv = exact(x, 1e-3) if bc == "dirichlet" else np.zeros(N)
    want = oracle.bdf_step(ref["row_ptr"], ref["col"], ref["val"], levels,
                           1e-3, f=f, row_kind=kind, bvals=bv)
    got, it, res = orbf.bdf_step(
        ctx, gpu(ref["row_ptr"]), gpu(ref["col"]), gpu(ref["val"]),
        [gpu(u) for u in levels], 1e-3, f=gpu(f), row_kind=gpu(kind),
        bvals=gpu(bv), tol=1e-12)
    err = np.abs(got.cpu().numpy() - want).max() / np.abs(want).max()
    _say(f"[gpu] BDF{k} {bc}: {it} iterations, err vs oracle {err:.2e}")
    assert err <= 1e-9


def test_bdf_rhs_errors(orbf, ctx):
    u = torch.ones(10, dtype=torch.float64, device="cuda:0")
    L = orbf.lib()
    P = orbf._ptr
    r = torch.empty_like(u)
    assert L.orbf_bdf_rhs(ctx._h, 10, 2, P(u), None, None, None, None, 1e-3,
                          None, None, P(r)) == orbf.EINVAL
    assert L.orbf_bdf_rhs(ctx._h, 10, 5, P(u), P(u), P(u), P(u), None, 1e-3,
                          None, None, P(r)) == orbf.EINVAL
    assert L.orbf_bdf_rhs(ctx._h, 10, 1, P(u), None, None, None, None, 0.0,
                          None, None, P(r)) == orbf.EINVAL
    assert L.orbf_bdf_rhs(ctx._h, 10, 1, P(u), None, None, None, None, 1e-3,
                          None, None, P(u)) == orbf.EINVAL
    assert L.orbf_bdf_rhs(ctx._h, 10, 1, P(u), None, None, None, None, 1e-3,
                          None, None, P(r)) == orbf.OK


def test_heat_equation_bdf4_converges(orbf, ctx):
    dt, T = 2.5e-4, 0.05
    hs, errs = [], []
    for Ni in (2000, 5000, 12000, 30000):
        Nb = int(round(3.5 * np.sqrt(Ni)))
        D = nodesets.disk(Ni, Nb, 1)
        x = D["x"]
        N = len(x)
        dm = orbf.build_dm(gpu(x), 31, 5, 4, 0.5,
                           eligible=gpu(D["eligible"]), ctx=ctx)
        kind = gpu(D["eligible"].astype(np.uint8))
        hist = [gpu(exact(x, 0.0))]
        iters = 0
        for s in range(int(round(T / dt))):
            t1 = (s + 1) * dt
            un, it, res = orbf.bdf_step(
                ctx, dm["row_ptr"], dm["col"], dm["val"], hist, dt,
                f=gpu(forcing(x, t1)), row_kind=kind,
                bvals=gpu(exact(x, t1)), tol=1e-12)
            assert res <= 1e-12
            iters += it
            hist = [un] + hist[:3]
        e = hist[0].cpu().numpy() - exact(x, T)
        inner = D["eligible"] != 0
        errs.append(float(np.sqrt(np.mean(e[inner] ** 2))))
        hs.append(1.0 / np.sqrt(N))
        _say(f"[gpu] heat BDF4 N={N}: RMS error {errs[-1]:.3e}, "
             f"{iters} BiCGSTAB iterations over {s + 1} steps")
    order = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    _say(f"[gpu] heat BDF4 observed order {order:.2f} (estimate 3)")
    assert errs[0] < 1e-5 and errs[2] < 7e-7
    assert order >= 2.6, (order, errs)


def test_heat_equation_neumann_refined_disk_converges(orbf, ctx):
    """The paper's disk problem (Sec. 7) on synthetic nodes: u_t = Lap u + f
    with Neumann data on the boundary-refined unit disk, manufactured
    solution u = 1 + e^(-pi t) sin(pi x) cos(pi y) (the forcing
    pi (2 pi - 1) sin(pi x) cos(pi y) e^(-pi t) the paper prints for
    nu = 1), boundary rows = the DM's normal-derivative rows with data
    du/dn, BDF4 from BDF1-3, Jacobi-preconditioned solves.  The RMS error
    at t = 0.05 falls with h."""
    dt, T = 2.5e-4, 0.05
    hs, errs = [], []

    def ex(x, t):
        return 1 + np.exp(-np.pi * t) * np.sin(np.pi * x[:, 0]) * \
            np.cos(np.pi * x[:, 1])

    def fo(x, t):
        return np.pi * (2 * np.pi - 1) * np.sin(np.pi * x[:, 0]) * \
            np.cos(np.pi * x[:, 1]) * np.exp(-np.pi * t)

    def dn(x, t):  # grad u . x on the unit circle
        e = np.exp(-np.pi * t)
        gx = np.pi * np.cos(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])
        gy = -np.pi * np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])
        return e * (gx * x[:, 0] + gy * x[:, 1])

    for Ni in (2000, 5000, 12000, 30000):
        Nb = int(round(3.5 * np.sqrt(Ni)))
        D = nodesets.disk(Ni, Nb, 1, refine=True)
        x, bnd = D["x"], D["boundary"]
        N = len(x)
        dm = orbf.build_dm(gpu(x), 31, 5, 4, 0.5,
                           eligible=gpu(D["eligible"]), boundary=gpu(bnd),
                           normals=gpu(D["normals"]), ctx=ctx)
        kind = np.ones(N, np.uint8)
        kind[bnd] = 2
        kd = gpu(kind)
        hist = [gpu(ex(x, 0.0))]
        iters = 0
        for s in range(int(round(T / dt))):
            t1 = (s + 1) * dt
            bv = np.zeros(N)
            bv[bnd] = dn(x[bnd], t1)
            un, it, res = orbf.bdf_step(
                ctx, dm["row_ptr"], dm["col"], dm["val"], hist, dt,
                f=gpu(fo(x, t1)), row_kind=kd, bvals=gpu(bv), tol=1e-12,
                precond="jacobi")
            assert res <= 1e-12
            iters += it
            hist = [un] + hist[:3]
        e = hist[0].cpu().numpy() - ex(x, T)
        errs.append(float(np.sqrt(np.mean(e ** 2))))
        hs.append(1.0 / np.sqrt(N))
        _say(f"[gpu] Neumann heat BDF4, refined disk N={N}: RMS error "
             f"{errs[-1]:.3e}, {iters} BiCGSTAB iterations")
    order = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    _say(f"[gpu] Neumann heat BDF4 observed order {order:.2f}")
    assert np.all(np.isfinite(errs))
    # observed 3.3 (estimate h^(l-1) = h^3); a lost order fails this
    assert order >= 2.8, (order, errs)
    # recorded RMS error at the finest size: 1.2e-7
    assert errs[-1] <= 2.0e-7, errs
