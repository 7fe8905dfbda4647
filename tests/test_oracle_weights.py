"""Pins of the oracle's local weights (eqs. rbffd_linsys, orbffd_eq,
orbffd_rhs of Sec. 4.1) and of the DM rows built from them.

What fixes the weights independently of the oracle's own code:
  - the constraint block row of eq. rbffd_linsys: the weights reproduce L on
    every polynomial of degree <= l (checked with sympy-derived derivatives);
  - 40-digit brute force: the same saddle system assembled from sympy
    derivatives of r^m and solved by mpmath LU;
  - the n = M closed form (polynomial finite differences);
  - delta = 1 recovers standard RBF-FD (Sec. 4.1); the column of a node does
    not depend on the other right-hand sides;
  - translation / rotation invariance, exact power-of-two scaling;
  - convergence of the DM Laplacian on smooth functions (Sec. 4.2.2 error
    estimate: order h^(l+1-theta) with theta = 2);
  - the degree rule of Sec. 2 with its printed values.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest
import sympy as sp

import nodesets
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def exps(d, l):
    out = []
    for deg in range(l + 1):
        if d == 2:
            out += [(a, deg - a) for a in range(deg, -1, -1)]
        else:
            out += [(a, b, deg - a - b) for a in range(deg, -1, -1)
                    for b in range(deg - a, -1, -1)]
    return out


def test_degree_rule_printed_values():
    g = json.load(open(os.path.join(GOLD, "degree_rule.json")))
    for c in g["cases"]:
        assert oracle.degree_rule(c["d"], c["n"]) == (c["s"], c["M"])
    for n in range(3, 400):  # the 2D closed form of Sec. 2
        s = math.floor(0.5 * (math.sqrt(4 * n + 1) - 3))
        assert oracle.degree_rule(2, n)[0] == s
    # the workloads' (n, l) pairs follow the same rule
    assert oracle.degree_rule(2, 12)[0] == 2
    assert oracle.degree_rule(2, 31)[0] == 4
    assert oracle.degree_rule(3, 50)[0] == 3


def _sym_ops(d, m):
    """sympy: Laplacian and gradient of |x - y|^m, as functions of (x, y)."""
    X = sp.symbols("x0:%d" % d, real=True)
    Y = sp.symbols("y0:%d" % d, real=True)
    r2 = sum((X[a] - Y[a]) ** 2 for a in range(d))
    phi = r2 ** sp.Rational(m, 2)
    lap = sp.simplify(sum(sp.diff(phi, X[a], 2) for a in range(d)))
    grad = [sp.simplify(sp.diff(phi, X[a])) for a in range(d)]
    return X, Y, phi, lap, grad


def _poly_ops(d, l, X):
    mons = [sp.Mul(*[X[a] ** e[a] for a in range(d)]) for e in exps(d, l)]
    laps = [sum(sp.diff(p, X[a], 2) for a in range(d)) for p in mons]
    grads = [[sp.diff(p, X[a]) for a in range(d)] for p in mons]
    return mons, laps, grads


def _stencil(rng, d, n, jitter=0.3):
    # quasi-uniform local cloud around the origin
    g = int(math.ceil(n ** (1.0 / d))) + 2
    ax = np.arange(g) - g // 2
    pts = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), -1).reshape(-1, d)
    pts = pts + rng.uniform(-jitter, jitter, pts.shape)
    o = np.argsort((pts * pts).sum(1), kind="stable")[:n]
    return pts[o] - pts[o[0]]


@pytest.mark.parametrize("d,m,l,n,op", [(2, 3, 2, 12, 0), (2, 5, 4, 31, 0),
                                        (3, 5, 3, 50, 0), (2, 5, 3, 21, 1),
                                        (3, 3, 2, 25, 1), (2, 7, 4, 40, 0)])
def test_polynomial_reproduction(d, m, l, n, op):
    """Second block row of eq. rbffd_linsys: sum_j w_j p(x_j) = L p(x_e)."""
    rng = np.random.default_rng(7 + n)
    P = _stencil(rng, d, n) * 0.01 + 0.3
    E = P[[0, 1, 3, n // 2]]
    nrm = None
    if op == 1:
        v = rng.normal(size=(len(E), d))
        nrm = v / np.linalg.norm(v, axis=1, keepdims=True)
    W = oracle.stencil_weights(P, E, m, l, op, nrm)
    X = sp.symbols("x0:%d" % d, real=True)
    mons, laps, grads = _poly_ops(d, l, X)
    rho = math.sqrt(((P - P[0]) ** 2).sum(1).max())
    for p, lp, gp in zip(mons, laps, grads):
        # monomials in local scaled coordinates keep the check well scaled
        sub = lambda q: {X[a]: (q[a] - P[0][a]) / rho for a in range(d)}
        vals = np.array([float(p.subs(sub(q))) for q in P])
        for e in range(len(E)):
            if op == 0:
                target = float(lp.subs(sub(E[e]))) / rho ** 2
            else:
                target = sum(float(gp[a].subs(sub(E[e]))) * nrm[e][a]
                             for a in range(d)) / rho
            got = float(np.dot(W[e], vals))
            scale = float(np.abs(W[e] * vals).sum()) + abs(target)
            assert abs(got - target) <= 1e-10 * scale, (p, e, got, target)


def test_row_sums_vanish():
    x = nodesets.square(45, 0)
    D = oracle.build_dm(x, 12, 3, 2, 0.5)
    h2 = (1 / 45) ** 2
    rs = np.add.reduceat(D["val"], D["row_ptr"][:-1])
    assert np.abs(rs).max() * h2 < 1e-11


@pytest.mark.parametrize("d,m,l,n,op", [(2, 3, 2, 12, 0), (2, 5, 2, 14, 1),
                                        (3, 3, 1, 12, 0), (2, 5, 3, 16, 0),
                                        (2, 3, -1, 12, 0), (3, 5, -1, 16, 1)])
def test_mpmath_bruteforce(d, m, l, n, op):
    """40-digit solve of the same saddle system, assembled from sympy
    derivatives of |x - y|^m, against the FP64 oracle (l = -1: no
    polynomial block, the unaugmented system A w = L phi)."""
    mpmath.mp.dps = 40
    rng = np.random.default_rng(11 + n + op)
    P = _stencil(rng, d, n)
    E = P[[0, 2, n - 1]]
    nrm = None
    if op == 1:
        v = rng.normal(size=(len(E), d))
        nrm = v / np.linalg.norm(v, axis=1, keepdims=True)
    W = oracle.stencil_weights(P, E, m, l, op, nrm)

    X, Y, phi, lap, grad = _sym_ops(d, m)
    mons, laps, grads = _poly_ops(d, l, X)
    f_phi = sp.lambdify(X + Y, phi, "mpmath")
    f_lap = sp.lambdify(X + Y, lap, "mpmath")
    f_grad = [sp.lambdify(X + Y, g, "mpmath") for g in grad]
    f_mon = [sp.lambdify(X, p, "mpmath") for p in mons]
    f_mlap = [sp.lambdify(X, p, "mpmath") for p in laps]
    f_mgrad = [[sp.lambdify(X, g, "mpmath") for g in gp] for gp in grads]
    M = len(mons)
    K = n + M
    Pm = [[mpmath.mpf(float(v)) for v in row] for row in P]
    A = mpmath.matrix(K, K)
    for i in range(n):
        for j in range(n):
            A[i, j] = f_phi(*(Pm[i] + Pm[j]))
        for t in range(M):
            A[i, n + t] = A[n + t, i] = f_mon[t](*Pm[i])
    for e in range(len(E)):
        Em = [mpmath.mpf(float(v)) for v in E[e]]
        B = mpmath.matrix(K, 1)
        for j in range(n):
            if op == 0:
                B[j] = f_lap(*(Em + Pm[j]))
            else:
                B[j] = sum(f_grad[a](*(Em + Pm[j])) * nrm[e][a]
                           for a in range(d))
        for t in range(M):
            if op == 0:
                B[n + t] = f_mlap[t](*Em)
            else:
                B[n + t] = sum(f_mgrad[t][a](*Em) * nrm[e][a]
                               for a in range(d))
        sol = mpmath.lu_solve(A, B)
        ref = np.array([float(sol[j]) for j in range(n)])
        err = np.abs(W[e] - ref).max() / np.abs(ref).max()
        assert err < 1e-11, err


def test_closed_form_polynomial_fd():
    g = json.load(open(os.path.join(GOLD, "closed_form_fd.json")))
    for c in g["cases"]:
        h = 0.0625  # power of two: the stencil is exact in binary
        P = np.array(c["offsets"], float) * h + 0.5
        for m in (3, 5, 7):  # independent of the kernel when n = M
            W = oracle.stencil_weights(P, P[:1], m, c["l"])
            ref = np.array(c["weights_times_h2"], float) / h ** 2
            assert np.abs(W[0] - ref).max() <= 1e-9 * np.abs(ref).max()


def test_delta_one_column_is_standard_rbffd():
    """delta = 1 recovers RBF-FD (Sec. 4.1); a center's column is the same,
    bit for bit, whatever other columns are solved with it."""
    x = nodesets.disk(4000, 150, 1)
    X, el = x["x"], x["eligible"]
    idx, rho2 = oracle.knn(X, 31)
    one = oracle.overlapped_rows(X, idx, rho2, 5, 4, 1.0, eligible=el)
    half = oracle.overlapped_rows(X, idx, rho2, 5, 4, 0.5, eligible=el)
    c = half["centers"]
    assert np.array_equal(one["W"][c], half["W"][c])
    assert np.array_equal(one["owner"][el == 1], np.nonzero(el)[0])


def test_invariances():
    rng = np.random.default_rng(3)
    P = _stencil(rng, 3, 50) * 0.02
    E = P[[0, 5, 9]]
    W = oracle.stencil_weights(P, E, 5, 3)
    # translation
    t = np.array([0.37, -0.21, 0.44])
    Wt = oracle.stencil_weights(P + t, E + t, 5, 3)
    assert np.abs(Wt - W).max() <= 1e-9 * np.abs(W).max()
    # rotation (the Laplacian is rotation invariant)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Wr = oracle.stencil_weights(P @ Q.T, E @ Q.T, 5, 3)
    assert np.abs(Wr - W).max() <= 1e-9 * np.abs(W).max()
    # scaling by 2^k: every step is exact, the weights scale by 4^-k
    for k in (-3, 1, 5):
        Ws = oracle.stencil_weights(P * 2.0 ** k, E * 2.0 ** k, 5, 3)
        assert np.array_equal(Ws, W * 4.0 ** (-k))


@pytest.mark.parametrize("d,n,m,l,delta", [(2, 12, 3, 2, 1.0),
                                           (2, 31, 5, 4, 0.5),
                                           (3, 30, 5, 2, 0.3)])
def test_convergence_order(d, n, m, l, delta):
    """Error estimate of Sec. 4.2.2: the DM Laplacian of a smooth function
    converges like h^(l+1-2); the fitted slope of the RMS error over
    interior nodes must reach l-1-0.25."""
    hs, errs = [], []
    sizes = [30, 60, 120, 240] if d == 2 else [16, 22, 30, 40]
    for g in sizes:
        if d == 2:
            x = nodesets.square(g, 5)
            f = np.sin(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])
            lapf = -2 * np.pi ** 2 * f
        else:
            ax = (np.arange(g) + 0.5) / g
            x = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1)
            x = x.reshape(-1, 3)
            x = x + np.random.default_rng(g).uniform(-0.2 / g, 0.2 / g, x.shape)
            f = (np.sin(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1])
                 * np.sin(np.pi * x[:, 2]))
            lapf = -3 * np.pi ** 2 * f
        D = oracle.build_dm(x, n, m, l, delta)
        Lf = np.add.reduceat(D["val"] * f[D["col"]], D["row_ptr"][:-1])
        rho = np.sqrt(D["rho2"]).max()
        inner = np.all((x > 2 * rho) & (x < 1 - 2 * rho), axis=1)
        hs.append(1.0 / g)
        # l2-type (RMS) error over nodes two stencil widths from the edge
        errs.append(np.sqrt(np.mean((Lf - lapf)[inner] ** 2)))
    assert np.all(np.isfinite(errs)), errs
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert slope >= l - 1 - 0.25, (slope, errs)
