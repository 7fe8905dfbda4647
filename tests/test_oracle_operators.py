"""Pins of the oracle's first-derivative (d/dx_a) and identity operators
(Sec. 4.1: the right-hand sides of eq. orbffd_rhs are L applied to the RBF
and polynomial basis at the evaluation point; the scaled solve is divided by
rho^theta, theta = 1 for a first derivative and 0 for the identity).

What fixes them independently of the oracle's own code:
  - the constraint block row of eq. rbffd_linsys: the weights reproduce L on
    every polynomial of degree <= l (sympy derivatives), at stencil nodes and
    at points between them;
  - 40-digit brute force: the saddle system assembled from sympy derivatives
    of |x - y|^m (or |x - y|^m itself) and solved by mpmath LU;
  - the identity at a stencil node is the unit vector of that node (the
    interpolant reproduces its data);
  - calculus: central differences of identity weights along e_a converge to
    the d/dx_a weights at second order;
  - exact power-of-two scaling: theta = 1 halves the weights when the
    stencil doubles, theta = 0 leaves them unchanged.
"""
import math

import mpmath
import numpy as np
import pytest
import sympy as sp

import nodesets
import oracle

OPS = {"dx": oracle.OP_DX, "dy": oracle.OP_DY, "dz": oracle.OP_DZ,
       "id": oracle.OP_IDENTITY}


def exps(d, l):
    out = []
    for deg in range(l + 1):
        if d == 2:
            out += [(a, deg - a) for a in range(deg, -1, -1)]
        else:
            out += [(a, b, deg - a - b) for a in range(deg, -1, -1)
                    for b in range(deg - a, -1, -1)]
    return out


def _stencil(rng, d, n, jitter=0.3):
    g = int(math.ceil(n ** (1.0 / d))) + 2
    ax = np.arange(g) - g // 2
    pts = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), -1).reshape(-1, d)
    pts = pts + rng.uniform(-jitter, jitter, pts.shape)
    o = np.argsort((pts * pts).sum(1), kind="stable")[:n]
    return pts[o] - pts[o[0]]


def _L_of(expr, X, op):
    """sympy: L applied to expr (a function of the symbols X)."""
    if op == oracle.OP_IDENTITY:
        return expr
    return sp.diff(expr, X[op - oracle.OP_DX])


@pytest.mark.parametrize("d,m,l,n,name", [(2, 3, 2, 12, "dx"),
                                          (2, 5, 4, 31, "dy"),
                                          (3, 5, 3, 50, "dz"),
                                          (3, 3, 2, 25, "dx"),
                                          (2, 5, 3, 21, "id"),
                                          (3, 5, 3, 50, "id")])
def test_polynomial_reproduction(d, m, l, n, name):
    """sum_j w_j p(x_j) = (L p)(x_e) for every monomial of degree <= l, at
    stencil nodes and at points off the nodes."""
    op = OPS[name]
    rng = np.random.default_rng(17 + n)
    P = _stencil(rng, d, n) * 0.01 + 0.3
    E = np.concatenate([P[[0, 1, n // 2]],
                        0.5 * (P[[2, 4]] + P[[3, 5]])])  # two midpoints
    W = oracle.stencil_weights(P, E, m, l, op)
    X = sp.symbols("x0:%d" % d, real=True)
    rho = math.sqrt(((P - P[0]) ** 2).sum(1).max())
    theta = 0 if op == oracle.OP_IDENTITY else 1
    for e_ in exps(d, l):
        mon = sp.Mul(*[X[a] ** e_[a] for a in range(d)])
        Lm = _L_of(mon, X, op)
        sub = lambda q: {X[a]: (q[a] - P[0][a]) / rho for a in range(d)}
        vals = np.array([float(mon.subs(sub(q))) for q in P])
        for e in range(len(E)):
            target = float(Lm.subs(sub(E[e]))) / rho ** theta
            got = float(np.dot(W[e], vals))
            scale = float(np.abs(W[e] * vals).sum()) + abs(target)
            assert abs(got - target) <= 1e-10 * scale, (e_, e, got, target)


@pytest.mark.parametrize("d,m,l,n,name", [(2, 3, 2, 12, "dx"),
                                          (3, 3, 1, 12, "dz"),
                                          (2, 5, 3, 16, "id"),
                                          (3, 3, 1, 12, "id")])
def test_mpmath_bruteforce(d, m, l, n, name):
    op = OPS[name]
    mpmath.mp.dps = 40
    rng = np.random.default_rng(31 + n + op)
    P = _stencil(rng, d, n)
    E = np.concatenate([P[[0, 2]], 0.5 * (P[[1]] + P[[n - 1]])])
    W = oracle.stencil_weights(P, E, m, l, op)

    X = sp.symbols("x0:%d" % d, real=True)
    Y = sp.symbols("y0:%d" % d, real=True)
    phi = sum((X[a] - Y[a]) ** 2 for a in range(d)) ** sp.Rational(m, 2)
    f_phi = sp.lambdify(X + Y, phi, "mpmath")
    f_Lphi = sp.lambdify(X + Y, _L_of(phi, X, op), "mpmath")
    mons = [sp.Mul(*[X[a] ** e_[a] for a in range(d)]) for e_ in exps(d, l)]
    f_mon = [sp.lambdify(X, p, "mpmath") for p in mons]
    f_Lmon = [sp.lambdify(X, _L_of(p, X, op), "mpmath") for p in mons]
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
            B[j] = f_Lphi(*(Em + Pm[j]))
        for t in range(M):
            B[n + t] = f_Lmon[t](*Em)
        sol = mpmath.lu_solve(A, B)
        ref = np.array([float(sol[j]) for j in range(n)])
        err = np.abs(W[e] - ref).max() / np.abs(ref).max()
        assert err < 1e-11, (e, err)


def test_identity_at_nodes_is_unit_vector():
    rng = np.random.default_rng(5)
    for d, m, l, n in ((2, 5, 4, 31), (3, 5, 3, 50)):
        P = _stencil(rng, d, n) * 0.02 - 0.1
        W = oracle.stencil_weights(P, P, m, l, oracle.OP_IDENTITY)
        assert np.abs(W - np.eye(n)).max() < 1e-10


@pytest.mark.parametrize("d,name", [(2, "dx"), (2, "dy"), (3, "dx"),
                                    (3, "dz")])
def test_derivative_is_limit_of_identity_differences(d, name):
    """(w_id(x + h e_a) - w_id(x - h e_a)) / 2h -> w_a(x) as h -> 0, with
    the error falling like h^2."""
    op = OPS[name]
    a = op - oracle.OP_DX
    rng = np.random.default_rng(3 + d + op)
    n, m, l = (31, 5, 4) if d == 2 else (50, 5, 3)
    P = _stencil(rng, d, n) * 0.05
    x0 = 0.5 * (P[1] + P[2]) + 0.01  # a point off the nodes
    Wd = oracle.stencil_weights(P, x0[None], m, l, op)[0]
    errs = []
    for h in (5e-4, 2.5e-4):  # the node spacing is 0.05
        ea = np.zeros(d)
        ea[a] = h
        Wp = oracle.stencil_weights(P, (x0 + ea)[None], m, l,
                                    oracle.OP_IDENTITY)[0]
        Wm = oracle.stencil_weights(P, (x0 - ea)[None], m, l,
                                    oracle.OP_IDENTITY)[0]
        fd = (Wp - Wm) / (2 * h)
        errs.append(np.abs(fd - Wd).max() / np.abs(Wd).max())
    assert errs[1] < 1e-4
    assert errs[1] < errs[0] / 3.0  # second order: ratio 4 up to rounding


def test_power_of_two_scaling():
    rng = np.random.default_rng(9)
    P = _stencil(rng, 2, 21) * 0.125
    E = P[[0, 3]]
    for op, theta in ((oracle.OP_DX, 1), (oracle.OP_DY, 1),
                      (oracle.OP_IDENTITY, 0)):
        W1 = oracle.stencil_weights(P, E, 5, 3, op)
        W2 = oracle.stencil_weights(2 * P, 2 * E, 5, 3, op)
        assert np.array_equal(W2 * 2 ** theta, W1)


def test_covered_rows_of_each_operator():
    """Rows on the greedy covering: identity rows are unit vectors at the
    node's own stencil position; derivative rows reproduce linear functions;
    the covering does not depend on the operator."""
    x = nodesets.ball(3000, 2)["x"]
    n, m, l, delta = 50, 5, 3, 0.3
    idx, rho2 = oracle.knn(x, n)
    lap = oracle.overlapped_rows(x, idx, rho2, m, l, delta)
    for name in ("dx", "dz", "id"):
        r = oracle.overlapped_rows_op(x, idx, rho2, m, l, delta, OPS[name])
        assert np.array_equal(r["owner"], lap["owner"])
        assert np.array_equal(r["centers"], lap["centers"])
        st = idx[r["owner"]]  # stencil of each row's owner
        if name == "id":
            unit = (st == np.arange(len(x))[:, None]).astype(float)
            assert np.abs(r["W"] - unit).max() < 1e-9
        else:
            a = OPS[name] - oracle.OP_DX
            f = 3.0 * x[:, a] - 2.0 * x[:, (a + 1) % 3] + 0.5
            got = (r["W"] * f[st]).sum(1)
            assert np.abs(got - 3.0).max() < 1e-8
