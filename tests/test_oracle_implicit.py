"""Pins of the oracle's implicit time step (Sec. 5: backward Euler with the
DM, interior rows I - nu dt L, boundary rows imposing the condition).

Closed forms that fix it independently of its code: the second-difference
operator on a uniform 1D grid has the discrete sines (Dirichlet ends) and
shifted cosines (a one-sided Neumann row at the left end) as eigenvectors,
with eigenvalues -(4/h^2) sin^2(w/2), so one step of alpha x - beta L x = u
from an eigenvector u divides it by alpha + beta * eigenvalue.
"""
import numpy as np
import pytest

import oracle


def _second_difference(N, h, left_row, right_row):
    """CSR of N + 2 nodes: rows 1..N hold (u_{k-1} - 2 u_k + u_{k+1}) / h^2,
    rows 0 and N+1 the given (col, val) lists."""
    rows = [left_row]
    for k in range(1, N + 1):
        rows.append(([k - 1, k, k + 1], [1 / h**2, -2 / h**2, 1 / h**2]))
    rows.append(right_row)
    row_ptr = np.zeros(N + 3, np.int64)
    col, val = [], []
    for i, (c, v) in enumerate(rows):
        col += c
        val += v
        row_ptr[i + 1] = len(col)
    return row_ptr, np.array(col, np.int32), np.array(val)


@pytest.mark.parametrize("alpha,beta", [(1.0, -1e-3), (2.0, -0.5e-4),
                                        (1.0, 0.0)])
@pytest.mark.parametrize("j", [1, 3, 17])
def test_dirichlet_sine_closed_form(alpha, beta, j):
    N = 63
    h = 1.0 / (N + 1)
    # boundary rows hold values that a Dirichlet row must ignore
    rp, col, val = _second_difference(N, h, ([0, 1], [5.0, 7.0]),
                                      ([N, N + 1], [-3.0, 2.0]))
    kind = np.ones(N + 2, np.uint8)
    kind[[0, N + 1]] = 0
    xs = np.arange(N + 2) * h
    u = np.sin(j * np.pi * xs)
    u[[0, N + 1]] = 0.0
    lam = -(4 / h**2) * np.sin(j * np.pi * h / 2) ** 2
    want = u / (alpha + beta * lam)
    got = oracle.solve_implicit(rp, col, val, u, kind, alpha, beta)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("j", [1, 2, 9])
def test_neumann_cosine_closed_form(j):
    """Left end: the boundary-operator row (x_1 - x_0) / h = 0 (row_kind 2);
    right end Dirichlet.  Eigenvectors cos(w (k - 1/2)) with
    w = (2j - 1) pi / (2N + 1)."""
    N = 40
    h = 1.0 / N
    dt = 2e-3
    rp, col, val = _second_difference(N, h, ([0, 1], [-1 / h, 1 / h]),
                                      ([N + 1], [1.0]))
    kind = np.ones(N + 2, np.uint8)
    kind[0] = 2
    kind[N + 1] = 0
    w = (2 * j - 1) * np.pi / (2 * N + 1)
    k = np.arange(N + 2)
    u = np.cos(w * (k - 0.5))
    lam = -(4 / h**2) * np.sin(w / 2) ** 2
    want = u / (1 + dt * (-lam))
    b = u.copy()
    b[0] = 0.0
    b[N + 1] = 0.0
    want[N + 1] = 0.0
    assert abs(u[N + 1]) < 1e-12  # the eigenvector vanishes there
    got = oracle.solve_implicit(rp, col, val, b, kind, 1.0, -dt)
    assert np.abs(got - want).max() <= 1e-12
    assert got[0] == pytest.approx(got[1], abs=1e-14)


def test_all_interior_default():
    """row_kind None: every row is alpha e_k + beta L_k."""
    N = 30
    h = 1.0 / (N + 1)
    rp, col, val = _second_difference(N, h, ([0, 1], [-2 / h**2, 1 / h**2]),
                                      ([N, N + 1], [1 / h**2, -2 / h**2]))
    # with these end rows L is the Dirichlet second difference on N + 2
    # unknowns (spacing h still in the values); its sines are those of the
    # N + 2 grid
    M = N + 2
    hh = 1.0 / (M + 1)
    xs = (np.arange(M) + 1) * hh
    u = np.sin(3 * np.pi * xs)
    lam = -(4 / h**2) * np.sin(3 * np.pi * hh / 2) ** 2
    got = oracle.solve_implicit(rp, col, val, u, None, 1.5, -1e-4)
    want = u / (1.5 - 1e-4 * lam)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


# BDF time stepping (Sec. 5: BDF4, started with BDF1-3).

def test_bdf4_coefficients_match_the_paper():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "bdf4_coefficients.json")))
    a, b = oracle.bdf_coefficients(g["order"])
    want = np.array(g["a_num"], dtype=float) / g["den"]
    assert np.abs(a - want).max() <= 1e-14
    assert abs(b - g["b_num"] / g["den"]) <= 1e-14


def test_bdf1_is_backward_euler_and_bdf2_textbook():
    a, b = oracle.bdf_coefficients(1)
    assert np.allclose(a, [1.0], rtol=0, atol=1e-15) and abs(b - 1.0) < 1e-15
    a, b = oracle.bdf_coefficients(2)
    assert np.allclose(a, [4 / 3, -1 / 3], rtol=0, atol=1e-15)
    assert abs(b - 2 / 3) < 1e-15


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_bdf_order_of_accuracy_on_scalar_ode(k):
    """u' = lam u through bdf_step on a one-node 'DM' L = [lam], from exact
    history: the error at t = 1 falls like dt^k."""
    lam = -1.3
    rp, col = np.array([0, 1], np.int64), np.array([0], np.int32)
    val = np.array([lam])
    errs = []
    for dt in (0.02, 0.01):
        steps = int(round(1.0 / dt))
        hist = [np.array([np.exp(lam * (-i) * dt)]) for i in range(k)]
        # hist[i] = u(t = -i dt): newest first at t = 0
        for s in range(steps):
            un = oracle.bdf_step(rp, col, val, hist, dt)
            hist = [un] + hist[:k - 1]
        errs.append(abs(hist[0][0] - np.exp(lam)))
    order = np.log2(errs[0] / errs[1])
    assert abs(order - k) < 0.25, (k, errs, order)


def test_bdf_rhs_boundary_rows():
    u0 = np.array([1.0, 2.0, 3.0])
    u1 = np.array([0.5, 0.5, 0.5])
    kind = np.array([1, 0, 2], np.uint8)
    bv = np.array([9.0, 7.0, -4.0])
    out = oracle.bdf_rhs([u0, u1], 0.1, f=np.ones(3), row_kind=kind, bvals=bv)
    assert out[0] == pytest.approx(4 / 3 * 1.0 - 1 / 3 * 0.5 + 2 / 3 * 0.1)
    assert out[1] == 7.0 and out[2] == -4.0
    out = oracle.bdf_rhs([u0, u1], 0.1, row_kind=kind)
    assert out[1] == 0.0 and out[2] == 0.0
