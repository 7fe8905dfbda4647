"""Pins of the oracle's L-Lebesgue rejection (Sec. 4.2.1) and CSR scatter
(Sec. 4.1).

  - Lambda_L(x_e) is the 1-norm of the row's weights (Sec. 4.2.1), so it can
    be recomputed from the CSR alone;
  - the Gershgorin radius of row k is Lambda_L(x_k) - |L_kk| (Sec. 4.2.1);
  - the center and the reference node are always kept, every eligible node
    still gets exactly one row, a kept node passes the test in the stencil
    that owns it, and a stricter threshold never needs fewer stencils;
  - CSR rows hold the owner's stencil indices, ascending, and L f equals the
    per-stencil dot products.
"""
import numpy as np
import pytest

import nodesets
import oracle


@pytest.fixture(scope="module")
def disk_small():
    D = nodesets.disk(4000, 150, 1)
    idx, rho2 = oracle.knn(D["x"], 31)
    return D, idx, rho2


@pytest.mark.parametrize("tau", [1.0, 2.0, 5.0, np.inf])
def test_lebesgue_rows(disk_small, tau):
    D, idx, rho2 = disk_small
    x, el = D["x"], D["eligible"]
    r = oracle.overlapped_rows(x, idx, rho2, 5, 4, 0.3, tau, el)
    owner, W, lam = r["owner"], r["W"], r["lam"]
    interior = np.nonzero(el)[0]
    assert (owner[interior] >= 0).all()
    # Lambda is the 1-norm of the row (Sec. 4.2.1)
    assert np.allclose(lam[interior], np.abs(W[interior]).sum(1), rtol=1e-13)
    # every kept non-center passes the test in its owner's stencil
    for j in interior[::5]:
        c = owner[j]
        if c == j or np.isinf(tau):
            continue
        st = idx[c]
        P = x[st]
        rel = P - P[0]
        cen = rel.sum(0) / len(st)
        ref = int(np.argmin(((rel - cen) ** 2).sum(1)))
        Wc = oracle.stencil_weights(P, P[[ref, list(st).index(j)]], 5, 4)
        assert np.abs(Wc[1]).sum() <= tau * np.abs(Wc[0]).sum() * (1 + 1e-12)


def test_stricter_threshold_needs_more_stencils(disk_small):
    D, idx, rho2 = disk_small
    counts = [len(oracle.overlapped_rows(D["x"], idx, rho2, 5, 4, 0.3, t,
                                         D["eligible"])["centers"])
              for t in (1.0, 1.5, 5.0, np.inf)]
    assert counts[0] >= counts[1] >= counts[2] >= counts[3]
    assert counts[0] > counts[3]  # tau = 1 (the paper's test) rejects some


def test_gershgorin_identity_and_csr(disk_small):
    D, idx, rho2 = disk_small
    x = D["x"]
    R = oracle.build_dm(x, 31, 5, 4, 0.5, tau=5.0, eligible=D["eligible"],
                        boundary=D["boundary"], normals=D["normals"])
    rp, col, val = R["row_ptr"], R["col"], R["val"]
    N, n = len(x), 31
    assert np.array_equal(rp, np.arange(N + 1) * n)
    c2 = col.reshape(N, n)
    assert (np.diff(c2, axis=1) > 0).all()  # strictly ascending
    owner = R["owner"]
    assert (owner >= 0).all()
    assert np.array_equal(owner[D["boundary"]], D["boundary"])
    for e in range(0, N, 37):
        assert set(c2[e]) == set(idx[owner[e]])
    # Gershgorin radius of row k = Lambda(x_k) - |L_kk|
    v2 = val.reshape(N, n)
    diag = np.array([v2[e][c2[e] == e][0] for e in range(N)])
    radius = np.abs(v2).sum(1) - np.abs(diag)
    off = np.where(c2 == np.arange(N)[:, None], 0.0, np.abs(v2)).sum(1)
    assert np.allclose(radius, off, rtol=1e-12, atol=0)
    inner = D["eligible"] == 1
    assert np.allclose(R["lam"][inner], np.abs(v2[inner]).sum(1), rtol=1e-13)
    # L f equals the per-stencil dot products
    f = np.random.default_rng(2).random(N)
    Lf = np.add.reduceat(val * f[col], rp[:-1])
    ref = np.einsum("ij,ij->i", R["W"], f[idx[owner]])
    assert np.allclose(Lf, ref, rtol=1e-12, atol=1e-9)


def test_gershgorin_disks_contain_the_spectrum():
    """Gershgorin circle theorem on small DMs: every eigenvalue of L lies in
    the union of the row disks, and the disk radius is the row's
    L-Lebesgue value minus |L_kk| (Sec. 4.2.1)."""
    for x, n, l, delta, tau in ((nodesets.square(22, 0), 12, 2, 0.5, np.inf),
                                (nodesets.square(22, 1), 12, 2, 0.2, 1.0)):
        R = oracle.build_dm(x, n, 3, l, delta, tau=tau)
        diag, radius, summ = oracle.gershgorin(R["row_ptr"], R["col"],
                                               R["val"])
        assert np.allclose(radius, R["lam"] - np.abs(diag), rtol=1e-12,
                           atol=1e-12 * R["lam"].max())
        N = len(x)
        L = np.zeros((N, N))
        for k in range(N):
            s0, s1 = R["row_ptr"][k], R["row_ptr"][k + 1]
            L[k, R["col"][s0:s1]] = R["val"][s0:s1]
        ev = np.linalg.eigvals(L)
        slack = 1e-9 * np.abs(L).sum(1).max()
        inside = (np.abs(ev[:, None] - diag[None, :]) <=
                  radius[None, :] + slack).any(1)
        assert inside.all()
        assert summ[0] >= ev.real.max() - slack  # the union bounds Re(lambda)
        assert summ[1] <= ev.real.min() + slack
        assert summ[2] == int((diag + radius > 0).sum())


def test_gershgorin_small_matrix():
    """Hand-checked disks of a 3 x 3 CSR matrix with an empty row."""
    rp = np.array([0, 2, 2, 5])
    col = np.array([0, 2, 0, 1, 2], np.int32)
    val = np.array([-4.0, 1.5, 2.0, -3.0, 0.5])
    d, r, s = oracle.gershgorin(rp, col, val)
    assert np.array_equal(d, [-4.0, 0.0, 0.5])
    assert np.array_equal(r, [1.5, 0.0, 5.0])
    assert s == (5.5, -5.5, 1)


def test_boundary_refinement_shrinks_neumann_lebesgue():
    """Sec. 6: adding a layer of nodes just inside the boundary shrinks the
    Neumann-Lebesgue function at the boundary nodes (Lambda = sum |w| of
    each normal-derivative row), which is why the paper refines its
    Neumann node sets."""
    vals = {}
    for refine in (False, True):
        D = nodesets.disk(5000, 200, 1, refine=refine)
        r = oracle.build_dm(D["x"], 31, 5, 4, 0.5, eligible=D["eligible"],
                            boundary=D["boundary"], normals=D["normals"])
        vals[refine] = np.abs(r["W"][D["boundary"]]).sum(1)
    assert vals[True].mean() < 0.95 * vals[False].mean()
    assert vals[True].max() < vals[False].max()
