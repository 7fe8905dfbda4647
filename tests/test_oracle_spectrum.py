"""Spectra of small oracle-built DMs (Sec. 6.2): on a 1,046-node disk with
n = 30 and delta = 0.2, the unstabilized Laplacian's interior block has
eigenvalues with positive real part, and the local L-Lebesgue stabilization
(eq. calLstab, tau = 1) removes them at the cost of more stencils, as the
paper reports.  Pinned independently by the continuous problem: the
rightmost eigenvalue of the stabilized interior block approximates the
first Dirichlet eigenvalue of the Laplacian on the unit disk, -j_{0,1}^2
(j_{0,1} = 2.404825557695773, the first zero of the Bessel function J_0).
"""
import numpy as np
import pytest

import nodesets
import oracle

J01 = 2.404825557695773


@pytest.mark.parametrize("seed", [1, 2])
def test_stabilization_removes_positive_eigenvalues(seed):
    D = nodesets.disk(946, 100, seed)
    x, el = D["x"], D["eligible"]
    inner = np.nonzero(el)[0]
    out = {}
    for tau in (np.inf, 1.0):
        R = oracle.build_dm(x, 30, 5, 4, 0.2, tau=tau, eligible=el)
        L = np.zeros((len(x), len(x)))
        for k in inner:
            s0, s1 = R["row_ptr"][k], R["row_ptr"][k + 1]
            L[k, R["col"][s0:s1]] = R["val"][s0:s1]
        ev = np.linalg.eigvals(L[np.ix_(inner, inner)])
        s = dict(max_real=ev.real.max(), n_positive_real=(ev.real > 0).sum())
        out[tau] = (len(R["centers"]), s)
    (nc_inf, s_inf), (nc_1, s_1) = out[np.inf], out[1.0]
    assert s_inf["n_positive_real"] > 0 and s_inf["max_real"] > 1.0
    assert s_1["n_positive_real"] == 0
    assert nc_1 > nc_inf  # the price: more stencils, still fewer than N
    assert nc_1 < len(inner)
    lam1 = J01 ** 2
    assert abs(s_1["max_real"] + lam1) / lam1 < 1e-4, s_1

