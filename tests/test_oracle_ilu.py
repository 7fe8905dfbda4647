"""Pins of the oracle's ILU(0) of the implicit step matrix (Sec. 5; Secs.
7.1 and 7.2 precondition GMRES and BiCGSTAB with it):
  - its defining property: (L U)_ij = A_ij on A's sparsity pattern;
  - where the pattern takes no fill (a banded matrix), it is the plain LU
    factorization without pivoting, L U = A everywhere;
  - a hand-factored 3 x 3 tridiagonal case;
  - with it, restarted GMRES solves the Neumann heat step of a
    boundary-refined disk at dt = 1e-3 in 10-15 iterations to 1e-12, as
    Sec. 7.1 reports (SciPy's GMRES, used here only as a reference solver).
"""
import numpy as np
import pytest
import scipy.sparse as sps
import scipy.sparse.linalg as spl

import nodesets
import oracle


def _lu_product(row_ptr, col, lu):
    N = len(row_ptr) - 1
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    low = col < rows
    L = sps.csr_matrix((np.where(low, lu, 0.0), col, row_ptr), shape=(N, N))
    U = sps.csr_matrix((np.where(low, 0.0, lu), col, row_ptr), shape=(N, N))
    return (L + sps.identity(N)) @ U, rows


@pytest.fixture(scope="module")
def neumann_disk():
    D = nodesets.disk(3000, 120, 1, refine=True)
    x, bnd = D["x"], D["boundary"]
    R = oracle.build_dm(x, 31, 5, 4, 0.5, eligible=D["eligible"],
                        boundary=bnd, normals=D["normals"])
    kind = np.ones(len(x), np.uint8)
    kind[bnd] = 2
    return R, kind


def test_lu_matches_a_on_the_pattern(neumann_disk):
    R, kind = neumann_disk
    rp, col = R["row_ptr"], R["col"]
    a = oracle.step_values(rp, col, R["val"], kind, 1.0, -1e-3)
    lu = oracle.ilu0(rp, col, a)
    P, rows = _lu_product(rp, col, lu)
    got = np.asarray(P.tocsr()[rows, col]).ravel()
    assert np.abs(got - a).max() <= 1e-13 * np.abs(a).max()
    # and it is not the exact factorization: fill outside the pattern
    assert np.abs((P - sps.csr_matrix((a, col, rp), shape=P.shape))).max() \
        > 1e-6 * np.abs(a).max()


def test_banded_matrix_is_plain_lu():
    rng = np.random.default_rng(3)
    N, bw = 60, 2
    dense = np.zeros((N, N))
    for i in range(N):
        for j in range(max(0, i - bw), min(N, i + bw + 1)):
            dense[i, j] = rng.uniform(-1, 1)
        dense[i, i] = 6.0 + rng.uniform(0, 1)
    A = sps.csr_matrix(dense)
    A.sort_indices()
    lu = oracle.ilu0(A.indptr, A.indices, A.data)
    P, _ = _lu_product(A.indptr, A.indices, lu)
    assert np.abs(P.toarray() - dense).max() <= 1e-14 * np.abs(dense).max()


def test_hand_factored_tridiagonal():
    # [[4,1,0],[2,5,1],[0,3,6]]: l21 = 1/2, u22 = 9/2, l32 = 2/3, u33 = 16/3
    rp = np.array([0, 2, 5, 7])
    col = np.array([0, 1, 0, 1, 2, 1, 2])
    a = np.array([4.0, 1.0, 2.0, 5.0, 1.0, 3.0, 6.0])
    lu = oracle.ilu0(rp, col, a)
    want = np.array([4.0, 1.0, 0.5, 4.5, 1.0, 2.0 / 3.0, 16.0 / 3.0])
    assert np.allclose(lu, want, rtol=1e-15, atol=0)


def test_gmres_with_ilu0_needs_few_iterations(neumann_disk):
    R, kind = neumann_disk
    rp, col = R["row_ptr"], R["col"]
    N = len(rp) - 1
    a = oracle.step_values(rp, col, R["val"], kind, 1.0, -1e-3)
    lu = oracle.ilu0(rp, col, a)
    rows = np.repeat(np.arange(N), np.diff(rp))
    low = col < rows
    L = (sps.csr_matrix((np.where(low, lu, 0.0), col, rp), shape=(N, N))
         + sps.identity(N)).tocsr()
    U = sps.csr_matrix((np.where(low, 0.0, lu), col, rp), shape=(N, N))
    M = spl.LinearOperator((N, N), matvec=lambda v: spl.spsolve_triangular(
        U, spl.spsolve_triangular(L, v, lower=True), lower=False))
    A = sps.csr_matrix((a, col, rp), shape=(N, N))
    b = np.random.default_rng(0).random(N)
    res = []
    x, info = spl.gmres(A, b, M=M, rtol=1e-12, restart=50,
                        callback=res.append, callback_type="pr_norm")
    assert info == 0
    assert 10 <= len(res) <= 15, len(res)
    assert np.linalg.norm(A @ x - b) <= 1e-11 * np.linalg.norm(b)


def _rand_nonsym(n, seed):
    rng = np.random.default_rng(seed)
    A = sps.random(n, n, density=0.05, random_state=seed, format="csr")
    A = A + sps.diags(4.0 + rng.random(n)) - 0.5 * A.T
    A = A.tocsr()
    A.sort_indices()
    return A


def test_bicgstab_solves_a_nonsymmetric_system():
    """Unpreconditioned BiCGSTAB reaches the requested residual and the
    direct solution of a diagonally dominant nonsymmetric system."""
    A = _rand_nonsym(300, 3)
    b = np.random.default_rng(4).random(300)
    x, it, res = oracle.bicgstab(A, b, np.zeros(300), 1e-12, 200)
    ref = spl.spsolve(A.tocsc(), b)
    assert res <= 1e-12
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1e-12
    assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max()
    assert 1 < it < 100


def test_bicgstab_exact_preconditioner_one_half_step():
    """With a preconditioner equal to A (ILU(0) of a tridiagonal matrix is
    its exact LU factorization) the first half step solves the system."""
    n = 200
    rng = np.random.default_rng(7)
    A = sps.diags([rng.random(n - 1) - 0.5, 3.0 + rng.random(n),
                   rng.random(n - 1) - 0.5], [-1, 0, 1], format="csr")
    A.sort_indices()
    lu = oracle.ilu0(A.indptr, A.indices, A.data)
    b = rng.random(n)
    x, it, res = oracle.bicgstab(A, b, np.zeros(n), 1e-12, 50,
                                 ilu=(A.indptr, A.indices, lu))
    assert it == 1 and res <= 1e-12
    assert np.abs(x - spl.spsolve(A.tocsc(), b)).max() <= 1e-12


def test_bicgstab_ilu0_matches_plain_solution(neumann_disk):
    """ILU(0)-preconditioned BiCGSTAB on the Neumann heat step converges to
    the direct solution in far fewer iterations than without it."""
    R, kind = neumann_disk
    rp, col = R["row_ptr"], R["col"]
    A = oracle.implicit_system(rp, col, R["val"], kind, 1.0, -1e-3)
    lu = oracle.ilu0(rp, col, oracle.step_values(rp, col, R["val"], kind, 1.0,
                                                 -1e-3))
    b = np.random.default_rng(5).random(len(rp) - 1)
    x, it, res = oracle.bicgstab(A, b, np.zeros_like(b), 1e-12, 500,
                                 ilu=(rp, col, lu))
    _, it0, _ = oracle.bicgstab(A, b, np.zeros_like(b), 1e-12, 500)
    ref = oracle.solve_implicit(rp, col, R["val"], b, kind, 1.0, -1e-3)
    assert res <= 1e-12
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()
    assert it * 4 < it0
