"""ctypes front end of the C oracle (test infrastructure only).

All arrays are numpy, C-contiguous.  Functions raise ``OracleError`` with the
C status code on failure.  Citations refer to sections and equations of the
paper; the arithmetic itself lives in ``orbf_oracle.c``.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborbf_oracle.so")

OK, EINVAL, EDUPLICATE, ESINGULAR = 0, 1, 2, 3
OP_LAPLACIAN, OP_NEUMANN, OP_DX, OP_DY, OP_DZ, OP_IDENTITY = 0, 1, 2, 3, 4, 5
_NAMES = {EINVAL: "EINVAL", EDUPLICATE: "EDUPLICATE", ESINGULAR: "ESINGULAR"}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what}: {_NAMES.get(code, code)}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_D = ctypes.c_double


def _declare(L):
    L.orc_num_monomials.argtypes = [_I, _I]
    L.orc_num_monomials.restype = _I
    L.orc_degree_rule.argtypes = [_I, _I, _P, _P]
    L.orc_degree_rule.restype = None
    for f in (L.orc_knn_brute, L.orc_knn_grid):
        f.argtypes = [_P, _I64, _I, _I, _P, _P]
        f.restype = _I
    L.orc_knn_one.argtypes = [_P, _I64, _I, _I, _I64, _P, _P]
    L.orc_knn_one.restype = _I
    L.orc_cover.argtypes = [_P, _I64, _I, _I, _P, _P, _D, _P, _P, _P, _P]
    L.orc_cover.restype = _I
    L.orc_stencil_weights.argtypes = [_I, _I, _I, _I, _I, _P, _I, _P, _P, _P]
    L.orc_stencil_weights.restype = _I
    L.orc_overlapped_rows.argtypes = [_P, _I64, _I, _I, _I, _I, _P, _P, _D,
                                      _D, _P, _P, _P, _P, _P, _P, _P, _I]
    L.orc_overlapped_rows.restype = _I
    L.orc_overlapped_rows_mode.argtypes = [_P, _I64, _I, _I, _I, _I, _P, _P,
                                           _D, _D, _I, _P, _P, _P, _P, _P, _P,
                                           _P, _I]
    L.orc_overlapped_rows_mode.restype = _I
    L.orc_overlapped_rows_op.argtypes = [_P, _I64, _I, _I, _I, _I, _I, _P,
                                         _P, _D, _P, _P, _P, _P, _P, _P, _I]
    L.orc_overlapped_rows_op.restype = _I
    L.orc_center_rows.argtypes = [_P, _I64, _I, _I, _I, _I, _I, _P, _I64, _P,
                                  _P, _P, _P, _I]
    L.orc_center_rows.restype = _I
    L.orc_csr.argtypes = [_I64, _I, _P, _P, _P, _P, _P, _P]
    L.orc_csr.restype = _I


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _check(code, what):
    if code != OK:
        raise OracleError(code, what)


def num_monomials(d, l):
    """M = C(l+d, d), the size of the polynomial space (Sec. 2)."""
    return lib().orc_num_monomials(d, l)


def degree_rule(d, n):
    """Degree s and monomial count M for stencil size n (Sec. 2)."""
    s = ctypes.c_int()
    M = ctypes.c_int()
    lib().orc_degree_rule(d, n, ctypes.byref(s), ctypes.byref(M))
    return s.value, M.value


def knn(x, n, method="auto"):
    """Stencils I^k (n nearest nodes, self first, ties by index) and rho_k^2.

    Sec. 2 / Sec. 4.1.  ``method``: 'brute', 'grid' or 'auto' (brute force up
    to 20000 nodes)."""
    x = _f64(x)
    N, d = x.shape
    out = np.empty((N, n), np.int32)
    rho2 = np.empty(N, np.float64)
    if method == "auto":
        method = "brute" if N <= 20000 else "grid"
    f = lib().orc_knn_brute if method == "brute" else lib().orc_knn_grid
    _check(f(_ptr(x), N, d, n, _ptr(out), _ptr(rho2)), "knn")
    return out, rho2


def knn_one(x, n, q):
    """Brute-force stencil of a single node q (sampled checks)."""
    x = _f64(x)
    N, d = x.shape
    out = np.empty(n, np.int32)
    r = ctypes.c_double()
    _check(lib().orc_knn_one(_ptr(x), N, d, n, int(q), _ptr(out),
                             ctypes.byref(r)), "knn_one")
    return out, r.value


def cover(x, knn_idx, rho2, delta, eligible=None):
    """Greedy overlapped covering without Lebesgue rejection (Sec. 4.1).

    Returns (owner[N], centers[N_delta])."""
    x = _f64(x)
    N, d = x.shape
    n = knn_idx.shape[1]
    knn_idx = _i32(knn_idx)
    rho2 = _f64(rho2)
    el = None if eligible is None else np.ascontiguousarray(eligible, np.uint8)
    owner = np.empty(N, np.int32)
    centers = np.empty(N, np.int32)
    nc = ctypes.c_int64()
    _check(lib().orc_cover(_ptr(x), N, d, n, _ptr(knn_idx), _ptr(rho2),
                           float(delta), _ptr(el), _ptr(owner), _ptr(centers),
                           ctypes.byref(nc)), "cover")
    return owner, centers[: nc.value].copy()


def stencil_weights(P, E, m, l, op=OP_LAPLACIAN, normals=None):
    """Weights of one stencil P (P[0] the center) at points E.

    Eqs. rbffd_linsys / orbffd_eq / orbffd_rhs (Sec. 4.1); returns
    W[ne, n], W[e, j] = weight of node j for point e, physical units."""
    P = _f64(P)
    E = _f64(np.atleast_2d(E))
    n, d = P.shape
    ne = E.shape[0]
    nr = None if normals is None else _f64(np.atleast_2d(normals))
    W = np.empty((ne, n), np.float64)
    _check(lib().orc_stencil_weights(d, m, l, op, n, _ptr(P), ne, _ptr(E),
                                     _ptr(nr), _ptr(W)), "stencil_weights")
    return W


def overlapped_rows(x, knn_idx, rho2, m, l, delta, tau=np.inf, eligible=None,
                    nthreads=0, prefix=False):
    """Laplacian DM rows with the greedy covering and, for finite tau, the
    L-Lebesgue acceptance test (Sec. 4.1, Sec. 4.2.1), node-wise or, with
    ``prefix``, as the radial prefix of each retention ball (the ball shrunk
    to just inside its first node that fails the test).

    Returns dict(owner, centers, W[N,n] (rows aligned with knn[owner]),
    lam[N], min_margin)."""
    x = _f64(x)
    N, d = x.shape
    n = knn_idx.shape[1]
    knn_idx = _i32(knn_idx)
    rho2 = _f64(rho2)
    el = None if eligible is None else np.ascontiguousarray(eligible, np.uint8)
    owner = np.empty(N, np.int32)
    centers = np.empty(N, np.int32)
    nc = ctypes.c_int64()
    W = np.zeros((N, n), np.float64)
    lam = np.zeros(N, np.float64)
    mm = ctypes.c_double()
    _check(lib().orc_overlapped_rows_mode(
        _ptr(x), N, d, n, m, l, _ptr(knn_idx), _ptr(rho2), float(delta),
        float(tau), int(bool(prefix)), _ptr(el), _ptr(owner), _ptr(centers),
        ctypes.byref(nc), _ptr(W), _ptr(lam), ctypes.byref(mm),
        int(nthreads)), "overlapped_rows")
    return dict(owner=owner, centers=centers[: nc.value].copy(), W=W, lam=lam,
                min_margin=mm.value)


def overlapped_rows_op(x, knn_idx, rho2, m, l, delta, op, eligible=None,
                       nthreads=0):
    """DM rows of operator op (LAPLACIAN, DX, DY, DZ or IDENTITY) on the
    greedy covering without the Lebesgue test (Sec. 4.1: the right-hand
    sides are L applied to the basis; weights divided by rho^theta).

    Returns dict(owner, centers, W[N,n], lam[N])."""
    x = _f64(x)
    N, d = x.shape
    n = knn_idx.shape[1]
    knn_idx = _i32(knn_idx)
    rho2 = _f64(rho2)
    el = None if eligible is None else np.ascontiguousarray(eligible, np.uint8)
    owner = np.empty(N, np.int32)
    centers = np.empty(N, np.int32)
    nc = ctypes.c_int64()
    W = np.zeros((N, n), np.float64)
    lam = np.zeros(N, np.float64)
    _check(lib().orc_overlapped_rows_op(_ptr(x), N, d, n, m, l, int(op),
                                        _ptr(knn_idx), _ptr(rho2),
                                        float(delta), _ptr(el), _ptr(owner),
                                        _ptr(centers), ctypes.byref(nc),
                                        _ptr(W), _ptr(lam), int(nthreads)),
           "overlapped_rows_op")
    return dict(owner=owner, centers=centers[: nc.value].copy(), W=W, lam=lam)


def center_rows(x, knn_idx, m, l, rows, op=OP_LAPLACIAN, normals=None,
                owner=None, W=None, nthreads=0):
    """delta = 1 rows of the listed nodes, each on its own stencil (boundary
    pass of Sec. 5).  Updates (or creates) owner and W in place."""
    x = _f64(x)
    N, d = x.shape
    n = knn_idx.shape[1]
    knn_idx = _i32(knn_idx)
    rows = _i32(rows)
    if owner is None:
        owner = np.full(N, -1, np.int32)
    if W is None:
        W = np.zeros((N, n), np.float64)
    nr = None if normals is None else _f64(normals)
    _check(lib().orc_center_rows(_ptr(x), N, d, n, m, l, op, _ptr(knn_idx),
                                 len(rows), _ptr(rows), _ptr(nr), _ptr(owner),
                                 _ptr(W), int(nthreads)), "center_rows")
    return owner, W


def csr(knn_idx, owner, W):
    """CSR of the DM, columns ascending in each row (Sec. 4.1 scatter)."""
    N, n = knn_idx.shape
    knn_idx = _i32(knn_idx)
    owner = _i32(owner)
    W = _f64(W)
    row_ptr = np.empty(N + 1, np.int64)
    col = np.empty(N * n, np.int32)
    val = np.empty(N * n, np.float64)
    _check(lib().orc_csr(N, n, _ptr(knn_idx), _ptr(owner), _ptr(W),
                         _ptr(row_ptr), _ptr(col), _ptr(val)), "csr")
    nnz = int(row_ptr[-1])
    return row_ptr, col[:nnz].copy(), val[:nnz].copy()


def gershgorin(row_ptr, col, val):
    """Gershgorin disks of the DM rows (Sec. 4.2.1): center L_kk and radius
    g_k = sum_{j != k} |L_kj| per row (0 and 0 for an empty row), and the
    summary (max_k L_kk + g_k, min_k L_kk - g_k, number of rows whose disk
    reaches Re > 0).  Plain definition, one row at a time."""
    N = len(row_ptr) - 1
    diag = np.zeros(N)
    radius = np.zeros(N)
    for k in range(N):
        for t in range(int(row_ptr[k]), int(row_ptr[k + 1])):
            if col[t] == k:
                diag[k] = val[t]
            else:
                radius[k] += abs(val[t])
    right = diag + radius
    left = diag - radius
    return diag, radius, (float(right.max()), float(left.min()),
                          int((right > 0).sum()))


def implicit_system(row_ptr, col, val, row_kind, alpha, beta):
    """The matrix of one implicit time step with a DM (Sec. 5): interior
    rows (row_kind 1) are alpha e_k + beta L_k, so backward Euler's block
    I - nu dt L_ii, -nu dt L_ib for alpha = 1, beta = -nu dt; Dirichlet rows
    (row_kind 0) are e_k; any other row_kind keeps the DM row L_k (a
    boundary operator such as a normal derivative).  ``row_kind`` None
    means every row is interior.  Returns a scipy CSR matrix."""
    import scipy.sparse as sps
    N = len(row_ptr) - 1
    L = sps.csr_matrix((val, col, row_ptr), shape=(N, N))
    kind = np.ones(N, np.uint8) if row_kind is None else np.asarray(row_kind)
    interior = (kind == 1).astype(float)
    dirichlet = (kind == 0).astype(float)
    other = 1.0 - interior - dirichlet
    eye = sps.identity(N, format="csr")
    A = (sps.diags(interior) @ (alpha * eye + beta * L)
         + sps.diags(dirichlet) @ eye + sps.diags(other) @ L)
    return A.tocsr()


def step_values(row_ptr, col, val, row_kind, alpha, beta):
    """Values of the implicit step matrix (``implicit_system``) on the DM's
    own sparsity pattern, aligned with ``col`` (zeros kept)."""
    A = implicit_system(row_ptr, col, val, row_kind, alpha, beta)
    N = len(row_ptr) - 1
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    return np.asarray(A[rows, col]).ravel()


def ilu0(row_ptr, col, a):
    """ILU(0) of the CSR matrix (row_ptr, col, a), columns ascending in each
    row: Gaussian elimination with no fill outside the sparsity pattern.
    For each row i and each k < i in row i, in ascending order,
    a_ik = a_ik / a_kk, then a_ij = a_ij - a_ik a_kj for every j > k that
    both rows hold.  Returns the values of L (unit lower, strictly below the
    diagonal) and U (on and above) aligned with ``col``."""
    lu = np.array(a, dtype=float)
    N = len(row_ptr) - 1
    pos = []   # per row: column -> position
    diag = np.empty(N, np.int64)
    for i in range(N):
        s0, s1 = int(row_ptr[i]), int(row_ptr[i + 1])
        pos.append({int(c): t for t, c in enumerate(col[s0:s1], start=s0)})
        if i not in pos[i]:
            raise ValueError(f"row {i} has no diagonal entry")
        diag[i] = pos[i][i]
    for i in range(N):
        s0, s1 = int(row_ptr[i]), int(row_ptr[i + 1])
        for t in range(s0, s1):
            k = int(col[t])
            if k >= i:
                break
            lu[t] = lu[t] / lu[diag[k]]
            for u in range(int(diag[k]) + 1, int(row_ptr[k + 1])):
                j = int(col[u])
                q = pos[i].get(j)
                if q is not None:
                    lu[q] = lu[q] - lu[t] * lu[u]
    return lu


def bicgstab(A, b, x0, tol, max_iter, ilu=None):
    """BiCGSTAB (van der Vorst, 1992; the paper's 3D solver, Sec. 7.2),
    right-preconditioned with ILU(0) factors ``ilu`` = (row_ptr, col, lu),
    as ``ilu0`` returns them for that pattern, or unpreconditioned (None).
    Stops when ||r|| / ||b|| <= tol, checked after each half step (on s)
    and each full step.  A is any scipy sparse matrix.
    Returns (x, iterations, relative residual)."""
    import scipy.sparse as sps
    import scipy.sparse.linalg as spl
    N = A.shape[0]
    if ilu is None:
        def M(v):
            return v
    else:
        F = sps.csr_matrix((ilu[2], ilu[1], ilu[0]), shape=A.shape)
        L = sps.tril(F, -1, format="csr") + sps.identity(N, format="csr")
        U = sps.triu(F, 0, format="csr")

        def M(v):
            y = spl.spsolve_triangular(L, v, lower=True, unit_diagonal=True)
            return spl.spsolve_triangular(U, y, lower=False)
    x = np.array(x0, dtype=float)
    b = np.asarray(b, dtype=float)
    nb = np.linalg.norm(b) or 1.0
    r = b - A @ x
    rh = r.copy()
    res = np.linalg.norm(r) / nb
    rho = al = om = 1.0
    v = np.zeros(N)
    p = np.zeros(N)
    it = 0
    while res > tol and it < max_iter:
        rho_new = rh @ r
        if rho_new == 0.0:
            break
        it += 1
        p = r + (rho_new / rho) * (al / om) * (p - om * v)
        ph = M(p)
        v = A @ ph
        al = rho_new / (rh @ v)
        s = r - al * v
        if np.linalg.norm(s) / nb <= tol:
            x = x + al * ph
            res = np.linalg.norm(s) / nb
            break
        sh = M(s)
        t = A @ sh
        om = (t @ s) / (t @ t)
        x = x + al * ph + om * sh
        r = s - om * t
        rho = rho_new
        res = np.linalg.norm(r) / nb
    return x, it, res


def solve_implicit(row_ptr, col, val, b, row_kind=None, alpha=1.0,
                   beta=-1.0):
    """x = A^{-1} b for the matrix of ``implicit_system`` (Sec. 5), by a
    direct sparse LU solve (SuperLU)."""
    import scipy.sparse.linalg as spl
    A = implicit_system(row_ptr, col, val, row_kind, alpha, beta)
    return spl.spsolve(A.tocsc(), np.asarray(b, dtype=float))


def bdf_coefficients(k):
    """Backward differentiation formula of order k (Sec. 5 steps with BDF4
    and starts with BDF1-3): u^{n+1} - sum_i a_i u^{n-i} = b dt u'(t^{n+1}).
    From its definition: exact for every polynomial of degree <= k in t on
    equal steps.  With s = (t - t^{n+1}) / dt the nodes are s = 0, -1, ...,
    -k and the conditions on s^j, j = 0..k, form a (k+1) x (k+1) linear
    system in (a_0..a_{k-1}, b).  Returns (a, b), a of length k."""
    # sum_i a_i (-(i+1))^j + b * [j == 1] = 0^j   (0^0 = 1)
    A = np.zeros((k + 1, k + 1))
    rhs = np.zeros(k + 1)
    for j in range(k + 1):
        for i in range(k):
            A[j, i] = float(-(i + 1)) ** j
        A[j, k] = 1.0 if j == 1 else 0.0
        rhs[j] = 1.0 if j == 0 else 0.0
    sol = np.linalg.solve(A, rhs)
    return sol[:k], float(sol[k])


def bdf_rhs(levels, dt, f=None, row_kind=None, bvals=None):
    """Right-hand side of one BDF step of u_t = nu L u + f (Sec. 5):
    sum_i a_i u^{n-i} + b dt f on interior rows (row_kind 1, or all rows if
    row_kind is None), the boundary value (or 0) elsewhere; ``levels`` =
    [u^n, u^{n-1}, ...], newest first, its length the order."""
    a, b = bdf_coefficients(len(levels))
    out = np.zeros_like(np.asarray(levels[0], dtype=float))
    for ai, u in zip(a, levels):
        out = out + ai * np.asarray(u, dtype=float)
    if f is not None:
        out = out + b * dt * np.asarray(f, dtype=float)
    if row_kind is not None:
        other = np.asarray(row_kind) != 1
        out[other] = 0.0 if bvals is None else np.asarray(bvals)[other]
    return out


def bdf_step(row_ptr, col, val, levels, dt, nu=1.0, f=None, row_kind=None,
             bvals=None):
    """u^{n+1} of one BDF step (Sec. 5): the implicit system with alpha = 1,
    beta = -b nu dt and the right-hand side of ``bdf_rhs``."""
    _, b = bdf_coefficients(len(levels))
    rhs = bdf_rhs(levels, dt, f, row_kind, bvals)
    return solve_implicit(row_ptr, col, val, rhs, row_kind, 1.0, -b * nu * dt)


def build_dm(x, n, m, l, delta, tau=np.inf, eligible=None, boundary=None,
             normals=None, nthreads=0, knn_method="auto", op=OP_LAPLACIAN,
             prefix=False):
    """Whole oracle pipeline: stencils, covering (+Lebesgue), interior rows
    of operator ``op`` (the Lebesgue test only with the Laplacian), optional
    normal-derivative rows at ``boundary`` nodes, CSR.  Returns a dict with
    every intermediate."""
    idx, rho2 = knn(x, n, knn_method)
    if op == OP_LAPLACIAN:
        r = overlapped_rows(x, idx, rho2, m, l, delta, tau, eligible,
                            nthreads, prefix)
    else:
        if not np.isinf(tau):
            raise ValueError("the Lebesgue test is defined for the Laplacian")
        r = overlapped_rows_op(x, idx, rho2, m, l, delta, op, eligible,
                               nthreads)
    owner, W = r["owner"], r["W"]
    if boundary is not None and len(boundary):
        center_rows(x, idx, m, l, boundary, OP_NEUMANN, normals, owner, W,
                    nthreads)
    row_ptr, col, val = csr(idx, owner, W)
    r.update(knn=idx, rho2=rho2, row_ptr=row_ptr, col=col, val=val)
    return r
