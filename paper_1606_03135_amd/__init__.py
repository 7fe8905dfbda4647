"""Overlapped RBF-FD differentiation matrices on MI355X (gfx950).

Thin ctypes binding of ``liborbf.so`` (C ABI in ``include/orbf.h``).  Every
numerical step runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch provides device memory and the current HIP stream.

The functions mirror the ABI:

    build_nodes_knn(ctx, xyz, n)                       -> knn, rho2
    select_overlapped_stencils(ctx, xyz, knn, rho2, delta, eligible=None)
                                                       -> centers, n_centers,
                                                          owner, p
    compute_weights(ctx, op, m, l, n, delta, xyz, knn, rho2, ...) -> W
    assemble_csr(ctx, knn, owner, W)                   -> row_ptr, col, val

and ``build_dm`` chains them for a whole node set (Sec. 4.1 of the paper:
stencils, greedy retention-ball covering, per-stencil saddle solves, CSR;
optional normal-derivative rows at listed boundary nodes, Sec. 5).

If the library has not been built the import still succeeds, but every call
raises ``RuntimeError``: there is no CPU fallback.
"""
import ctypes
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborbf.so")

OK, EINVAL, EDUPLICATE, ESINGULAR, ENOMEM, EBUDGET, EHIP, EINTERNAL = range(8)
OP_LAPLACIAN, OP_NEUMANN, OP_DX, OP_DY, OP_DZ, OP_IDENTITY = 0, 1, 2, 3, 4, 5
PREC_FP64, PREC_FP32_IR = 0, 1
STATUS_NAMES = ["OK", "EINVAL", "EDUPLICATE", "ESINGULAR", "ENOMEM",
                "EBUDGET", "EHIP", "EINTERNAL"]

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_D = ctypes.c_double


class OrbfError(RuntimeError):
    def __init__(self, code, msg):
        name = STATUS_NAMES[code] if 0 <= code < len(STATUS_NAMES) else code
        super().__init__(f"orbf {name}: {msg}")
        self.code = code


class WeightsArgs(ctypes.Structure):
    _fields_ = [("xyz", _P), ("N", _I64), ("d", _I), ("knn", _P),
                ("rho2", _P), ("rows", _P), ("n_rows", _I64),
                ("centers", _P), ("n_centers", _P), ("owner", _P),
                ("eligible", _P), ("normals", _P), ("tau", _D), ("prec", _I),
                ("W", _P), ("lebesgue", _P), ("ir_steps", _P),
                ("tau_mode", _I)]


class SetDesc(ctypes.Structure):
    _fields_ = [("xyz", _P), ("N", _I64), ("d", _I), ("n", _I), ("m", _I),
                ("l", _I), ("delta", _D), ("tau", _D), ("prec", _I),
                ("eligible", _P), ("boundary", _P), ("n_boundary", _I64),
                ("normals", _P), ("knn", _P), ("rho2", _P), ("centers", _P),
                ("n_centers", _P), ("owner", _P), ("W", _P),
                ("lebesgue", _P), ("ir_steps", _P), ("row_ptr", _P),
                ("col", _P), ("val", _P)]


class Request(ctypes.Structure):
    _fields_ = [("xyz", _P), ("N", _I64), ("d", _I), ("n", _I), ("m", _I),
                ("l", _I), ("delta", _D), ("tau", _D), ("prec", _I),
                ("t_arrival", _D), ("ready", _P)]


class Result(ctypes.Structure):
    _fields_ = [("status", _I), ("N", _I64), ("n", _I), ("n_centers", _I64),
                ("t_arrival", _D), ("t_admit", _D), ("t_done", _D)]


_lib = None


def lib():
    """The loaded liborbf (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "liborbf.so is not built; run __graft_entry__.build() or "
                "python paper_1606_03135_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        L.orbf_create.argtypes = [_I, _P, ctypes.c_size_t, ctypes.c_void_p]
        L.orbf_create.restype = _I
        L.orbf_destroy.argtypes = [_P]
        L.orbf_destroy.restype = None
        L.orbf_last_error.argtypes = [_P]
        L.orbf_last_error.restype = ctypes.c_char_p
        L.orbf_sync.argtypes = [_P]
        L.orbf_sync.restype = _I
        L.orbf_workspace_size.argtypes = [_I64, _I, _I, _I, _I]
        L.orbf_workspace_size.restype = ctypes.c_size_t
        L.orbf_build_nodes_knn.argtypes = [_P, _P, _I64, _I, _I, _P, _P]
        L.orbf_build_nodes_knn.restype = _I
        L.orbf_select_overlapped_stencils.argtypes = [
            _P, _P, _P, _P, _I64, _I, _I, _D, _P, _P, _P, _P, _P]
        L.orbf_select_overlapped_stencils.restype = _I
        L.orbf_compute_weights.argtypes = [_P, _I, _I, _I, _I, _D,
                                           ctypes.POINTER(WeightsArgs)]
        L.orbf_compute_weights.restype = _I
        L.orbf_assemble_csr.argtypes = [_P, _I64, _I, _P, _P, _P, _P, _P, _P]
        L.orbf_assemble_csr.restype = _I
        L.orbf_assemble_csr_noalloc.argtypes = [_P, _I64, _I, _P, _P, _P, _P,
                                                _P, _P]
        L.orbf_assemble_csr_noalloc.restype = _I
        L.orbf_spmv.argtypes = [_P, _I64, _P, _P, _P, _P, _P]
        L.orbf_spmv.restype = _I
        L.orbf_gershgorin.argtypes = [_P, _I64, _P, _P, _P, _P, _P, _P]
        L.orbf_gershgorin.restype = _I
        L.orbf_solve_implicit.argtypes = [
            _P, _I64, _P, _P, _P, _P, _D, _D, _P, _P, _D, _I, _I,
            ctypes.POINTER(_I), ctypes.POINTER(_D)]
        L.orbf_solve_implicit.restype = _I
        L.orbf_implicit_ilu0.argtypes = [_P, _I64, _P, _P, _P, _P, _D, _D,
                                         _P]
        L.orbf_implicit_ilu0.restype = _I
        L.orbf_solve_implicit_krylov.argtypes = [
            _P, _I64, _P, _P, _P, _P, _D, _D, _P, _P, _D, _I, _I, _I, _I, _P,
            ctypes.POINTER(_I), ctypes.POINTER(_D)]
        L.orbf_solve_implicit_krylov.restype = _I
        L.orbf_bdf_coefficients.argtypes = [_I, ctypes.POINTER(_D),
                                             ctypes.POINTER(_D)]
        L.orbf_bdf_coefficients.restype = _I
        L.orbf_bdf_rhs.argtypes = [_P, _I64, _I, _P, _P, _P, _P, _P, _D, _P,
                                   _P, _P]
        L.orbf_bdf_rhs.restype = _I
        L.orbf_phase_times.argtypes = [_P, ctypes.POINTER(_D)]
        L.orbf_phase_times.restype = _I
        L.orbf_measure_fp64_fma.argtypes = [_P, ctypes.POINTER(_D)]
        L.orbf_measure_fp64_fma.restype = _I
        L.orbf_build_dm_batched.argtypes = [_P, ctypes.POINTER(SetDesc), _I]
        L.orbf_build_dm_batched.restype = _I
        L.orbf_set_workers.argtypes = [_P, _I]
        L.orbf_set_workers.restype = _I
        L.orbf_set_ir_max_corrections.argtypes = [_P, _I]
        L.orbf_set_ir_max_corrections.restype = _I
        L.orbf_server_create.argtypes = [_I, _I, ctypes.c_size_t,
                                         ctypes.c_size_t, _P]
        L.orbf_server_create.restype = _I
        L.orbf_server_destroy.argtypes = [_P]
        L.orbf_server_destroy.restype = None
        L.orbf_server_last_error.argtypes = [_P]
        L.orbf_server_last_error.restype = ctypes.c_char_p
        L.orbf_server_now.argtypes = []
        L.orbf_server_now.restype = _D
        L.orbf_request_bytes.argtypes = [_I64, _I, _I, _I]
        L.orbf_request_bytes.restype = ctypes.c_size_t
        L.orbf_server_submit.argtypes = [_P, ctypes.POINTER(Request),
                                         ctypes.POINTER(ctypes.c_uint64)]
        L.orbf_server_submit.restype = _I
        L.orbf_server_poll.argtypes = [_P, ctypes.POINTER(ctypes.c_uint64),
                                       _I, ctypes.POINTER(_I)]
        L.orbf_server_poll.restype = _I
        L.orbf_server_result.argtypes = [_P, ctypes.c_uint64,
                                         ctypes.POINTER(Result)]
        L.orbf_server_result.restype = _I
        L.orbf_server_fetch.argtypes = [_P, ctypes.c_uint64,
                                        ctypes.POINTER(SetDesc)]
        L.orbf_server_fetch.restype = _I
        L.orbf_server_release.argtypes = [_P, ctypes.c_uint64]
        L.orbf_server_release.restype = _I
        L.orbf_server_stats.argtypes = [_P, ctypes.POINTER(_I64)]
        L.orbf_server_stats.restype = _I
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    return t.contiguous()


class Context:
    """Library context bound to a device and a HIP stream (default: torch's
    current stream on ``device``).  ``budget`` caps the scratch memory in
    bytes (0 = no cap)."""

    def __init__(self, device=0, stream=None, budget=0):
        L = lib()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = ctypes.c_void_p()
        rc = L.orbf_create(device, ctypes.c_void_p(stream.cuda_stream),
                           int(budget), ctypes.byref(h))
        if rc != OK:
            raise OrbfError(rc, "orbf_create failed")
        self._h = h

    def check(self, rc):
        if rc != OK:
            msg = lib().orbf_last_error(self._h).decode()
            raise OrbfError(rc, msg)

    def sync(self):
        """Wait for the stream and raise any error the device recorded."""
        self.check(lib().orbf_sync(self._h))

    def set_ir_max_corrections(self, k):
        """FP32 + refinement: corrections allowed before a stencil is
        solved again in FP64 (default 8; 0 sends every stencil the first
        FP32 solve does not settle to FP64)."""
        self.check(lib().orbf_set_ir_max_corrections(self._h, int(k)))

    def phase_times(self):
        """[kNN, covering, weights, CSR, last weights kernel] in ms."""
        a = (_D * 5)()
        self.check(lib().orbf_phase_times(self._h, a))
        return list(a)

    def measure_fp64_fma(self):
        """The FP64 vector FMA rate this device reaches, in TFLOP/s (a
        measurement helper, blocking)."""
        v = _D()
        self.check(lib().orbf_measure_fp64_fma(self._h, ctypes.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "_h", None):
            lib().orbf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_size(N, d, n, l, prec=PREC_FP64):
    return lib().orbf_workspace_size(int(N), int(d), int(n), int(l), int(prec))


def build_nodes_knn(ctx, xyz, n):
    """Stencils (Sec. 2, Sec. 4.1): knn[N, n] int32 (self first), rho2[N]."""
    xyz = _dev(xyz, torch.float64, "xyz")
    N, d = xyz.shape
    knn = torch.empty((N, n), dtype=torch.int32, device=xyz.device)
    rho2 = torch.empty(N, dtype=torch.float64, device=xyz.device)
    ctx.check(lib().orbf_build_nodes_knn(ctx._h, _ptr(xyz), N, d, n,
                                         _ptr(knn), _ptr(rho2)))
    return knn, rho2


def select_overlapped_stencils(ctx, xyz, knn, rho2, delta, eligible=None):
    """Greedy overlapped covering (Sec. 4.1).  Returns centers (capacity N;
    the first n_centers entries are valid), n_centers (device int64 scalar
    tensor), owner[N] and p (rows per center, aligned with centers)."""
    xyz = _dev(xyz, torch.float64, "xyz")
    knn = _dev(knn, torch.int32, "knn")
    rho2 = _dev(rho2, torch.float64, "rho2")
    N, d = xyz.shape
    n = knn.shape[1]
    if eligible is not None:
        eligible = _dev(eligible, torch.uint8, "eligible")
    dev = xyz.device
    centers = torch.empty(N, dtype=torch.int32, device=dev)
    n_centers = torch.zeros(1, dtype=torch.int64, device=dev)
    owner = torch.empty(N, dtype=torch.int32, device=dev)
    p = torch.empty(N, dtype=torch.int32, device=dev)
    ctx.check(lib().orbf_select_overlapped_stencils(
        ctx._h, _ptr(xyz), _ptr(knn), _ptr(rho2), N, d, n, float(delta),
        _ptr(eligible), _ptr(centers), _ptr(n_centers), _ptr(owner), _ptr(p)))
    return centers, n_centers, owner, p


def compute_weights(ctx, op, m, l, n, delta, xyz, knn, rho2, *, centers=None,
                    n_centers=None, owner=None, rows=None, normals=None,
                    eligible=None, tau=math.inf, prec=PREC_FP64, W=None,
                    lebesgue=None, ir_steps=None, tau_mode=0):
    """Local weights (Sec. 4.1 eqs. rbffd_linsys / orbffd_eq / orbffd_rhs).

    Rows come from the covering (centers, n_centers, owner) or from an
    explicit ``rows`` list (each at its own node, delta = 1, e.g. boundary
    normal-derivative rows with ``normals``).  Returns W[N, n]: row e holds
    the weights of stencil owner[e] in stencil order."""
    xyz = _dev(xyz, torch.float64, "xyz")
    knn = _dev(knn, torch.int32, "knn")
    rho2 = _dev(rho2, torch.float64, "rho2")
    N, d = xyz.shape
    if W is None:
        W = torch.empty((N, n), dtype=torch.float64, device=xyz.device)
    a = WeightsArgs()
    a.xyz, a.N, a.d, a.knn, a.rho2 = _ptr(xyz), N, d, _ptr(knn), _ptr(rho2)
    if rows is not None:
        rows = _dev(rows, torch.int32, "rows")
        a.rows, a.n_rows = _ptr(rows), rows.numel()
        if owner is not None:
            a.owner = _ptr(owner)
    else:
        a.centers, a.n_centers, a.owner = (_ptr(centers), _ptr(n_centers),
                                           _ptr(owner))
    if normals is not None:
        normals = _dev(normals, torch.float64, "normals")
        a.normals = _ptr(normals)
    if eligible is not None:
        a.eligible = _ptr(_dev(eligible, torch.uint8, "eligible"))
    a.tau = float(tau)
    a.tau_mode = int(tau_mode)
    a.prec = int(prec)
    a.W = _ptr(W)
    a.lebesgue = _ptr(lebesgue)
    a.ir_steps = _ptr(ir_steps)
    ctx.check(lib().orbf_compute_weights(ctx._h, int(op), int(m), int(l),
                                         int(n), float(delta),
                                         ctypes.byref(a)))
    return W


def assemble_csr(ctx, knn, owner, W):
    """CSR of the DM (Sec. 4.1 scatter), columns ascending per row."""
    knn = _dev(knn, torch.int32, "knn")
    owner = _dev(owner, torch.int32, "owner")
    W = _dev(W, torch.float64, "W")
    N, n = knn.shape
    dev = knn.device
    row_ptr = torch.empty(N + 1, dtype=torch.int64, device=dev)
    col = torch.empty(N * n, dtype=torch.int32, device=dev)
    val = torch.empty(N * n, dtype=torch.float64, device=dev)
    ctx.check(lib().orbf_assemble_csr(ctx._h, N, n, _ptr(knn), _ptr(owner),
                                      _ptr(W), _ptr(row_ptr), _ptr(col),
                                      _ptr(val)))
    return row_ptr, col, val


def assemble_csr_noalloc(ctx, knn, owner, W, row_ptr, col, val):
    """``assemble_csr`` into caller-allocated outputs through the
    allocation-free entry point (its scratch is a fixed device array of the
    library): row_ptr int64 [N + 1], col int32 [N n], val float64 [N n]."""
    knn = _dev(knn, torch.int32, "knn")
    owner = _dev(owner, torch.int32, "owner")
    W = _dev(W, torch.float64, "W")
    N, n = knn.shape
    for t, dt, cnt, name in ((row_ptr, torch.int64, N + 1, "row_ptr"),
                             (col, torch.int32, N * n, "col"),
                             (val, torch.float64, N * n, "val")):
        if _dev(t, dt, name).data_ptr() != t.data_ptr() or t.numel() < cnt:
            raise ValueError(f"{name}: contiguous {dt}, >= {cnt} entries")
    ctx.check(lib().orbf_assemble_csr_noalloc(
        ctx._h, N, n, _ptr(knn), _ptr(owner), _ptr(W), _ptr(row_ptr),
        _ptr(col), _ptr(val)))
    return row_ptr, col, val


def spmv(ctx, row_ptr, col, val, x, y=None):
    """y = L x for a DM in CSR (device tensors); returns y."""
    row_ptr = _dev(row_ptr, torch.int64, "row_ptr")
    col = _dev(col, torch.int32, "col")
    val = _dev(val, torch.float64, "val")
    x = _dev(x, torch.float64, "x")
    N = row_ptr.numel() - 1
    if y is None:
        y = torch.empty(N, dtype=torch.float64, device=x.device)
    ctx.check(lib().orbf_spmv(ctx._h, N, _ptr(row_ptr), _ptr(col), _ptr(val),
                              _ptr(x), _ptr(y)))
    return y


def gershgorin(ctx, row_ptr, col, val, rows=True):
    """Gershgorin disks of a DM in CSR (Sec. 4.2.1): per-row centers L_kk
    and radii sum_{j != k} |L_kj| (None unless ``rows``), and the summary
    tensor [max_k L_kk + g_k, min_k L_kk - g_k, rows with L_kk + g_k > 0]."""
    row_ptr = _dev(row_ptr, torch.int64, "row_ptr")
    col = _dev(col, torch.int32, "col")
    val = _dev(val, torch.float64, "val")
    N = row_ptr.numel() - 1
    dev = row_ptr.device
    diag = radius = None
    if rows:
        diag = torch.empty(N, dtype=torch.float64, device=dev)
        radius = torch.empty(N, dtype=torch.float64, device=dev)
    summary = torch.empty(3, dtype=torch.float64, device=dev)
    ctx.check(lib().orbf_gershgorin(ctx._h, N, _ptr(row_ptr), _ptr(col),
                                    _ptr(val), _ptr(diag), _ptr(radius),
                                    _ptr(summary)))
    return diag, radius, summary


PRECONDS = {"none": 0, "jacobi": 1, "ilu0": 2}


def implicit_ilu0(ctx, row_ptr, col, val, *, alpha=1.0, beta=-1.0,
                  row_kind=None):
    """ILU(0) factors of the implicit step matrix (``orbf_implicit_ilu0``,
    the preconditioner of Secs. 7.1 and 7.2): a device tensor aligned with
    ``col``, L strictly below the diagonal (unit diagonal implied), U on and
    above."""
    row_ptr = _dev(row_ptr, torch.int64, "row_ptr")
    col = _dev(col, torch.int32, "col")
    val = _dev(val, torch.float64, "val")
    N = row_ptr.numel() - 1
    if row_kind is not None:
        row_kind = _dev(row_kind, torch.uint8, "row_kind")
        if row_kind.numel() != N:
            raise ValueError("row_kind must have one entry per DM row")
    lu = torch.empty_like(val)
    ctx.check(lib().orbf_implicit_ilu0(ctx._h, N, _ptr(row_ptr), _ptr(col),
                                       _ptr(val), _ptr(row_kind),
                                       float(alpha), float(beta), _ptr(lu)))
    return lu


METHODS = {"bicgstab": 0, "gmres": 1}


def solve_implicit(ctx, row_ptr, col, val, b, *, alpha=1.0, beta=-1.0,
                   row_kind=None, x0=None, tol=1e-10, max_iter=1000,
                   precond="none", method="bicgstab", restart=30, lu=None):
    """One implicit time step with a DM (Sec. 5): solve A x = b with row e
    of A equal to alpha x_e + beta (L x)_e where row_kind[e] == 1 (or
    everywhere if ``row_kind`` is None), x_e where it is 0 (Dirichlet) and
    (L x)_e elsewhere, from ``x0`` (zeros if None), by ``method``
    "bicgstab" or "gmres" (restarted after ``restart`` steps), ``precond``
    "none", "jacobi" or "ilu0" (``lu`` from ``implicit_ilu0`` of the same
    alpha, beta and row_kind; computed here if None).  Returns (x,
    iterations, relative residual)."""
    if precond not in PRECONDS:
        raise ValueError("precond must be 'none', 'jacobi' or 'ilu0'")
    if method not in METHODS:
        raise ValueError("method must be 'bicgstab' or 'gmres'")
    row_ptr = _dev(row_ptr, torch.int64, "row_ptr")
    col = _dev(col, torch.int32, "col")
    val = _dev(val, torch.float64, "val")
    b = _dev(b, torch.float64, "b")
    N = row_ptr.numel() - 1
    if b.numel() != N:
        raise ValueError("b must have one entry per DM row")
    if row_kind is not None:
        row_kind = _dev(row_kind, torch.uint8, "row_kind")
        if row_kind.numel() != N:
            raise ValueError("row_kind must have one entry per DM row")
    x = (torch.zeros_like(b) if x0 is None
         else _dev(x0, torch.float64, "x0").clone())
    if x.numel() != N:
        raise ValueError("x0 must have one entry per DM row")
    it = _I(0)
    res = _D(0.0)
    if method == "bicgstab" and precond != "ilu0":
        ctx.check(lib().orbf_solve_implicit(
            ctx._h, N, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(row_kind),
            float(alpha), float(beta), _ptr(b), _ptr(x), float(tol),
            int(max_iter), PRECONDS[precond], ctypes.byref(it),
            ctypes.byref(res)))
        return x, it.value, res.value
    if precond == "ilu0" and lu is None:
        lu = implicit_ilu0(ctx, row_ptr, col, val, alpha=alpha, beta=beta,
                           row_kind=row_kind)
    if lu is not None:
        lu = _dev(lu, torch.float64, "lu")
        if lu.numel() != val.numel():
            raise ValueError("lu must be aligned with col")
    ctx.check(lib().orbf_solve_implicit_krylov(
        ctx._h, N, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(row_kind),
        float(alpha), float(beta), _ptr(b), _ptr(x), float(tol),
        int(max_iter), METHODS[method], int(restart), PRECONDS[precond],
        _ptr(lu), ctypes.byref(it), ctypes.byref(res)))
    return x, it.value, res.value


def bdf_coefficients(order):
    """(a[0..3], b) of the BDF of ``order`` 1..4 (Sec. 5):
    u^{n+1} - sum_i a[i] u^{n-i} = b dt F(u^{n+1})."""
    a = (_D * 4)()
    b = _D(0.0)
    if lib().orbf_bdf_coefficients(int(order), a, ctypes.byref(b)) != OK:
        raise ValueError("BDF order must be 1..4")
    return list(a), b.value


def bdf_step(ctx, row_ptr, col, val, levels, dt, *, nu=1.0, f=None,
             row_kind=None, bvals=None, tol=1e-12, max_iter=1000,
             precond="none", method="bicgstab", restart=30, lu=None):
    """One BDF step of u_t = nu L u + f with the DM (Sec. 5), of order
    len(levels) (1..4; ``levels`` = [u^n, u^{n-1}, ...], newest first):
    orbf_bdf_rhs, then the implicit solve from u^n (``method``,
    ``precond``, ``lu`` as for ``solve_implicit``; an ILU(0) ``lu`` must be
    that of beta = -b_k nu dt).  Returns (u^{n+1}, iterations, relative
    residual)."""
    k = len(levels)
    if not 1 <= k <= 4:
        raise ValueError("BDF order must be 1..4")
    levels = [_dev(u, torch.float64, "u") for u in levels]
    N = levels[0].numel()
    if f is not None:
        f = _dev(f, torch.float64, "f")
    if row_kind is not None:
        row_kind = _dev(row_kind, torch.uint8, "row_kind")
    if bvals is not None:
        bvals = _dev(bvals, torch.float64, "bvals")
    for t in [f, row_kind, bvals] + levels:
        if t is not None and t.numel() != N:
            raise ValueError("every vector needs one entry per DM row")
    rhs = torch.empty_like(levels[0])
    u = levels + [None] * (4 - k)
    ctx.check(lib().orbf_bdf_rhs(ctx._h, N, k, _ptr(u[0]), _ptr(u[1]),
                                 _ptr(u[2]), _ptr(u[3]), _ptr(f), float(dt),
                                 _ptr(row_kind), _ptr(bvals), _ptr(rhs)))
    _, b = bdf_coefficients(k)
    return solve_implicit(ctx, row_ptr, col, val, rhs, alpha=1.0,
                          beta=-b * nu * dt, row_kind=row_kind, x0=levels[0],
                          tol=tol, max_iter=max_iter, precond=precond,
                          method=method, restart=restart, lu=lu)


def build_dm(xyz, n, m, l, delta, *, tau=math.inf, eligible=None,
             boundary=None, normals=None, prec=PREC_FP64, ctx=None,
             sync=True, op=OP_LAPLACIAN, tau_mode=0):
    """Whole DM build on the device: stencils, covering, interior rows of
    operator ``op`` (LAPLACIAN, DX, DY, DZ or IDENTITY; a finite ``tau``
    only with the Laplacian), optional normal-derivative rows at
    ``boundary`` nodes, CSR.  Returns a dict of device tensors (plus
    ``ctx``)."""
    own_ctx = ctx is None
    if own_ctx:
        ctx = Context(xyz.device.index or 0)
    knn, rho2 = build_nodes_knn(ctx, xyz, n)
    if math.isinf(tau):
        centers, n_centers, owner, p = select_overlapped_stencils(
            ctx, xyz, knn, rho2, delta, eligible)
    else:
        # the covering with the Lebesgue test is made by compute_weights
        N = xyz.shape[0]
        centers = torch.empty(N, dtype=torch.int32, device=xyz.device)
        n_centers = torch.zeros(1, dtype=torch.int64, device=xyz.device)
        owner = torch.empty(N, dtype=torch.int32, device=xyz.device)
        p = None
    lam = torch.zeros(xyz.shape[0], dtype=torch.float64, device=xyz.device)
    ir_steps = None
    if prec == PREC_FP32_IR:
        ir_steps = torch.empty(xyz.shape[0], dtype=torch.int32,
                               device=xyz.device)
    W = compute_weights(ctx, op, m, l, n, delta, xyz, knn, rho2,
                        centers=centers, n_centers=n_centers, owner=owner,
                        eligible=eligible, tau=tau, prec=prec, lebesgue=lam,
                        ir_steps=ir_steps, tau_mode=tau_mode)
    if boundary is not None and len(boundary):
        compute_weights(ctx, OP_NEUMANN, m, l, n, 1.0, xyz, knn, rho2,
                        rows=boundary, normals=normals, owner=owner, W=W,
                        lebesgue=lam, prec=prec)
    row_ptr, col, val = assemble_csr(ctx, knn, owner, W)
    if sync:
        ctx.sync()
    return dict(knn=knn, rho2=rho2, centers=centers, n_centers=n_centers,
                owner=owner, p=p, W=W, lam=lam, row_ptr=row_ptr, col=col,
                val=val, ir_steps=ir_steps, ctx=ctx)


def _outputs(N, n, dev, prec):
    """Device output tensors of one DM build."""
    o = dict(knn=torch.empty((N, n), dtype=torch.int32, device=dev),
             rho2=torch.empty(N, dtype=torch.float64, device=dev),
             centers=torch.empty(N, dtype=torch.int32, device=dev),
             n_centers=torch.zeros(1, dtype=torch.int64, device=dev),
             owner=torch.empty(N, dtype=torch.int32, device=dev),
             W=torch.empty((N, n), dtype=torch.float64, device=dev),
             lam=torch.zeros(N, dtype=torch.float64, device=dev),
             ir_steps=None,
             row_ptr=torch.empty(N + 1, dtype=torch.int64, device=dev),
             col=torch.empty(N * n, dtype=torch.int32, device=dev),
             val=torch.empty(N * n, dtype=torch.float64, device=dev))
    if prec == PREC_FP32_IR:
        o["ir_steps"] = torch.empty(N, dtype=torch.int32, device=dev)
    return o


def _fill_outputs(dsc, o):
    dsc.knn, dsc.rho2 = _ptr(o["knn"]), _ptr(o["rho2"])
    dsc.centers, dsc.n_centers = _ptr(o["centers"]), _ptr(o["n_centers"])
    dsc.owner, dsc.W, dsc.lebesgue = (_ptr(o["owner"]), _ptr(o["W"]),
                                      _ptr(o["lam"]))
    dsc.ir_steps = _ptr(o["ir_steps"])
    dsc.row_ptr, dsc.col, dsc.val = (_ptr(o["row_ptr"]), _ptr(o["col"]),
                                     _ptr(o["val"]))


def build_dm_batched(ctx, sets, outputs=None, sync=True):
    """Many DM builds in one call (``orbf_build_dm_batched``).

    ``sets``: list of dicts with ``xyz`` (device float64 [N, d]), ``n``,
    ``m``, ``l``, ``delta`` and optionally ``tau``, ``prec``, ``eligible``,
    ``boundary``, ``normals``.  ``outputs``: the list this function returned
    before, to build into the same buffers (a repeated batch with the same
    buffers is replayed from a HIP graph).  Returns one dict of device
    tensors per set."""
    descs = (SetDesc * len(sets))()
    keep = []
    if outputs is None:
        outputs = []
        for s in sets:
            x = s["xyz"]
            outputs.append(_outputs(x.shape[0], s["n"], x.device,
                                    s.get("prec", PREC_FP64)))
    for i, s in enumerate(sets):
        x = _dev(s["xyz"], torch.float64, "xyz")
        dsc = descs[i]
        dsc.xyz, dsc.N, dsc.d = _ptr(x), x.shape[0], x.shape[1]
        dsc.n, dsc.m, dsc.l = int(s["n"]), int(s["m"]), int(s["l"])
        dsc.delta = float(s["delta"])
        dsc.tau = float(s.get("tau", math.inf))
        dsc.prec = int(s.get("prec", PREC_FP64))
        if s.get("eligible") is not None:
            el = _dev(s["eligible"], torch.uint8, "eligible")
            keep.append(el)
            dsc.eligible = _ptr(el)
        if s.get("boundary") is not None:
            b = _dev(s["boundary"], torch.int32, "boundary")
            nr = _dev(s["normals"], torch.float64, "normals")
            keep += [b, nr]
            dsc.boundary, dsc.n_boundary, dsc.normals = (_ptr(b), b.numel(),
                                                         _ptr(nr))
        keep.append(x)
        _fill_outputs(dsc, outputs[i])
    ctx.check(lib().orbf_build_dm_batched(ctx._h, descs, len(sets)))
    if sync:
        ctx.sync()
    ctx._batch_keep = keep  # inputs stay alive while the batch may run
    return outputs


class Server:
    """Request engine with continuous admission (``orbf_server_*``).

    ``slots`` concurrent builds; ``arena`` bytes of device memory for the
    outputs of admitted requests; ``slot_scratch`` bytes of scratch per
    slot (a request needs orbf_workspace_size of it)."""

    def __init__(self, device=0, slots=4, arena=6 << 30,
                 slot_scratch=512 << 20):
        L = lib()
        h = ctypes.c_void_p()
        rc = L.orbf_server_create(int(device), int(slots), int(arena),
                                  int(slot_scratch), ctypes.byref(h))
        if rc != OK:
            raise OrbfError(rc, "orbf_server_create failed")
        self._h = h
        self.device = device
        self._inputs = {}

    def check(self, rc):
        if rc != OK:
            raise OrbfError(rc, lib().orbf_server_last_error(self._h).decode())

    @staticmethod
    def now():
        return lib().orbf_server_now()

    def submit(self, xyz, n, m, l, delta, tau=math.inf, prec=PREC_FP64,
               t_arrival=None):
        x = _dev(xyz, torch.float64, "xyz")
        # the slot waits for this event, so coordinates still being written
        # on the current stream are read only once complete
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(x.device))
        r = Request(xyz=_ptr(x), N=x.shape[0], d=x.shape[1], n=int(n),
                    m=int(m), l=int(l), delta=float(delta), tau=float(tau),
                    prec=int(prec),
                    t_arrival=self.now() if t_arrival is None else t_arrival,
                    ready=ev.cuda_event)
        t = ctypes.c_uint64()
        self.check(lib().orbf_server_submit(self._h, ctypes.byref(r),
                                            ctypes.byref(t)))
        # the request reads x, and waits on ev, until it is done
        self._inputs[t.value] = (x, ev)
        return t.value

    def poll(self, cap=1024):
        buf = (ctypes.c_uint64 * cap)()
        k = _I()
        self.check(lib().orbf_server_poll(self._h, buf, cap, ctypes.byref(k)))
        return [buf[i] for i in range(k.value)]

    def result(self, ticket):
        r = Result()
        self.check(lib().orbf_server_result(self._h, ticket, ctypes.byref(r)))
        return dict(status=r.status, N=r.N, n=r.n, n_centers=r.n_centers,
                    t_arrival=r.t_arrival, t_admit=r.t_admit,
                    t_done=r.t_done)

    def fetch(self, ticket, prec=PREC_FP64):
        """Copy a finished request's outputs into new device tensors."""
        info = self.result(ticket)
        o = _outputs(info["N"], info["n"], torch.device("cuda", self.device),
                     prec)
        dsc = SetDesc()
        _fill_outputs(dsc, o)
        # the copies are not stream-ordered: nothing pending may still use
        # the memory the new tensors took
        torch.cuda.current_stream(o["knn"].device).synchronize()
        self.check(lib().orbf_server_fetch(self._h, ticket,
                                           ctypes.byref(dsc)))
        return o

    def release(self, ticket):
        self.check(lib().orbf_server_release(self._h, ticket))
        self._inputs.pop(ticket, None)

    def stats(self):
        a = (_I64 * 5)()
        self.check(lib().orbf_server_stats(self._h, a))
        return dict(waiting=a[0], running=a[1], finished=a[2],
                    arena_used=a[3], arena_bytes=a[4])

    def close(self):
        if getattr(self, "_h", None):
            lib().orbf_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

