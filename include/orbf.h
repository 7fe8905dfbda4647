/*
 * orbf.h -- C ABI of liborbf, an MI355X (gfx950) builder of overlapped
 * RBF-FD differentiation matrices (V. Shankar, "The Overlapped Radial Basis
 * Function-Finite Difference (RBF-FD) Method: A Generalization of RBF-FD").
 *
 * The build has four stream-ordered stages, each an entry point below:
 *   1. orbf_build_nodes_knn            stencils: each node and its n-1
 *                                      nearest neighbours (Sec. 2, Sec. 4.1)
 *   2. orbf_select_overlapped_stencils greedy choice of stencil centers and
 *                                      of the retention ball rows each one
 *                                      computes (Sec. 4.1)
 *   3. orbf_compute_weights            per-center augmented polyharmonic
 *                                      spline saddle solve with one right-hand
 *                                      side per retained node (eqs.
 *                                      rbffd_linsys, orbffd_eq, orbffd_rhs),
 *                                      optional L-Lebesgue rejection
 *                                      (Sec. 4.2.1, eq. calLstab)
 *   4. orbf_assemble_csr               scatter of the weights into the sparse
 *                                      DM, L(R_i, I_j) = W_{j,i} (Sec. 4.1)
 *
 * Conventions for every entry point:
 *   - Pointers to arrays are DEVICE pointers on the context's device unless
 *     a comment says "host".  The caller allocates every input and output
 *     and keeps ownership; the library never frees caller memory.
 *   - Node coordinates are FP64, array-of-structures: xyz[i*d + a], d = 2|3.
 *   - All work is enqueued on the context's HIP stream and is asynchronous:
 *     outputs are valid once the stream (or orbf_sync) has completed.
 *   - Host-side argument errors return at once and enqueue nothing.
 *     Errors found on the device (coincident nodes, a singular local system)
 *     are recorded in a device status word and returned by the next
 *     orbf_sync; orbf_last_error then names the offending node or stencil.
 *   - No C++ exception crosses this interface.  A context is used by one
 *     host thread at a time.
 */
#ifndef ORBF_H
#define ORBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum orbf_status {
  ORBF_OK = 0,
  ORBF_EINVAL = 1,     /* invalid argument: d not 2|3, n > N, n < M, even or
                          too small PHS exponent, delta outside [0,1], tau < 1,
                          NULL pointer, unsupported size                     */
  ORBF_EDUPLICATE = 2, /* two distinct nodes at squared distance zero         */
  ORBF_ESINGULAR = 3,  /* a local saddle system had an exact zero pivot       */
  ORBF_ENOMEM = 4,     /* device allocation of context scratch failed         */
  ORBF_EBUDGET = 5,    /* scratch would exceed the context's HBM budget       */
  ORBF_EHIP = 6,       /* a HIP runtime call failed                           */
  ORBF_EINTERNAL = 7   /* an internal limit was hit (message says which)      */
} orbf_status;

/* The operator L whose DM is built (Sec. 4.1: the right-hand sides are L
 * applied to the RBF and polynomial basis at each computed row's node, and
 * the weights are unscaled by rho^theta, theta the order of L). */
typedef enum orbf_op {
  ORBF_OP_LAPLACIAN = 0, /* L = Laplacian (interior rows, Sec. 4.1 / Sec. 7),
                            theta = 2                                        */
  ORBF_OP_NEUMANN = 1,   /* L = n . grad, the normal derivative of the
                            Neumann boundary operator (Sec. 5), theta = 1;
                            explicit rows with normals only                  */
  ORBF_OP_DX = 2,        /* L = d/dx, theta = 1                              */
  ORBF_OP_DY = 3,        /* L = d/dy, theta = 1                              */
  ORBF_OP_DZ = 4,        /* L = d/dz (d = 3), theta = 1                      */
  ORBF_OP_IDENTITY = 5   /* L = I (interpolation at the row's node),
                            theta = 0: every row is the unit vector of its
                            node, up to rounding                             */
} orbf_op;

typedef enum orbf_prec {
  ORBF_PREC_FP64 = 0,   /* factor and solve in FP64                          */
  ORBF_PREC_FP32_IR = 1 /* elimination and its replays in FP32; residuals
                           B_hat - A_hat X, the accumulated solution X, the
                           weights and the Lebesgue sums in FP64; refinement
                           until max|dX| <= 1e-11 max|X| over the weights of
                           every column (at most 8 corrections), stencils
                           that do not settle solved again in FP64.  The
                           covering decisions of mode (c) use FP64 solves.   */
} orbf_prec;

typedef struct orbf_ctx orbf_ctx;

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  `hbm_budget_bytes` caps the
 * scratch memory the context may hold (0 = no cap).  *out receives the
 * context.  Returns ORBF_EHIP if the device cannot be selected. */
orbf_status orbf_create(int device, void* hip_stream, size_t hbm_budget_bytes,
                        orbf_ctx** out);

/* Free the context and its scratch (waits for its stream first). */
void orbf_destroy(orbf_ctx* ctx);

/* Message of the last error on this context ("" if none).  The string is
 * owned by the context and valid until the next call on it. */
const char* orbf_last_error(const orbf_ctx* ctx);

/* Wait for the context's stream, then return (and clear) the first error the
 * device recorded since the previous orbf_sync. */
orbf_status orbf_sync(orbf_ctx* ctx);

/* Bytes of context scratch one build of N nodes needs (dimension d, stencil
 * size n, polynomial degree l): what admission control reserves per
 * request. */
size_t orbf_workspace_size(int64_t N, int d, int n, int l, orbf_prec prec);

/* Stencils (Sec. 2; Sec. 4.1 with I^k_1 = k).
 * For every node i, the n nodes nearest to it, itself included, ordered by
 * the key (squared distance, global index) ascending, so knn[i*n] == i.
 * Squared distances are ((dx*dx)+(dy*dy))+(dz*dz) in FP64 with every
 * operation rounded separately; ties are broken by the smaller index.
 *   xyz  : N*d   FP64 input
 *   knn  : N*n   int32 output
 *   rho2 : N     FP64 output, squared stencil width rho_k^2 = squared
 *                distance to the n-th neighbour (Sec. 4.1)
 * The context also keeps the n squared distances of every stencil (N*n
 * FP64 of its scratch) together with the xyz and knn pointers; see
 * orbf_select_overlapped_stencils.
 * Errors: EINVAL (d, n < 1, n > N, N > 2^31-1, NULL), EDUPLICATE at sync
 * time if two nodes coincide. */
orbf_status orbf_build_nodes_knn(orbf_ctx* ctx, const double* xyz, int64_t N,
                                 int d, int n, int32_t* knn, double* rho2);

/* Greedy overlapped covering (Sec. 4.1), without Lebesgue rejection.
 * Nodes are visited in ascending index.  An eligible node not yet claimed
 * becomes a center k and claims every eligible, unclaimed node j of its
 * stencil inside the closed retention ball
 *     d^2(x_k, x_j) <= ((1-delta)*(1-delta)) * rho2[k]
 * (retention distance (1-delta) rho_k; delta = 1 gives standard RBF-FD with
 * every eligible node its own center, delta = 0 keeps the whole stencil).
 * The result is the sequential greedy result exactly, although the device
 * evaluates it in parallel: each decided node updates its successors once.
 *   eligible  : N uint8 (nonzero = gets an interior row) or NULL for all
 *   centers   : capacity N int32 output, centers in ascending order
 *   n_centers : 1 int64 output (device): number of centers N_delta
 *   owner     : N int32 output: center whose stencil computes row j, -1 for
 *               ineligible nodes (owner[k] == k for centers)
 *   p         : capacity N int32 output: p[c] = rows computed by centers[c]
 * When xyz and knn are the arrays of this context's latest
 * orbf_build_nodes_knn call (same pointers and sizes), the squared distances
 * it recorded are used instead of gathering coordinates; they are the same
 * values.  A caller that changes those arrays in place between the two
 * calls must run orbf_build_nodes_knn again.  The same holds for the
 * Lebesgue covering of orbf_compute_weights (mode c).
 * Errors: EINVAL (delta outside [0,1] or NaN, sizes, NULL). */
orbf_status orbf_select_overlapped_stencils(
    orbf_ctx* ctx, const double* xyz, const int32_t* knn, const double* rho2,
    int64_t N, int d, int n, double delta, const uint8_t* eligible,
    int32_t* centers, int64_t* n_centers, int32_t* owner, int32_t* p);

/* Arguments of orbf_compute_weights beyond the operator description. */
typedef struct orbf_weights_args {
  const double* xyz;     /* N*d nodes                                        */
  int64_t N;             /* number of nodes                                  */
  int d;                 /* dimension, 2 or 3                                */
  const int32_t* knn;    /* N*n stencils from orbf_build_nodes_knn           */
  const double* rho2;    /* N squared stencil widths                         */
  /* Row selection, one of three modes:
   *  (a) rows != NULL: explicit rows; row rows[i] is computed at its own node
   *      on its own stencil (delta = 1), e.g. the boundary rows of Sec. 5;
   *      owner[rows[i]] is set to rows[i].
   *  (b) rows == NULL, tau infinite: the covering of
   *      orbf_select_overlapped_stencils; `centers`, `n_centers` and `owner`
   *      are its outputs, read here.
   *  (c) rows == NULL, tau finite: the covering is recomputed with the
   *      L-Lebesgue rejection of Sec. 4.2.1 and `centers`, `n_centers`,
   *      `owner` are OUTPUTS (capacities N). */
  const int32_t* rows;   /* n_rows explicit row nodes, or NULL               */
  int64_t n_rows;        /* number of explicit rows (host value)             */
  int32_t* centers;      /* see above                                        */
  int64_t* n_centers;    /* device scalar, see above                         */
  int32_t* owner;        /* N, see above                                     */
  const uint8_t* eligible; /* mode (c): nodes that get rows (NULL = all)     */
  const double* normals; /* n_rows*d unit normals (ORBF_OP_NEUMANN)          */
  double tau;            /* Lebesgue threshold: node e of stencil k is kept
                            iff e is the center or
                            Lambda(x_e) <= tau * Lambda(x_ref), x_ref the
                            stencil node nearest the stencil centroid; tau = 1
                            is eq. calLstab; INFINITY disables the test     */
  orbf_prec prec;        /* ORBF_PREC_FP64 or ORBF_PREC_FP32_IR              */
  double* W;             /* N*n output: W[e*n + q] is the weight of node
                            knn[owner[e]*n + q] in row e (physical units)    */
  double* lebesgue;      /* N output or NULL: Lambda of each computed row    */
  int32_t* ir_steps;     /* N output or NULL, written when prec is FP32_IR
                            in modes (b)/(c): the number of FP64-residual
                            corrections after the first FP32 solve of the
                            row's right-hand-side block; -1 where the row was
                            solved in FP64 (FP32 zero pivot, no convergence
                            within the correction cap, 8 unless
                            orbf_set_ir_max_corrections, n + M > 72, no
                            owner).  Mode (a) rows are always FP64 and leave
                            it untouched.                                    */
  int tau_mode;          /* mode (c): how the threshold shrinks a stencil's
                            retained set.  0: node by node, as `tau` says.
                            1: radial prefix (the overlap ball shrunk for the
                            stencil, Sec. 4.2.1 with Sec. 4.4's delta-free
                            retention): with q* the first stencil position
                            of an eligible node of the retention ball,
                            claimed by an earlier center or not, that fails
                            the test, the center keeps only its unclaimed
                            eligible ball nodes before q*.  0 when zeroed. */
} orbf_weights_args;

/* Local weights (Sec. 4.1, eqs. rbffd_linsys, orbffd_eq, orbffd_rhs).
 * For each center k: scaled coordinates xi = (x - x_k)/rho_k, the
 * (n+M) x (n+M) system [A Psi; Psi^T 0] with A_ij = |xi_i - xi_j|^m and Psi
 * the M = C(l+d, d) monomials of degree <= l, one right-hand side per
 * computed row e holding L|xi - xi_j|^m and L psi at xi_e; partial-pivot LU
 * and triangular solves; weights unscaled by rho_k^theta (2 for the
 * Laplacian, 1 for first derivatives, 0 for the identity); W^psi is
 * discarded.
 *   op : LAPLACIAN, DX, DY, DZ or IDENTITY in modes (a) and (b); NEUMANN in
 *        mode (a) only; mode (c), the Lebesgue test, with the LAPLACIAN
 *   m  : odd PHS exponent >= 3;
 *   l  : polynomial degree >= 0, or -1 for no polynomial part (M = 0: the
 *        unaugmented system A w = L phi that Sec. 4.3's cost count also
 *        covers; A alone can be singular for PHS, reported as ESINGULAR
 *        only when a pivot is exactly zero);
 *   n  : stencil size (>= M);    delta : overlap parameter in [0,1] (mode c)
 * Errors: EINVAL (parameters, NULL outputs, n + M > 144, mode/op mismatch),
 * ESINGULAR at sync time (exact zero pivot; the stencil's rows are NaN). */
orbf_status orbf_compute_weights(orbf_ctx* ctx, orbf_op op, int m, int l,
                                 int n, double delta,
                                 const orbf_weights_args* args);

/* Sparse DM in CSR (Sec. 4.1: L(R^k_i, I^k_j) = W^{phi,k}_{j,i}).
 * Row e holds the n indices of stencil owner[e] in ascending order with the
 * matching weights of W (row e); rows with owner[e] < 0 are empty.
 *   row_ptr : N+1 int64 output;  col : N*n int32;  val : N*n FP64 outputs
 *             (only row_ptr[N] entries are written). */
orbf_status orbf_assemble_csr(orbf_ctx* ctx, int64_t N, int n,
                              const int32_t* knn, const int32_t* owner,
                              const double* W, int64_t* row_ptr, int32_t* col,
                              double* val);

/* orbf_assemble_csr for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result, bit for bit, but the
 * scratch (row lengths, per-stencil ranks, scan temporaries: about
 * N * (n + 4) bytes) lives in a fixed 64 MiB device array of the library,
 * one per device, set up by orbf_create; no call allocates or frees
 * anything.  Arguments, layout and ownership as for orbf_assemble_csr;
 * owner must be as the covering makes it (owner[owner[e]] == owner[e]).
 * Errors: EINVAL as orbf_assemble_csr; EBUDGET if N and n need more than
 * the 64 MiB (N * n up to about 6.4e7: the 1M-node, n = 50 DM fits).
 * Calls that overlap on one device share the array and race: serialise
 * them (one stream, or events). */
orbf_status orbf_assemble_csr_noalloc(orbf_ctx* ctx, int64_t N, int n,
                                      const int32_t* knn,
                                      const int32_t* owner, const double* W,
                                      int64_t* row_ptr, int32_t* col,
                                      double* val);

/* y = L x for a DM in CSR: the discrete operator applied to nodal values
 * x (Sec. 4.1: (L f)(x_i) is approximated by sum_j L_ij f(x_j)), the
 * product every use of the DM (time stepping, Krylov solves, Sec. 5) is
 * built on.
 *   row_ptr, col, val : the CSR (device; as from orbf_assemble_csr)
 *   x : N FP64 input (device; indexed by col);  y : N FP64 output (device)
 * Each y[i] sums its row's products in a fixed order (deterministic).
 * Errors: EINVAL (N out of range, NULL pointer, x == y). */
orbf_status orbf_spmv(orbf_ctx* ctx, int64_t N, const int64_t* row_ptr,
                      const int32_t* col, const double* val, const double* x,
                      double* y);

/* Gershgorin disks of a DM in CSR (Sec. 4.2.1, "Improving stability"): row
 * k's disk has center L_kk and radius g_k = sum_{j != k} |L_kj| (for a DM
 * row, its L-Lebesgue value minus |L_kk|); every eigenvalue of L lies in
 * their union, so no eigenvalue can have a positive real part unless some
 * disk reaches past 0.  An empty row has center 0 and radius 0.
 *   row_ptr, col, val : the CSR (device; as from orbf_assemble_csr)
 *   diag, radius      : N FP64 outputs (device), each may be NULL
 *   summary           : 3 FP64 outputs (device): max_k (L_kk + g_k),
 *                       min_k (L_kk - g_k), and the number of rows with
 *                       L_kk + g_k > 0
 * The radii are sums in an order of the library's choosing (deterministic
 * for a given N).  Errors: EINVAL (N out of range, NULL input or summary). */
orbf_status orbf_gershgorin(orbf_ctx* ctx, int64_t N, const int64_t* row_ptr,
                            const int32_t* col, const double* val,
                            double* diag, double* radius, double* summary);

/* One implicit time step with a DM (Sec. 5, "Time-Stepping": the backward
 * Euler system whose interior block is I - nu dt L and whose boundary rows
 * impose the boundary condition): solve A x = b, where row e of A is
 *   row_kind[e] == 1 : alpha x_e + beta (L x)_e   (interior; backward Euler
 *                      has alpha = 1, beta = -nu dt)
 *   row_kind[e] == 0 : x_e                        (Dirichlet)
 *   any other value  : (L x)_e                    (a boundary-operator row
 *                      of the DM, e.g. a normal derivative for Neumann data)
 * by BiCGSTAB (van der Vorst 1992), started from x, unpreconditioned or
 * with Jacobi right preconditioning (D = diag A).
 *   row_ptr, col, val : the CSR of L (device; as from orbf_assemble_csr)
 *   row_kind : N bytes (device), or NULL for all rows interior
 *   b        : N FP64 right-hand side (device);  x : N FP64 (device), in:
 *              the initial guess (e.g. the previous time level), out: the
 *              solution
 *   tol      : stop when ||b - A x||_2 <= tol ||b||_2 (the recurrence
 *              residual; ||b|| = 0 is taken as 1)
 *   max_iter : iteration limit
 *   precond  : ORBF_PRECOND_NONE or ORBF_PRECOND_JACOBI.  Jacobi evens out
 *              the row scales of boundary-operator rows (about 1/h) and
 *              interior rows (about 1 + dt |L_ee|): it cuts the iterations of
 *              Neumann steps 2-3x but costs iterations on Dirichlet steps
 *   iters, relres : host outputs (each may be NULL): iterations done and
 *              the final relative residual
 * Synchronous: returns after the solve, reading four inner products back
 * to the host per iteration; every inner product is summed in a fixed
 * order, so a solve is deterministic.  Not converging within max_iter, or a
 * BiCGSTAB breakdown, is not an error: relres says how far it got.  Scratch:
 * 10 N FP64 plus 16 KB of the context.
 * Errors: EINVAL (N out of range, NULL input, b == x, tol < 0 or NaN,
 * max_iter < 0, alpha or beta not finite, unknown precond), ENOMEM,
 * EHIP. */
enum {
  ORBF_PRECOND_NONE = 0,
  ORBF_PRECOND_JACOBI = 1,
  ORBF_PRECOND_ILU0 = 2  /* orbf_solve_implicit_krylov only */
};
orbf_status orbf_solve_implicit(orbf_ctx* ctx, int64_t N,
                                const int64_t* row_ptr, const int32_t* col,
                                const double* val, const uint8_t* row_kind,
                                double alpha, double beta, const double* b,
                                double* x, double tol, int max_iter,
                                int precond, int* iters, double* relres);

/* ILU(0) of the implicit step matrix A of orbf_solve_implicit (rows chosen
 * by row_kind, alpha, beta), the preconditioner Secs. 7.1 and 7.2 use:
 * Gaussian elimination restricted to A's sparsity pattern, which is the
 * DM's (for each row i and each k < i in it, ascending: a_ik /= a_kk, then
 * a_ij -= a_ik a_kj for the j > k present in both rows).  L (unit lower)
 * and U are written to lu, aligned with the CSR (lu[t] belongs to col[t]).
 * Every row must hold its diagonal (DM rows do).
 *   row_ptr, col, val : the CSR of L (device);  row_kind, alpha, beta : as
 *   for orbf_solve_implicit;  lu : nnz FP64 output (device, not aliasing
 *   val)
 * Asynchronous.  One launch factors all rows: each row waits for the rows
 * it depends on, in order.  Errors: EINVAL (sizes, NULL, lu == val); at
 * sync time EINVAL (a row without a diagonal entry), ESINGULAR (a zero
 * pivot), EINTERNAL (a bounded wait ran out).  Scratch: 16 N bytes. */
orbf_status orbf_implicit_ilu0(orbf_ctx* ctx, int64_t N,
                               const int64_t* row_ptr, const int32_t* col,
                               const double* val, const uint8_t* row_kind,
                               double alpha, double beta, double* lu);

/* The implicit step of orbf_solve_implicit with a choice of Krylov method
 * and preconditioner (Sec. 5; Sec. 7.1 uses GMRES with ILU(0) in 2D, Sec.
 * 7.2 BiCGSTAB with ILU(0) in 3D):
 *   method   : ORBF_KRYLOV_BICGSTAB, or ORBF_KRYLOV_GMRES (restarted after
 *              `restart` steps, 1..64; classical Gram-Schmidt twice)
 *   precond  : ORBF_PRECOND_NONE, _JACOBI, or _ILU0 with lu from
 *              orbf_implicit_ilu0 of the same row_kind, alpha and beta (right
 *              preconditioning: A M^-1 y = b, x = M^-1 y)
 * Other arguments, stopping rule and outputs as for orbf_solve_implicit
 * (GMRES stops on its residual estimate and reports the true residual of
 * the last restart).  Synchronous.  Scratch: BiCGSTAB 10 N FP64, GMRES
 * (restart + 5) N FP64, ILU(0) 16 N bytes, plus 0.6 MB.
 * Errors: as orbf_solve_implicit; EINVAL also for an unknown method, a
 * restart out of range, ILU0 without lu. */
enum { ORBF_KRYLOV_BICGSTAB = 0, ORBF_KRYLOV_GMRES = 1 };
orbf_status orbf_solve_implicit_krylov(
    orbf_ctx* ctx, int64_t N, const int64_t* row_ptr, const int32_t* col,
    const double* val, const uint8_t* row_kind, double alpha, double beta,
    const double* b, double* x, double tol, int max_iter, int method,
    int restart, int precond, const double* lu, int* iters, double* relres);

/* Coefficients of the backward differentiation formula of order k = 1..4
 * (Sec. 5 time-steps with BDF4 and starts it with BDF1-3):
 *     u^{n+1} - sum_{i<k} a[i] u^{n-i} = b dt F(u^{n+1}),
 * k = 4: a = (48, -36, 16, -3)/25, b = 12/25.  a: 4 host doubles (zero
 * past k), b: 1 host double.  Needs no context.  Errors: EINVAL. */
orbf_status orbf_bdf_coefficients(int order, double* a, double* b);

/* Right-hand side of one BDF step of u_t = nu L u + f with the DM (Sec. 5):
 *     rhs_e = sum_{i<k} a[i] u_i[e] + b dt f[e]   where row_kind[e] == 1
 *     rhs_e = bvals[e] (0 if bvals is NULL)        elsewhere
 * with a, b from orbf_bdf_coefficients.  Solving
 * orbf_solve_implicit(..., row_kind, 1, -b nu dt, rhs, x, ...) then gives
 * u^{n+1}: interior rows satisfy the BDF formula, Dirichlet rows take
 * bvals, boundary-operator rows (e.g. Neumann) equal bvals.
 *   order    : k = 1..4
 *   u0..u3   : N FP64 (device): u0 = u^n (newest), u1 = u^{n-1}, ...; the
 *              first k must be non-NULL, the rest are ignored
 *   f        : N FP64 forcing at t^{n+1} (device), or NULL for none
 *   row_kind : N bytes (device), as for orbf_solve_implicit, or NULL
 *   bvals    : N FP64 boundary data at t^{n+1} (device), or NULL
 *   rhs      : N FP64 output (device), must not alias a time level
 * Errors: EINVAL (N out of range, order, NULL level or rhs, aliasing,
 * dt not finite and positive). */
orbf_status orbf_bdf_rhs(orbf_ctx* ctx, int64_t N, int order,
                         const double* u0, const double* u1,
                         const double* u2, const double* u3, const double* f,
                         double dt, const uint8_t* row_kind,
                         const double* bvals, double* rhs);

/* Kernel schedules for the weights.  Stencils of one system size K = n + M
 * are solved by one of these kernels; which is fastest depends on K and on
 * how many rows a stencil keeps, estimated as n (1-delta)^d: p-class 0 for
 * at most 8, p-class 1 above (explicit rows are p-class 0).  The table is
 * filled by an autotuner that times the candidates (Python:
 * paper_1606_03135_amd.tune) and consulted by orbf_compute_weights; sizes
 * without an entry use SPLIT for K <= 72 on N >= 65536 nodes (WAVE16 on
 * fewer) and GROUP16 up to 144.  SPLIT takes each stencil's retained-row
 * count from the covering when handed that covering's own centers and owner
 * arrays (else it counts them, one extra pass over the stencils); the
 * weights are the same bit for bit whatever the pass width.  Batched builds
 * pass the table to their workers. */
typedef enum orbf_schedule {
  ORBF_SCHED_DEFAULT = -1,
  ORBF_SCHED_WAVE16 = 0,  /* one wavefront per stencil, 16 right-hand sides
                             per pass (K <= 72)                              */
  ORBF_SCHED_WAVE8 = 1,   /* one wavefront, 8 right-hand sides per pass
                             (K <= 72): fewer registers                      */
  ORBF_SCHED_GROUP16 = 2, /* four wavefronts on a 16 x 16 lane grid, 16
                             right-hand sides per pass (K <= 144)            */
  ORBF_SCHED_SPLIT = 3,   /* one wavefront per stencil, with 8, 16 or 24
                             right-hand sides per pass chosen per stencil
                             from its retained-row count p (p <= 8, <= 16,
                             above): stencils are sorted into three lists on
                             the device and each list is one launch
                             (K <= 72)                                       */
  ORBF_SCHED_MATRIX = 4   /* one wavefront per stencil, blocked elimination
                             whose updates run on the FP64 matrix cores,
                             16 right-hand sides per pass (32 < K <= 80)     */
} orbf_schedule;

/* Set (or with ORBF_SCHED_DEFAULT clear) the schedule of (K, pclass).
 * EINVAL if the schedule cannot serve K. */
orbf_status orbf_set_schedule(orbf_ctx* ctx, int K, int pclass,
                              orbf_schedule schedule);

/* FP32 + refinement (ORBF_PREC_FP32_IR, Sec. 4.3's one decomposition per
 * stencil done in FP32 and won back by FP64 residual corrections): the
 * number of corrections a stencil may take before it is solved again from
 * scratch in FP64 (default 8).  0 sends every stencil that the first FP32
 * solve does not settle to the FP64 kernel.  EINVAL outside 0..64.  Affects
 * later calls on this context and on its batched workers. */
orbf_status orbf_set_ir_max_corrections(orbf_ctx* ctx, int corrections);

/* Copy the table out: up to cap rows of (K, pclass, schedule) to out (host,
 * 3*cap int32); *count receives the number of rows. */
orbf_status orbf_get_schedules(orbf_ctx* ctx, int32_t* out, int cap,
                               int* count);

/* Phase timing of the most recent calls on this context, in milliseconds of
 * stream time (HIP events around each entry point's kernels): [0] kNN,
 * [1] covering, [2] weights, [3] CSR, [4] duration of the weights kernel's
 * last launch.  Valid after orbf_sync. */
orbf_status orbf_phase_times(orbf_ctx* ctx, double* ms5 /* host, 5 */);

/* Measurement helper, not a step of the method: the FP64 vector FMA rate
 * this device reaches (TFLOP/s, written to *tflops, host), from a kernel of
 * independent FMA chains at two wavefronts per SIMD, best of three timed
 * launches after one warm-up.  Blocking (synchronises the context's
 * stream); uses the context's scratch.  It is reported beside the published
 * FP64 peak that roofline fractions are taken against. */
orbf_status orbf_measure_fp64_fma(orbf_ctx* ctx, double* tflops);

/* ------------------------------------------------------------------------
 * Batched builds: many independent node sets in one call.
 * ---------------------------------------------------------------------- */

/* One node set of a batch: inputs, parameters and caller-allocated device
 * outputs (the arrays of the single-set calls above, same layouts).  Every
 * set gets the whole path: stencils, covering (with the Lebesgue test when
 * tau is finite), Laplacian rows at the eligible nodes, normal-derivative
 * rows at the boundary nodes, CSR. */
typedef struct orbf_set_desc {
  const double* xyz;        /* N*d coordinates                               */
  int64_t N;
  int d;                    /* 2 or 3                                        */
  int n;                    /* stencil size                                  */
  int m;                    /* odd PHS exponent >= 3                         */
  int l;                    /* polynomial degree (-1: none, M = 0)           */
  double delta;             /* overlap parameter in [0,1]                    */
  double tau;               /* Lebesgue threshold, INFINITY = off            */
  orbf_prec prec;
  const uint8_t* eligible;  /* N or NULL = every node gets a Laplacian row   */
  const int32_t* boundary;  /* n_boundary nodes with normal-derivative rows,
                               or NULL                                      */
  int64_t n_boundary;
  const double* normals;    /* n_boundary*d unit normals                     */
  int32_t* knn;             /* outputs: N*n                                  */
  double* rho2;             /* N                                             */
  int32_t* centers;         /* N (capacity)                                  */
  int64_t* n_centers;       /* 1                                             */
  int32_t* owner;           /* N                                             */
  double* W;                /* N*n                                           */
  double* lebesgue;         /* N or NULL                                     */
  int32_t* ir_steps;        /* N or NULL                                     */
  int64_t* row_ptr;         /* N+1                                           */
  int32_t* col;             /* N*n                                           */
  double* val;              /* N*n                                           */
} orbf_set_desc;

/* Build the DMs of `nsets` node sets.  The sets are dealt to the context's
 * worker streams (each with its own scratch), largest estimated cost first
 * to the least-loaded worker, and joined back onto the context's stream; the
 * call is asynchronous like the others.  A batch whose descriptors are
 * byte-identical to the previous call's is captured into a HIP graph on its
 * second occurrence and replayed from the third on (only when every set has
 * tau = INFINITY, whose path has no host round trip).  A set's results do
 * not depend on the other sets of the batch.
 * Errors: EINVAL naming the first bad set; device errors at orbf_sync. */
orbf_status orbf_build_dm_batched(orbf_ctx* ctx, const orbf_set_desc* sets,
                                  int nsets);

/* Number of worker streams for batched builds (1..16, default 4).  Each
 * worker holds its own scratch within the context's HBM budget divided by
 * the number of workers. */
orbf_status orbf_set_workers(orbf_ctx* ctx, int workers);

/* ------------------------------------------------------------------------
 * Serving: a request engine with continuous admission.
 * ---------------------------------------------------------------------- */

/* A server owns `slots` streams (each with its own scratch) and one arena of
 * device memory that holds the outputs of admitted requests.  Requests wait
 * in FIFO order; a request is admitted when a slot is free and its outputs
 * fit in the arena (first fit); a later, smaller request may pass a waiting
 * head at most 8 times before the head blocks admission.  Admitted requests
 * run concurrently on their slots; results stay on the device until
 * released.  Progress is driven by orbf_server_poll (no hidden threads).
 * A finished request keeps its arena memory until orbf_server_release: a
 * caller that holds every result until all requests are done can stall
 * admission once the arena is full of finished results.
 * Device memory held: arena_bytes + slots * slot_scratch_bytes. */
typedef struct orbf_server orbf_server;

typedef struct orbf_request {
  const double* xyz;   /* N*d device coordinates, caller-owned; must stay
                          valid until the request is done, and be written
                          by then: see `ready`                              */
  int64_t N;
  int d, n, m, l;
  double delta;
  double tau;          /* INFINITY = off                                     */
  orbf_prec prec;
  double t_arrival;    /* arrival time on the orbf_server_now clock          */
  void* ready;         /* hipEvent_t recorded by the caller after the work
                          that writes xyz (on any stream), or NULL.  The
                          slot's stream waits for it before the build, so
                          coordinates produced on the device just before
                          submit are read only once written.  With NULL the
                          caller guarantees that xyz is complete when the
                          request is admitted (e.g. by a stream sync before
                          submit).  The event must stay valid until the
                          request is done; the server never destroys it.    */
} orbf_request;

typedef struct orbf_result {
  int status;          /* orbf_status of the build (device errors included)  */
  int64_t N;
  int n;
  int64_t n_centers;   /* number of stencils                                 */
  double t_arrival;    /* seconds, orbf_server_now clock                     */
  double t_admit;      /* admitted to a slot                                 */
  double t_done;       /* completion observed by orbf_server_poll            */
} orbf_result;

orbf_status orbf_server_create(int device, int slots, size_t arena_bytes,
                               size_t slot_scratch_bytes, orbf_server** out);
void orbf_server_destroy(orbf_server* srv);  /* waits for running requests   */
const char* orbf_server_last_error(const orbf_server* srv);
double orbf_server_now(void);  /* steady clock, seconds                      */

/* Device bytes a request's outputs take in the arena. */
size_t orbf_request_bytes(int64_t N, int d, int n, orbf_prec prec);

/* Queue a request; *ticket identifies it.  EINVAL for bad parameters,
 * EBUDGET if it could never fit (outputs larger than the arena, or
 * orbf_workspace_size larger than slot_scratch_bytes). */
orbf_status orbf_server_submit(orbf_server* srv, const orbf_request* req,
                               uint64_t* ticket);

/* Retire finished requests and admit waiting ones.  Writes up to `cap`
 * tickets finished since the previous call to done[] (host array) and their
 * number to *n_done. */
orbf_status orbf_server_poll(orbf_server* srv, uint64_t* done, int cap,
                             int* n_done);

/* Status and timing of a finished request (EINVAL if unknown or not done).
 * n_centers is 0 for a request whose build failed before its covering ran
 * (the status says why). */
orbf_status orbf_server_result(orbf_server* srv, uint64_t ticket,
                               orbf_result* out);

/* Copy a finished request's outputs into caller device buffers: the output
 * fields of `dst` (knn, rho2, centers, n_centers, owner, W, lebesgue,
 * ir_steps, row_ptr, col, val; NULL fields are skipped).  Synchronous: the
 * copies are complete when it returns.  They are not ordered after work
 * pending on the caller's streams, so no such work may still use the
 * destination buffers (a fresh allocation after a sync of its stream). */
orbf_status orbf_server_fetch(orbf_server* srv, uint64_t ticket,
                              const orbf_set_desc* dst);

/* Free a finished request's arena memory; its ticket becomes unknown. */
orbf_status orbf_server_release(orbf_server* srv, uint64_t ticket);

/* [0] waiting, [1] running, [2] finished and not released, [3] arena bytes
 * in use, [4] arena bytes in total. */
orbf_status orbf_server_stats(orbf_server* srv, int64_t out5[5]);

#ifdef __cplusplus
}
#endif
#endif /* ORBF_H */
