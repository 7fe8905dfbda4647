// C ABI of liborbf: contexts, argument checking, scratch management, phase
// timing and the device status word.  The numerical work is in knn.hip,
// cover.hip, weights.hip and csr.hip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>

#include "orbf_internal.hpp"

namespace orbf {

orbf_status fail(orbf_ctx* ctx, orbf_status code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

orbf_status hip_check(orbf_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return ORBF_OK;
  return fail(ctx, ORBF_EHIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

// Grow-only scratch buffer `id`.  A larger request frees the old buffer;
// hipFree waits for the device, so kernels still using it have finished.
void* scratch(orbf_ctx* ctx, int id, size_t bytes, orbf_status* st) {
  if (*st != ORBF_OK) return nullptr;
  Buffer& b = ctx->buf[id];
  if (bytes == 0) bytes = 8;
  if (b.bytes >= bytes) return b.ptr;
  size_t want = bytes + bytes / 8 + 256;
  if (ctx->budget && ctx->held - b.bytes + want > ctx->budget) {
    *st = fail(ctx, ORBF_EBUDGET,
               "scratch of " + std::to_string(want) +
                   " bytes exceeds the context's HBM budget");
    return nullptr;
  }
  if (b.ptr) {
    hipFree(b.ptr);
    ctx->held -= b.bytes;
    b.ptr = nullptr;
    b.bytes = 0;
  }
  if (hipMalloc(&b.ptr, want) != hipSuccess) {
    b.ptr = nullptr;
    *st = fail(ctx, ORBF_ENOMEM, "hipMalloc of " + std::to_string(want) +
                                     " bytes of scratch failed");
    return nullptr;
  }
  b.bytes = want;
  ctx->held += want;
  return b.ptr;
}

// Free every scratch buffer of an idle context (hipFree waits for the
// device).  Grow-only buffers keep the largest size each id has seen over
// many builds, which can exceed what any one build needs.
void release_scratch(orbf_ctx* ctx) {
  for (auto& b : ctx->buf) {
    if (b.ptr) hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
  }
  ctx->held = 0;
  ctx->d2_cache = D2Cache();
  ctx->p_cache = PCache();
}

int schedule_for(const orbf_ctx* ctx, int K, int pclass) {
  for (size_t i = 0; i + 2 < ctx->schedules.size(); i += 3)
    if (ctx->schedules[i] == K && ctx->schedules[i + 1] == pclass)
      return ctx->schedules[i + 2];
  return ORBF_SCHED_DEFAULT;
}

static int num_monomials(int d, int l) {
  long num = 1, den = 1;
  for (int i = 1; i <= d; ++i) {
    num *= (l + i);
    den *= i;
  }
  return (int)(num / den);
}

}  // namespace orbf

using namespace orbf;

namespace {

const char* status_name(int c) {
  switch (c) {
    case ORBF_OK: return "OK";
    case ORBF_EINVAL: return "EINVAL";
    case ORBF_EDUPLICATE: return "EDUPLICATE";
    case ORBF_ESINGULAR: return "ESINGULAR";
    case ORBF_ENOMEM: return "ENOMEM";
    case ORBF_EBUDGET: return "EBUDGET";
    case ORBF_EHIP: return "EHIP";
    default: return "EINTERNAL";
  }
}

orbf_status check_common(orbf_ctx* ctx, int64_t N, int d, int n) {
  if (!ctx) return ORBF_EINVAL;
  if (d != 2 && d != 3) return fail(ctx, ORBF_EINVAL, "d must be 2 or 3");
  if (N < 1 || N > INT32_MAX) return fail(ctx, ORBF_EINVAL, "N out of range");
  if (n < 1 || n > N) return fail(ctx, ORBF_EINVAL, "need 1 <= n <= N");
  if (n > 128) return fail(ctx, ORBF_EINVAL, "stencil size n > 128");
  return ORBF_OK;
}

struct PhaseTimer {
  orbf_ctx* ctx;
  int slot;
  PhaseTimer(orbf_ctx* c, int s) : ctx(c), slot(s) {
    if (ctx->timing) hipEventRecord(ctx->ev[2 * s], ctx->stream);
  }
  ~PhaseTimer() {
    if (!ctx->timing) return;
    hipEventRecord(ctx->ev[2 * slot + 1], ctx->stream);
    ctx->phase_valid[slot] = true;
  }
};

}  // namespace

extern "C" {

orbf_status orbf_create(int device, void* hip_stream, size_t hbm_budget_bytes,
                        orbf_ctx** out) {
  if (!out) return ORBF_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return ORBF_EHIP;
  orbf_ctx* ctx = new (std::nothrow) orbf_ctx();
  if (!ctx) return ORBF_ENOMEM;
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->budget = hbm_budget_bytes;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess)
    ctx->num_cus = prop.multiProcessorCount;
  if (hipMalloc(&ctx->status, sizeof(DevStatus)) != hipSuccess ||
      hipHostMalloc((void**)&ctx->status_host, sizeof(DevStatus),
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&ctx->host_counter, sizeof(int64_t),
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&ctx->host_scalars, 128 * sizeof(double),
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&ctx->cover_extra_host, sizeof(int64_t),
                    hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->cover_ev, hipEventDisableTiming) !=
          hipSuccess) {
    delete ctx;
    return ORBF_ENOMEM;
  }
  hipMemset(ctx->status, 0, sizeof(DevStatus));
  for (auto& e : ctx->ev) hipEventCreate(&e);
  // the allocation-free CSR entry point's scratch on this device
  if (csr_noalloc_setup(ctx) != ORBF_OK) {
    const orbf_status st = ORBF_EHIP;
    orbf_destroy(ctx);
    return st;
  }
  *out = ctx;
  return ORBF_OK;
}

void orbf_destroy(orbf_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  for (orbf_ctx* w : ctx->workers) orbf_destroy(w);
  for (hipEvent_t e : ctx->join_ev) hipEventDestroy(e);
  if (ctx->fork_ev) hipEventDestroy(ctx->fork_ev);
  drop_graph(ctx);
  if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
  for (auto& b : ctx->buf)
    if (b.ptr) hipFree(b.ptr);
  if (ctx->status) hipFree(ctx->status);
  if (ctx->status_host) hipHostFree(ctx->status_host);
  if (ctx->host_counter) hipHostFree(ctx->host_counter);
  if (ctx->host_scalars) hipHostFree(ctx->host_scalars);
  if (ctx->cover_extra_host) hipHostFree(ctx->cover_extra_host);
  if (ctx->cover_ev) hipEventDestroy(ctx->cover_ev);
  if (ctx->cover_tab_host) hipHostFree(ctx->cover_tab_host);
  for (auto& e : ctx->ev)
    if (e) hipEventDestroy(e);
  if (ctx->owns_stream && ctx->stream) hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char* orbf_last_error(const orbf_ctx* ctx) {
  return ctx ? ctx->err.c_str() : "no context";
}

orbf_status orbf_sync(orbf_ctx* ctx) {
  if (!ctx) return ORBF_EINVAL;
  hipSetDevice(ctx->device);
  hipError_t e = hipMemcpyAsync(ctx->status_host, ctx->status,
                                sizeof(DevStatus), hipMemcpyDeviceToHost,
                                ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_check(ctx, e, "sync");
  // batched builds: the workers' status words (their streams joined ours)
  for (orbf_ctx* w : ctx->workers) {
    const orbf_status ws = orbf_sync(w);
    if (ws != ORBF_OK) {
      ctx->err = "batch worker: " + w->err;
      return ws;
    }
  }
  const DevStatus s = *ctx->status_host;
  if (s.code == 0) return ORBF_OK;
  hipMemsetAsync(ctx->status, 0, sizeof(DevStatus), ctx->stream);
  hipStreamSynchronize(ctx->stream);
  char msg[160];
  snprintf(msg, sizeof msg, "device reported %s at node/stencil %d",
           status_name(s.code), s.where);
  ctx->err = msg;
  return (orbf_status)s.code;
}

size_t orbf_workspace_size(int64_t N, int d, int n, int l, orbf_prec prec) {
  (void)l;
  (void)prec;
  if (N < 1 || n < 1 || (d != 2 && d != 3)) return 0;
  // Every scratch buffer is grow-only and rounded up by scratch(); the sum
  // over buffer ids of the largest request each id sees in a build bounds
  // what a context holds (kNN, covering with or without the Lebesgue test,
  // weights in either precision, CSR, Gershgorin disks, implicit solve).
  auto want = [](size_t b) { return (b ? b : 8) + (b ? b : 8) / 8 + 256; };
  const size_t Nn = (size_t)N;
  size_t t = 0;
  t += want(sizeof(GridParams));        // B_GRID_PARAMS
  t += want(1024 * 6 * 8);              // B_PARTIAL
  t += want(Nn * 4) * 2;                // B_CELL_OF, B_CELL_RANK
  t += want((Nn + 65) * 4);             // B_FLAGS (cell counts, flags)
  t += want((Nn + 66) * 8);             // B_CELL_START
  t += want(Nn * 4);                    // B_PERM
  t += want(Nn * (size_t)d * 8);        // B_XS
  t += want(Nn * 16);                   // B_BALL
  t += want((Nn + 1) * 4) * 3;          // B_INDEG, B_PRED_FILL, B_ROWPTR_TMP
  t += want((Nn + 2) * 8);              // B_CENTER_POS
  t += want(Nn * 4);                    // B_STATE
  t += want((Nn + 1) * 12);             // B_PRED (Lebesgue level lists)
  t += want(Nn * 16);                   // B_W_TMP (Lebesgue covering)
  t += want(64) + want(8);              // B_MISC2, B_MISC
  t += want(scan_tmp_elems((int64_t)Nn + 66) * 8);  // B_SCAN_TMP
  t += want(Nn * 4) + want(8);          // B_IR_FALLBACK, B_IR_COUNT
  t += want(Nn * (size_t)n * 8);        // B_KNN_D2
  t += want(Nn * (size_t)n);            // B_CSR_RANK
  t += want(Nn * 12) + want(24);        // B_CLASS, B_CLASS_N
  t += want(Nn * 4);                    // B_P_CACHE
  t += want(gershgorin_scratch_bytes()); // B_GERSH
  t += want(krylov_scratch_bytes(N, 0));  // B_KRYLOV (BiCGSTAB)
  return t;
}

orbf_status orbf_build_nodes_knn(orbf_ctx* ctx, const double* xyz, int64_t N,
                                 int d, int n, int32_t* knn, double* rho2) {
  orbf_status st = check_common(ctx, N, d, n);
  if (st) return st;
  if (!xyz || !knn || !rho2) return fail(ctx, ORBF_EINVAL, "NULL pointer");
  hipSetDevice(ctx->device);
  PhaseTimer t(ctx, 0);
  return launch_knn(ctx, xyz, N, d, n, knn, rho2);
}

orbf_status orbf_select_overlapped_stencils(
    orbf_ctx* ctx, const double* xyz, const int32_t* knn, const double* rho2,
    int64_t N, int d, int n, double delta, const uint8_t* eligible,
    int32_t* centers, int64_t* n_centers, int32_t* owner, int32_t* p) {
  orbf_status st = check_common(ctx, N, d, n);
  if (st) return st;
  if (!(delta >= 0.0 && delta <= 1.0))
    return fail(ctx, ORBF_EINVAL, "delta must lie in [0, 1]");
  if (!xyz || !knn || !rho2 || !centers || !n_centers || !owner)
    return fail(ctx, ORBF_EINVAL, "NULL pointer");
  hipSetDevice(ctx->device);
  const double t = 1.0 - delta;
  const double t2 = t * t;
  PhaseTimer tm(ctx, 1);
  return launch_cover(ctx, xyz, knn, rho2, N, d, n, t2, eligible, centers,
                      n_centers, owner, p);
}

orbf_status orbf_compute_weights(orbf_ctx* ctx, orbf_op op, int m, int l,
                                 int n, double delta,
                                 const orbf_weights_args* a) {
  if (!ctx || !a) return ORBF_EINVAL;
  orbf_status st = check_common(ctx, a->N, a->d, n);
  if (st) return st;
  if (op < ORBF_OP_LAPLACIAN || op > ORBF_OP_IDENTITY)
    return fail(ctx, ORBF_EINVAL, "unknown operator");
  if (op == ORBF_OP_DZ && a->d != 3)
    return fail(ctx, ORBF_EINVAL, "d/dz needs d = 3");
  if (m < 3 || m % 2 == 0)
    return fail(ctx, ORBF_EINVAL, "PHS exponent m must be odd and >= 3");
  // l = -1: no polynomial augmentation (M = 0, K = n), the unaugmented
  // RBF-FD of Sec. 4.3's count
  if (l < -1) return fail(ctx, ORBF_EINVAL, "polynomial degree l < -1");
  const int M = num_monomials(a->d, l);
  if (n < M) return fail(ctx, ORBF_EINVAL, "stencil size n < C(l+d, d)");
  if (n + M > 144) return fail(ctx, ORBF_EINVAL, "n + M > 144");
  if (!(delta >= 0.0 && delta <= 1.0))
    return fail(ctx, ORBF_EINVAL, "delta must lie in [0, 1]");
  if (!(a->tau >= 1.0)) return fail(ctx, ORBF_EINVAL, "tau must be >= 1");
  if (a->tau_mode != 0 && a->tau_mode != 1)
    return fail(ctx, ORBF_EINVAL, "tau_mode must be 0 or 1");
  if (!a->xyz || !a->knn || !a->rho2 || !a->W)
    return fail(ctx, ORBF_EINVAL, "NULL pointer");
  if (a->prec != ORBF_PREC_FP64 && a->prec != ORBF_PREC_FP32_IR)
    return fail(ctx, ORBF_EINVAL, "unknown precision");
  const bool explicit_rows = a->rows != nullptr;
  if (explicit_rows) {
    if (a->n_rows < 0) return fail(ctx, ORBF_EINVAL, "n_rows < 0");
    if (op == ORBF_OP_NEUMANN && !a->normals)
      return fail(ctx, ORBF_EINVAL, "NEUMANN rows need normals");
  } else {
    if (op == ORBF_OP_NEUMANN)
      return fail(ctx, ORBF_EINVAL,
                  "normal-derivative rows need normals: list them explicitly");
    if (op != ORBF_OP_LAPLACIAN && !isinf(a->tau))
      return fail(ctx, ORBF_EINVAL,
                  "the Lebesgue test (finite tau) is for the Laplacian");
    if (!a->centers || !a->n_centers || !a->owner)
      return fail(ctx, ORBF_EINVAL, "NULL covering pointer");
  }
  hipSetDevice(ctx->device);
  const double t = 1.0 - delta;
  PhaseTimer tm(ctx, 2);
  return launch_weights(ctx, op, m, l, n, t * t, a);
}

orbf_status orbf_assemble_csr(orbf_ctx* ctx, int64_t N, int n,
                              const int32_t* knn, const int32_t* owner,
                              const double* W, int64_t* row_ptr, int32_t* col,
                              double* val) {
  if (!ctx) return ORBF_EINVAL;
  if (N < 1 || N > INT32_MAX || n < 1 || n > 128)
    return fail(ctx, ORBF_EINVAL, "N or n out of range");
  if (!knn || !owner || !W || !row_ptr || !col || !val)
    return fail(ctx, ORBF_EINVAL, "NULL pointer");
  hipSetDevice(ctx->device);
  PhaseTimer tm(ctx, 3);
  return launch_csr(ctx, N, n, knn, owner, W, row_ptr, col, val);
}

orbf_status orbf_assemble_csr_noalloc(orbf_ctx* ctx, int64_t N, int n,
                                      const int32_t* knn,
                                      const int32_t* owner, const double* W,
                                      int64_t* row_ptr, int32_t* col,
                                      double* val) {
  if (!ctx) return ORBF_EINVAL;
  if (N < 1 || N > INT32_MAX || n < 1 || n > 128)
    return fail(ctx, ORBF_EINVAL, "N or n out of range");
  if (!knn || !owner || !W || !row_ptr || !col || !val)
    return fail(ctx, ORBF_EINVAL, "NULL pointer");
  hipSetDevice(ctx->device);
  PhaseTimer tm(ctx, 3);
  return launch_csr_noalloc(ctx, N, n, knn, owner, W, row_ptr, col, val);
}

orbf_status orbf_spmv(orbf_ctx* ctx, int64_t N, const int64_t* row_ptr,
                      const int32_t* col, const double* val, const double* x,
                      double* y) {
  if (!ctx) return ORBF_EINVAL;
  if (N < 1 || N > INT32_MAX) return fail(ctx, ORBF_EINVAL, "N out of range");
  if (!row_ptr || !col || !val || !x || !y)
    return fail(ctx, ORBF_EINVAL, "NULL pointer");
  if (x == y) return fail(ctx, ORBF_EINVAL, "x and y must not alias");
  hipSetDevice(ctx->device);
  return launch_spmv(ctx, N, row_ptr, col, val, x, y);
}

orbf_status orbf_gershgorin(orbf_ctx* ctx, int64_t N, const int64_t* row_ptr,
                            const int32_t* col, const double* val,
                            double* diag, double* radius, double* summary) {
  if (!ctx) return ORBF_EINVAL;
  if (N < 1 || N > INT32_MAX) return fail(ctx, ORBF_EINVAL, "N out of range");
  if (!row_ptr || !col || !val || !summary)
    return fail(ctx, ORBF_EINVAL, "NULL pointer");
  hipSetDevice(ctx->device);
  return launch_gershgorin(ctx, N, row_ptr, col, val, diag, radius, summary);
}

orbf_status orbf_solve_implicit(orbf_ctx* ctx, int64_t N,
                                const int64_t* row_ptr, const int32_t* col,
                                const double* val, const uint8_t* row_kind,
                                double alpha, double beta, const double* b,
                                double* x, double tol, int max_iter,
                                int precond, int* iters, double* relres) {
  if (!ctx) return ORBF_EINVAL;
  if (N < 1 || N > INT32_MAX) return fail(ctx, ORBF_EINVAL, "N out of range");
  if (!row_ptr || !col || !val || !b || !x)
    return fail(ctx, ORBF_EINVAL, "NULL pointer");
  if (b == x) return fail(ctx, ORBF_EINVAL, "b and x must not alias");
  if (!(tol >= 0.0) || max_iter < 0)
    return fail(ctx, ORBF_EINVAL, "tol >= 0 and max_iter >= 0 required");
  if (!isfinite(alpha) || !isfinite(beta))
    return fail(ctx, ORBF_EINVAL, "alpha and beta must be finite");
  if (precond != ORBF_PRECOND_NONE && precond != ORBF_PRECOND_JACOBI)
    return fail(ctx, ORBF_EINVAL, "unknown preconditioner");
  hipSetDevice(ctx->device);
  return launch_solve_implicit(ctx, N, row_ptr, col, val, row_kind, alpha,
                               beta, b, x, tol, max_iter, precond, nullptr, 0,
                               0, iters, relres);
}

orbf_status orbf_implicit_ilu0(orbf_ctx* ctx, int64_t N,
                               const int64_t* row_ptr, const int32_t* col,
                               const double* val, const uint8_t* row_kind,
                               double alpha, double beta, double* lu) {
  if (!ctx) return ORBF_EINVAL;
  if (N < 1 || N > INT32_MAX) return fail(ctx, ORBF_EINVAL, "N out of range");
  if (!row_ptr || !col || !val || !lu)
    return fail(ctx, ORBF_EINVAL, "NULL pointer");
  if (lu == val) return fail(ctx, ORBF_EINVAL, "lu and val must not alias");
  if (!isfinite(alpha) || !isfinite(beta))
    return fail(ctx, ORBF_EINVAL, "alpha and beta must be finite");
  hipSetDevice(ctx->device);
  return launch_ilu0(ctx, N, row_ptr, col, val, row_kind, alpha, beta, lu);
}

orbf_status orbf_solve_implicit_krylov(
    orbf_ctx* ctx, int64_t N, const int64_t* row_ptr, const int32_t* col,
    const double* val, const uint8_t* row_kind, double alpha, double beta,
    const double* b, double* x, double tol, int max_iter, int method,
    int restart, int precond, const double* lu, int* iters, double* relres) {
  if (!ctx) return ORBF_EINVAL;
  if (N < 1 || N > INT32_MAX) return fail(ctx, ORBF_EINVAL, "N out of range");
  if (!row_ptr || !col || !val || !b || !x)
    return fail(ctx, ORBF_EINVAL, "NULL pointer");
  if (b == x) return fail(ctx, ORBF_EINVAL, "b and x must not alias");
  if (!(tol >= 0.0) || max_iter < 0)
    return fail(ctx, ORBF_EINVAL, "tol >= 0 and max_iter >= 0 required");
  if (!isfinite(alpha) || !isfinite(beta))
    return fail(ctx, ORBF_EINVAL, "alpha and beta must be finite");
  if (method != ORBF_KRYLOV_BICGSTAB && method != ORBF_KRYLOV_GMRES)
    return fail(ctx, ORBF_EINVAL, "unknown Krylov method");
  if (method == ORBF_KRYLOV_GMRES && (restart < 1 || restart > 64))
    return fail(ctx, ORBF_EINVAL, "GMRES restart must be in 1..64");
  if (precond != ORBF_PRECOND_NONE && precond != ORBF_PRECOND_JACOBI &&
      precond != ORBF_PRECOND_ILU0)
    return fail(ctx, ORBF_EINVAL, "unknown preconditioner");
  if (precond == ORBF_PRECOND_ILU0 && !lu)
    return fail(ctx, ORBF_EINVAL, "ILU(0) preconditioning needs lu");
  hipSetDevice(ctx->device);
  return launch_solve_implicit(ctx, N, row_ptr, col, val, row_kind, alpha,
                               beta, b, x, tol, max_iter, precond, lu, method,
                               restart, iters, relres);
}

orbf_status orbf_bdf_coefficients(int order, double* a, double* b) {
  if (order < 1 || order > 4 || !a || !b) return ORBF_EINVAL;
  bdf_coefficients(order, a, b);
  return ORBF_OK;
}

orbf_status orbf_bdf_rhs(orbf_ctx* ctx, int64_t N, int order,
                         const double* u0, const double* u1,
                         const double* u2, const double* u3, const double* f,
                         double dt, const uint8_t* row_kind,
                         const double* bvals, double* rhs) {
  if (!ctx) return ORBF_EINVAL;
  if (N < 1 || N > INT32_MAX) return fail(ctx, ORBF_EINVAL, "N out of range");
  if (order < 1 || order > 4)
    return fail(ctx, ORBF_EINVAL, "BDF order must be 1..4");
  const double* u[4] = {u0, u1, u2, u3};
  for (int i = 0; i < order; ++i)
    if (!u[i]) return fail(ctx, ORBF_EINVAL, "NULL time level");
  if (!rhs) return fail(ctx, ORBF_EINVAL, "NULL pointer");
  for (int i = 0; i < order; ++i)
    if (u[i] == rhs) return fail(ctx, ORBF_EINVAL, "rhs aliases a time level");
  if (!isfinite(dt) || dt <= 0.0)
    return fail(ctx, ORBF_EINVAL, "dt must be finite and positive");
  hipSetDevice(ctx->device);
  return launch_bdf_rhs(ctx, N, order, u, f, dt, row_kind, bvals, rhs);
}

orbf_status orbf_set_ir_max_corrections(orbf_ctx* ctx, int corrections) {
  if (!ctx) return ORBF_EINVAL;
  if (corrections < 0 || corrections > 64)
    return fail(ctx, ORBF_EINVAL, "ir_max_corrections: 0..64");
  ctx->ir_max_corrections = corrections;
  drop_graph(ctx);
  return ORBF_OK;
}

orbf_status orbf_set_schedule(orbf_ctx* ctx, int K, int pclass,
                              orbf_schedule schedule) {
  if (!ctx) return ORBF_EINVAL;
  if (K < 1 || K > 144 || pclass < 0 || pclass > 1)
    return fail(ctx, ORBF_EINVAL, "schedule: K in 1..144, pclass 0 or 1");
  if ((schedule == ORBF_SCHED_WAVE16 || schedule == ORBF_SCHED_WAVE8 ||
       schedule == ORBF_SCHED_SPLIT) &&
      K > 72)
    return fail(ctx, ORBF_EINVAL, "one-wavefront schedules need K <= 72");
  if (schedule == ORBF_SCHED_GROUP16 && K > 144)
    return fail(ctx, ORBF_EINVAL, "the workgroup schedule needs K <= 144");
  if (schedule == ORBF_SCHED_MATRIX && (K <= 32 || K > 80))
    return fail(ctx, ORBF_EINVAL, "the matrix-core schedule needs 32 < K <= 80");
  if (schedule < ORBF_SCHED_DEFAULT || schedule > ORBF_SCHED_MATRIX)
    return fail(ctx, ORBF_EINVAL, "unknown schedule");
  auto& t = ctx->schedules;
  for (size_t i = 0; i + 2 < t.size(); i += 3)
    if (t[i] == K && t[i + 1] == pclass) {
      t.erase(t.begin() + i, t.begin() + i + 3);
      break;
    }
  if (schedule != ORBF_SCHED_DEFAULT) t.insert(t.end(), {K, pclass, schedule});
  drop_graph(ctx);
  return ORBF_OK;
}

orbf_status orbf_get_schedules(orbf_ctx* ctx, int32_t* out, int cap,
                               int* count) {
  if (!ctx || !count || (cap > 0 && !out)) return ORBF_EINVAL;
  const int rows = (int)(ctx->schedules.size() / 3);
  for (int i = 0; i < rows && i < cap; ++i)
    for (int k = 0; k < 3; ++k) out[3 * i + k] = ctx->schedules[3 * i + k];
  *count = rows;
  return ORBF_OK;
}

orbf_status orbf_phase_times(orbf_ctx* ctx, double* ms5) {
  if (!ctx || !ms5) return ORBF_EINVAL;
  for (int s = 0; s < 5; ++s) {
    ms5[s] = -1.0;
    if (!ctx->phase_valid[s]) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[2 * s], ctx->ev[2 * s + 1]) ==
        hipSuccess)
      ms5[s] = ms;
  }
  return ORBF_OK;
}

}  // extern "C"
