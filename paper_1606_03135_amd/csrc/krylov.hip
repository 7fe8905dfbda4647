// Implicit time step with the DM (Sec. 5): solve A x = b where, for a DM L
// in CSR, row e of A is chosen by row_kind[e]:
//   1 (interior): alpha x_e + beta (L x)_e
//   0 (Dirichlet): x_e
//   2 (boundary operator): (L x)_e, e.g. a normal-derivative row
// With alpha = 1 and beta = -nu dt this is the backward-Euler system of
// Sec. 5 (BDF4 takes beta = -(12/25) nu dt): interior rows of I - nu dt L,
// boundary rows that impose the boundary condition.
//
// Two Krylov methods, each unpreconditioned or right-preconditioned
// (A M^-1 y = b, x = M^-1 y) with Jacobi (M = diag A) or with the ILU(0)
// factors of A (ilu.hip), which is what Secs. 7.1 and 7.2 use:
//   - BiCGSTAB (van der Vorst, 1992);
//   - GMRES(m) with classical Gram-Schmidt applied twice, Givens rotations
//     on the host and restarts after m steps.
// A normal-derivative row scales like 1/h and an interior row like
// 1 + dt |L_ee|: on Neumann steps Jacobi cuts the iterations 2-3x, on
// Dirichlet and all-interior steps it costs iterations (disk at dt = 1e-2:
// 75 -> 98; the 1M-node ball step: 7 -> 12), so the caller chooses.
// Products with A use sixteen lanes per row; every inner product is summed
// in a fixed order (per-block partials, then one wavefront), so a solve is
// deterministic.  The host drives the iteration and reads the inner
// products back through pinned memory: four times per BiCGSTAB iteration,
// once per GMRES step (the Gram-Schmidt coefficients stay on the device).
#include <algorithm>
#include <vector>

#include "orbf_internal.hpp"

namespace orbf {

namespace {

constexpr int kDotBlocks = 1024;
constexpr int kMaxRestart = 64;  // GMRES(m): m <= 64

__global__ __launch_bounds__(256) void apply_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const uint8_t* __restrict__ row_kind,
    double alpha, double beta, const double* __restrict__ x, int64_t N,
    double* __restrict__ y) {
  const int pl = threadIdx.x & 15;
  for (int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4; e < N;
       e += (int64_t)gridDim.x * 16) {
    const int kind = row_kind ? row_kind[e] : 1;
    double acc = 0.0;
    if (kind != 0) {
      const int64_t s0 = row_ptr[e], s1 = row_ptr[e + 1];
      for (int64_t t = s0 + pl; t < s1; t += 16)
        acc = fma(val[t], x[col[t]], acc);
    }
    for (int o = 1; o < 16; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (pl == 0)
      y[e] = kind == 1 ? fma(beta, acc, alpha * x[e]) : kind == 0 ? x[e] : acc;
  }
}

// partials of a.b and (if c) c.d, one pair per block
__global__ __launch_bounds__(256) void dot2_kernel(
    const double* __restrict__ a, const double* __restrict__ b,
    const double* __restrict__ c, const double* __restrict__ d, int64_t N,
    double* __restrict__ part) {
  __shared__ double s1[4], s2[4];
  double u = 0.0, w = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    u = fma(a[i], b[i], u);
    if (c) w = fma(c[i], d[i], w);
  }
  for (int o = 32; o >= 1; o >>= 1) {
    u += __shfl_xor(u, o, 64);
    w += __shfl_xor(w, o, 64);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s1[wv] = u;
    s2[wv] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ((s1[0] + s1[1]) + s1[2]) + s1[3];
    part[2 * blockIdx.x + 1] = ((s2[0] + s2[1]) + s2[2]) + s2[3];
  }
}

__global__ __launch_bounds__(64) void dot2_final_kernel(
    const double* __restrict__ part, int nparts, double* __restrict__ out) {
  double u = 0.0, w = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 64) {
    u += part[2 * i];
    w += part[2 * i + 1];
  }
  for (int o = 32; o >= 1; o >>= 1) {
    u += __shfl_xor(u, o, 64);
    w += __shfl_xor(w, o, 64);
  }
  if (threadIdx.x == 0) {
    out[0] = u;
    out[1] = w;
  }
}

// dinv[e] = 1 / diag(A)_e (1 where that is zero), sixteen lanes per row:
// alpha + beta L_ee on interior rows, 1 on Dirichlet rows, L_ee elsewhere
__global__ __launch_bounds__(256) void jacobi_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const uint8_t* __restrict__ row_kind,
    double alpha, double beta, int64_t N, double* __restrict__ dinv) {
  const int pl = threadIdx.x & 15;
  for (int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4; e < N;
       e += (int64_t)gridDim.x * 16) {
    const int kind = row_kind ? row_kind[e] : 1;
    double dg = 0.0;
    if (kind != 0)
      for (int64_t t = row_ptr[e] + pl; t < row_ptr[e + 1]; t += 16)
        if (col[t] == e) dg = val[t];
    for (int o = 1; o < 16; o <<= 1) dg += __shfl_xor(dg, o, 64);
    if (pl == 0) {
      const double a = kind == 1 ? fma(beta, dg, alpha) : kind == 0 ? 1.0 : dg;
      dinv[e] = a != 0.0 ? 1.0 / a : 1.0;
    }
  }
}

// out = dinv * in
__global__ __launch_bounds__(256) void scale_kernel(
    const double* __restrict__ dinv, const double* __restrict__ in, int64_t N,
    double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256)
    out[i] = dinv[i] * in[i];
}

// r = b - y, rh = r, p = v = 0
__global__ __launch_bounds__(256) void bicg_init_kernel(
    const double* __restrict__ b, const double* __restrict__ y, int64_t N,
    double* __restrict__ r, double* __restrict__ rh, double* __restrict__ p,
    double* __restrict__ v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    const double ri = b[i] - y[i];
    r[i] = ri;
    rh[i] = ri;
    p[i] = 0.0;
    v[i] = 0.0;
  }
}

// p = r + bt (p - om v)
__global__ __launch_bounds__(256) void bicg_p_kernel(
    const double* __restrict__ r, const double* __restrict__ v, double bt,
    double om, int64_t N, double* __restrict__ p) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256)
    p[i] = r[i] + bt * (p[i] - om * v[i]);
}

// s = r - al v
__global__ __launch_bounds__(256) void bicg_s_kernel(
    const double* __restrict__ r, const double* __restrict__ v, double al,
    int64_t N, double* __restrict__ s) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256)
    s[i] = r[i] - al * v[i];
}

// x += al ph + om sh;  r = s - om t  (r NULL: x += al ph only)
__global__ __launch_bounds__(256) void bicg_x_kernel(
    const double* __restrict__ ph, const double* __restrict__ sh,
    const double* __restrict__ t, double al, double om, int64_t N,
    double* __restrict__ x, double* __restrict__ r,
    const double* __restrict__ s) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    x[i] += r ? al * ph[i] + om * sh[i] : al * ph[i];
    if (r) r[i] = s[i] - om * t[i];
  }
}

// Right-hand side of one BDF-k step (k = 1..4): on interior rows
// sum_i a_i u_i + b_k dt f, u_0 the newest level; elsewhere the boundary
// value (0 if none is given).
__global__ __launch_bounds__(256) void bdf_rhs_kernel(
    int64_t N, int k, const double* __restrict__ u0,
    const double* __restrict__ u1, const double* __restrict__ u2,
    const double* __restrict__ u3, double a0, double a1, double a2, double a3,
    const double* __restrict__ f, double cf, const uint8_t* __restrict__ kind,
    const double* __restrict__ bvals, double* __restrict__ rhs) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N;
       e += (int64_t)gridDim.x * 256) {
    if (kind && kind[e] != 1) {
      rhs[e] = bvals ? bvals[e] : 0.0;
      continue;
    }
    double v = a0 * u0[e];
    if (k > 1) v = fma(a1, u1[e], v);
    if (k > 2) v = fma(a2, u2[e], v);
    if (k > 3) v = fma(a3, u3[e], v);
    if (f) v = fma(cf, f[e], v);
    rhs[e] = v;
  }
}

// per-block partials of v_i . w for the k vectors v_i = V + i N
__global__ __launch_bounds__(256) void mdot_kernel(
    const double* __restrict__ V, int k, const double* __restrict__ w,
    int64_t N, double* __restrict__ part) {
  __shared__ double s[4][kMaxRestart + 1];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = 0; i < k; ++i) {
    const double* v = V + (int64_t)i * N;
    double u = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < N;
         t += (int64_t)gridDim.x * 256)
      u = fma(v[t], w[t], u);
    for (int o = 32; o >= 1; o >>= 1) u += __shfl_xor(u, o, 64);
    if (lane == 0) s[wv][i] = u;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += 256)
    part[(int64_t)blockIdx.x * (kMaxRestart + 1) + i] =
        ((s[0][i] + s[1][i]) + s[2][i]) + s[3][i];
}

// out[i] = sum over blocks of part[b][i], i < k, in a fixed order
__global__ __launch_bounds__(64) void mdot_final_kernel(
    const double* __restrict__ part, int nparts, int k,
    double* __restrict__ out) {
  for (int i = 0; i < k; ++i) {
    double u = 0.0;
    for (int b = threadIdx.x; b < nparts; b += 64)
      u += part[(int64_t)b * (kMaxRestart + 1) + i];
    for (int o = 32; o >= 1; o >>= 1) u += __shfl_xor(u, o, 64);
    if (threadIdx.x == 0) out[i] = u;
  }
}

// w -= sum_i h[i] v_i with h on the device; acc[i] += h[i] (one thread)
__global__ __launch_bounds__(256) void msub_kernel(
    const double* __restrict__ V, int k, const double* __restrict__ h,
    int64_t N, double* __restrict__ w, double* __restrict__ acc) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < N;
       t += (int64_t)gridDim.x * 256) {
    double v = w[t];
    for (int i = 0; i < k; ++i) v = fma(-h[i], V[(int64_t)i * N + t], v);
    w[t] = v;
  }
  if (acc && blockIdx.x == 0)
    for (int i = threadIdx.x; i < k; i += 256) acc[i] += h[i];
}

struct Coeffs {
  double c[kMaxRestart];
};

// h[0..k) = 0
__global__ void lround_zero(double* h, int k) {
  for (int i = threadIdx.x; i < k; i += 64) h[i] = 0.0;
}

// out = s * in
__global__ __launch_bounds__(256) void vscale_kernel(
    const double* __restrict__ in, double sc, int64_t N,
    double* __restrict__ out) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < N;
       t += (int64_t)gridDim.x * 256)
    out[t] = sc * in[t];
}

// out = sum_i y_i v_i
__global__ __launch_bounds__(256) void lincomb_kernel(
    const double* __restrict__ V, int k, Coeffs y, int64_t N,
    double* __restrict__ out) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < N;
       t += (int64_t)gridDim.x * 256) {
    double v = 0.0;
    for (int i = 0; i < k; ++i) v = fma(y.c[i], V[(int64_t)i * N + t], v);
    out[t] = v;
  }
}

// x += z; r = b - y
__global__ __launch_bounds__(256) void xadd_res_kernel(
    const double* __restrict__ z, const double* __restrict__ b,
    const double* __restrict__ y, int64_t N, double* __restrict__ x,
    double* __restrict__ r) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < N;
       t += (int64_t)gridDim.x * 256) {
    if (z) x[t] += z[t];
    if (r) r[t] = b[t] - y[t];
  }
}

}  // namespace

// Backward differentiation formulas (the textbook BDF-k; Sec. 5 uses BDF4
// started by BDF1-3): u^{n+1} - sum_i a_i u^{n-i} = b_k dt F(u^{n+1}).
void bdf_coefficients(int k, double a[4], double* b) {
  static const double A[4][4] = {{1.0, 0.0, 0.0, 0.0},
                                 {4.0 / 3.0, -1.0 / 3.0, 0.0, 0.0},
                                 {18.0 / 11.0, -9.0 / 11.0, 2.0 / 11.0, 0.0},
                                 {48.0 / 25.0, -36.0 / 25.0, 16.0 / 25.0,
                                  -3.0 / 25.0}};
  static const double B[4] = {1.0, 2.0 / 3.0, 6.0 / 11.0, 12.0 / 25.0};
  for (int i = 0; i < 4; ++i) a[i] = A[k - 1][i];
  *b = B[k - 1];
}

orbf_status launch_bdf_rhs(orbf_ctx* ctx, int64_t N, int k,
                           const double* const u[4], const double* f,
                           double dt, const uint8_t* row_kind,
                           const double* bvals, double* rhs) {
  double a[4], b;
  bdf_coefficients(k, a, &b);
  const int64_t vb = (N + 255) / 256;
  const unsigned g = (unsigned)(vb < 65536 ? vb : 65536);
  hipLaunchKernelGGL(bdf_rhs_kernel, dim3(g), dim3(256), 0, ctx->stream, N, k,
                     u[0], u[1], u[2], u[3], a[0], a[1], a[2], a[3], f,
                     b * dt, row_kind, bvals, rhs);
  return hip_check(ctx, hipGetLastError(), "BDF right-hand side");
}

size_t krylov_scratch_bytes(int64_t N, int restart) {
  // BiCGSTAB: ten vectors; GMRES(m): the m + 1 basis vectors and four more
  const size_t vecs = restart > 0 ? (size_t)restart + 5 : 10;
  return (size_t)N * vecs * 8 +
         (size_t)kDotBlocks * (kMaxRestart + 1) * 8 + 64 * 8 * 4;
}

orbf_status launch_solve_implicit(orbf_ctx* ctx, int64_t N,
                                  const int64_t* row_ptr, const int32_t* col,
                                  const double* val, const uint8_t* row_kind,
                                  double alpha, double beta, const double* b,
                                  double* x, double tol, int max_iter,
                                  int precond, const double* lu, int method,
                                  int restart, int* iters, double* relres) {
  orbf_status st = ORBF_OK;
  const int m = method == 1 ? restart : 0;
  auto* w = (double*)scratch(ctx, B_KRYLOV, krylov_scratch_bytes(N, m), &st);
  if (st) return st;
  hipStream_t sm = ctx->stream;
  const int64_t rows_blocks = (N + 15) / 16;
  const unsigned ga = (unsigned)(rows_blocks < 65536 ? rows_blocks : 65536);
  const int64_t vb = (N + 255) / 256;
  const unsigned gv = (unsigned)(vb < 65536 ? vb : 65536);
  const int gd = (int)(vb < kDotBlocks ? vb : kDotBlocks);
  double* h = ctx->host_scalars;
  double* part = w + (size_t)N * (m > 0 ? (size_t)m + 5 : 10);
  double* out = part + (size_t)kDotBlocks * (kMaxRestart + 1);
  auto apply = [&](const double* in, double* res) {
    hipLaunchKernelGGL(apply_kernel, dim3(ga), dim3(256), 0, sm, row_ptr, col,
                       val, row_kind, alpha, beta, in, N, res);
  };
  // (a.b, c.d) on the host
  auto dots = [&](const double* a, const double* bb, const double* c,
                  const double* d, double* o1, double* o2) -> orbf_status {
    hipLaunchKernelGGL(dot2_kernel, dim3(gd), dim3(256), 0, sm, a, bb, c, d,
                       N, part);
    hipLaunchKernelGGL(dot2_final_kernel, dim3(1), dim3(64), 0, sm, part, gd,
                       out);
    hipError_t e = hipMemcpyAsync(h, out, 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, sm);
    if (e == hipSuccess) e = hipStreamSynchronize(sm);
    if (e != hipSuccess) return hip_check(ctx, e, "solve: inner product");
    *o1 = h[0];
    if (o2) *o2 = h[1];
    return ORBF_OK;
  };
  // z = M^-1 v (right preconditioner); dinv is the Jacobi diagonal
  double* dinv = nullptr;
  auto precondition = [&](const double* v, double* z) -> orbf_status {
    if (precond == 1) {
      hipLaunchKernelGGL(scale_kernel, dim3(gv), dim3(256), 0, sm, dinv, v, N,
                         z);
      return ORBF_OK;
    }
    return launch_ilu_apply(ctx, N, row_ptr, col, lu, v, z);
  };
  if (precond == 2 && (st = launch_ilu_prepare(ctx, N, row_ptr, col)))
    return st;

  if (method == 1) {
    // ---- GMRES(m), right-preconditioned ----
    double* V = w;                       // m + 1 basis vectors
    double* z = V + (size_t)(m + 1) * N;  // M^-1 v
    double* wv = z + N;                  // A z, orthogonalized
    double* r = wv + N;
    dinv = r + N;
    double* hsum = out + kMaxRestart + 1;  // device: h of this column
    if (precond == 1)
      hipLaunchKernelGGL(jacobi_kernel, dim3(ga), dim3(256), 0, sm, row_ptr,
                         col, val, row_kind, alpha, beta, N, dinv);
    double bb = 0.0, rr = 0.0;
    apply(x, wv);
    hipLaunchKernelGGL(xadd_res_kernel, dim3(gv), dim3(256), 0, sm,
                       (const double*)nullptr, b, wv, N, x, r);
    if ((st = dots(b, b, r, r, &bb, &rr))) return st;
    const double nb = bb > 0.0 ? sqrt(bb) : 1.0;
    double res = sqrt(rr) / nb;
    int it = 0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
    while (res > tol && it < max_iter) {
      const double beta0 = sqrt(rr);
      if (!(beta0 > 0.0)) break;
      hipLaunchKernelGGL(vscale_kernel, dim3(gv), dim3(256), 0, sm, r,
                         1.0 / beta0, N, V);
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta0;
      int j = 0;
      for (; j < m && it < max_iter; ++j) {
        ++it;
        const double* vj = V + (size_t)j * N;
        if (precond) {
          if ((st = precondition(vj, z))) return st;
          apply(z, wv);
        } else {
          apply(vj, wv);
        }
        // classical Gram-Schmidt twice; coefficients stay on the device
        hipLaunchKernelGGL(lround_zero, dim3(1), dim3(64), 0, sm, hsum,
                           j + 1);
        for (int pass = 0; pass < 2; ++pass) {
          hipLaunchKernelGGL(mdot_kernel, dim3(gd), dim3(256), 0, sm, V,
                             j + 1, wv, N, part);
          hipLaunchKernelGGL(mdot_final_kernel, dim3(1), dim3(64), 0, sm,
                             part, gd, j + 1, out);
          hipLaunchKernelGGL(msub_kernel, dim3(gv), dim3(256), 0, sm, V,
                             j + 1, out, N, wv, hsum);
        }
        hipLaunchKernelGGL(dot2_kernel, dim3(gd), dim3(256), 0, sm, wv, wv,
                           (const double*)nullptr, (const double*)nullptr, N,
                           part);
        hipLaunchKernelGGL(dot2_final_kernel, dim3(1), dim3(64), 0, sm, part,
                           gd, hsum + j + 1);
        hipError_t e = hipMemcpyAsync(h, hsum, (j + 2) * sizeof(double),
                                      hipMemcpyDeviceToHost, sm);
        if (e == hipSuccess) e = hipStreamSynchronize(sm);
        if (e != hipSuccess) return hip_check(ctx, e, "GMRES: Arnoldi");
        double* col_j = H.data() + (size_t)j * (m + 1);
        for (int i = 0; i <= j; ++i) col_j[i] = h[i];
        const double hn = h[j + 1] > 0.0 ? sqrt(h[j + 1]) : 0.0;
        col_j[j + 1] = hn;
        // previous rotations, then a new one that zeroes H[j+1][j]
        for (int i = 0; i < j; ++i) {
          const double t0 = cs[i] * col_j[i] + sn[i] * col_j[i + 1];
          col_j[i + 1] = -sn[i] * col_j[i] + cs[i] * col_j[i + 1];
          col_j[i] = t0;
        }
        const double den = hypot(col_j[j], col_j[j + 1]);
        cs[j] = den > 0.0 ? col_j[j] / den : 1.0;
        sn[j] = den > 0.0 ? col_j[j + 1] / den : 0.0;
        col_j[j] = den;
        col_j[j + 1] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        res = fabs(g[j + 1]) / nb;
        if (res <= tol || !(hn > 0.0)) {
          ++j;
          break;
        }
        if (j + 1 < m)
          hipLaunchKernelGGL(vscale_kernel, dim3(gv), dim3(256), 0, sm, wv,
                             1.0 / hn, N, V + (size_t)(j + 1) * N);
      }
      // y = R^-1 g (upper triangular, j x j); x += M^-1 V y
      Coeffs y;
      for (int i = j - 1; i >= 0; --i) {
        double v = g[i];
        for (int k = i + 1; k < j; ++k)
          v -= H[(size_t)k * (m + 1) + i] * y.c[k];
        y.c[i] = v / H[(size_t)i * (m + 1) + i];
      }
      hipLaunchKernelGGL(lincomb_kernel, dim3(gv), dim3(256), 0, sm, V, j, y,
                         N, wv);
      if (precond) {
        if ((st = precondition(wv, z))) return st;
        hipLaunchKernelGGL(xadd_res_kernel, dim3(gv), dim3(256), 0, sm, z,
                           (const double*)nullptr, (const double*)nullptr, N,
                           x, (double*)nullptr);
      } else {
        hipLaunchKernelGGL(xadd_res_kernel, dim3(gv), dim3(256), 0, sm, wv,
                           (const double*)nullptr, (const double*)nullptr, N,
                           x, (double*)nullptr);
      }
      // the true residual decides
      apply(x, wv);
      hipLaunchKernelGGL(xadd_res_kernel, dim3(gv), dim3(256), 0, sm,
                         (const double*)nullptr, b, wv, N, x, r);
      if ((st = dots(r, r, nullptr, nullptr, &rr, nullptr))) return st;
      res = sqrt(rr) / nb;
    }
    if (iters) *iters = it;
    if (relres) *relres = res;
    return hip_check(ctx, hipGetLastError(), "GMRES");
  }

  // ---- BiCGSTAB ----
  double* r = w;
  double* rh = r + N;
  double* p = rh + N;
  double* v = p + N;
  double* s = v + N;
  double* t = s + N;
  double* y = t + N;
  dinv = y + N;           // Jacobi (right) preconditioner
  double* ph = dinv + N;  // M^-1 p
  double* sh = ph + N;    // M^-1 s
  if (precond == 1)
    hipLaunchKernelGGL(jacobi_kernel, dim3(ga), dim3(256), 0, sm, row_ptr,
                       col, val, row_kind, alpha, beta, N, dinv);
  // without preconditioning the scaled vectors are the vectors themselves
  if (!precond) {
    ph = p;
    sh = s;
  }
  apply(x, y);
  hipLaunchKernelGGL(bicg_init_kernel, dim3(gv), dim3(256), 0, sm, b, y, N,
                     r, rh, p, v);
  double bb = 0.0, rr = 0.0;
  if ((st = dots(b, b, r, r, &bb, &rr))) return st;
  const double nb = bb > 0.0 ? sqrt(bb) : 1.0;
  double res = sqrt(rr) / nb;
  int it = 0;
  double rho = 1.0, al = 1.0, om = 1.0, rho_new = 0.0;
  if ((st = dots(rh, r, nullptr, nullptr, &rho_new, nullptr))) return st;
  while (res > tol && it < max_iter) {
    if (rho_new == 0.0) break;  // breakdown: report the residual reached
    ++it;
    const double bt = (rho_new / rho) * (al / om);
    hipLaunchKernelGGL(bicg_p_kernel, dim3(gv), dim3(256), 0, sm, r, v, bt,
                       om, N, p);
    if (precond && (st = precondition(p, ph))) return st;
    apply(ph, v);
    double rhv = 0.0;
    if ((st = dots(rh, v, nullptr, nullptr, &rhv, nullptr))) return st;
    if (rhv == 0.0) break;
    al = rho_new / rhv;
    hipLaunchKernelGGL(bicg_s_kernel, dim3(gv), dim3(256), 0, sm, r, v, al, N,
                       s);
    double ss = 0.0;
    if ((st = dots(s, s, nullptr, nullptr, &ss, nullptr))) return st;
    if (sqrt(ss) / nb <= tol) {  // converged on the half step
      hipLaunchKernelGGL(bicg_x_kernel, dim3(gv), dim3(256), 0, sm, ph, ph, t,
                         al, 0.0, N, x, (double*)nullptr, (const double*)s);
      res = sqrt(ss) / nb;
      break;
    }
    if (precond && (st = precondition(s, sh))) return st;
    apply(sh, t);
    double ts = 0.0, tt = 0.0;
    if ((st = dots(t, s, t, t, &ts, &tt))) return st;
    if (tt == 0.0) break;
    om = ts / tt;
    hipLaunchKernelGGL(bicg_x_kernel, dim3(gv), dim3(256), 0, sm, ph, sh, t,
                       al, om, N, x, r, s);
    rho = rho_new;
    if ((st = dots(rh, r, r, r, &rho_new, &rr))) return st;
    res = sqrt(rr) / nb;
    if (om == 0.0) break;
  }
  if (iters) *iters = it;
  if (relres) *relres = res;
  return hip_check(ctx, hipGetLastError(), "solve");
}

}  // namespace orbf
