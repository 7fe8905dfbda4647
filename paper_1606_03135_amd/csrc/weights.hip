// Local RBF-FD weights (Sec. 4.1, eqs. rbffd_linsys, orbffd_eq, orbffd_rhs).
//
// One wavefront per stencil center k:
//   - scaled coordinates xi_q = (x_{I_q} - x_k) / rho_k of the n stencil
//     nodes,
//   - the saddle matrix [A Psi; Psi^T 0] (K = n + M) and one right-hand side
//     per computed row e: (L|xi - xi_j|^m, L psi_t) at xi_e,
//   - Gaussian elimination with row partial pivoting (the zero diagonal of
//     A and the zero block make pivoting necessary from the first step),
//   - back substitution, unscaling by rho_k^theta, W^psi dropped,
//   - the L-Lebesgue value of each row, Lambda = sum_j |w_j| (Sec. 4.2.1).
// The augmented matrix lives in LDS; right-hand sides beyond the LDS
// capacity are solved in further chunks against the stored factors.
#include <math.h>

#include "orbf_internal.hpp"
#include "weights_common.hpp"

namespace orbf {

namespace {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}



// r^k for odd k >= 1, from r2 = r^2
__device__ __forceinline__ double odd_pow(double r2, int k) {
  double p = sqrt(r2);
  for (int i = 0; i < (k - 1) / 2; ++i) p *= r2;
  return p;
}

__device__ __forceinline__ double ipow(double v, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= v;
  return r;
}

__device__ __forceinline__ double mono(const double* p, const int8_t* e,
                                       int d) {
  double r = ipow(p[0], e[0]) * ipow(p[1], e[1]);
  if (d == 3) r *= ipow(p[2], e[2]);
  return r;
}

// L psi at p: Laplacian sum_a e_a(e_a-1) p^(e-2eps_a), identity p^e, or a
// first derivative along nrm (a normal, or e_a for d/dx_a)
__device__ double mono_op(const double* p, const int8_t* e, int d, int op,
                          const double* nrm) {
  if (op == ORBF_OP_IDENTITY) return mono(p, e, d);
  double s = 0.0;
  for (int a = 0; a < d; ++a) {
    int f[3] = {e[0], e[1], d == 3 ? e[2] : 0};
    if (op == ORBF_OP_LAPLACIAN) {
      if (f[a] < 2) continue;
      const double c = (double)(f[a] * (f[a] - 1));
      f[a] -= 2;
      double v = ipow(p[0], f[0]) * ipow(p[1], f[1]);
      if (d == 3) v *= ipow(p[2], f[2]);
      s += c * v;
    } else {
      if (f[a] < 1) continue;
      const double c = (double)f[a];
      f[a] -= 1;
      double v = ipow(p[0], f[0]) * ipow(p[1], f[1]);
      if (d == 3) v *= ipow(p[2], f[2]);
      s += nrm[a] * (c * v);
    }
  }
  return s;
}

// L |xi - xi_j|^m at p
__device__ __forceinline__ double phs_op(const double* p, const double* q,
                                         int d, int m, int op,
                                         const double* nrm) {
  const double dx = p[0] - q[0], dy = p[1] - q[1];
  const double dz = (d == 3) ? p[2] - q[2] : 0.0;
  const double r2 = dx * dx + dy * dy + dz * dz;
  if (op == ORBF_OP_LAPLACIAN)  // Laplacian of r^m: m (m + d - 2) r^(m-2)
    return (double)(m * (m + d - 2)) * odd_pow(r2, m - 2);
  if (op == ORBF_OP_IDENTITY) return odd_pow(r2, m);
  // gradient of r^m: m r^(m-2) (x - x_j)
  double dot = dx * nrm[0] + dy * nrm[1];
  if (d == 3) dot += dz * nrm[2];
  return ((double)m * odd_pow(r2, m - 2)) * dot;
}

__global__ __launch_bounds__(64) void weights_lds_kernel(WeightsParams P) {
  extern __shared__ double smem[];
  const int lane = threadIdx.x;
  const int n = P.n, K = P.K, d = P.d, ldm = P.ldm, M = P.M;
  double* A = smem;                         // K x ldm
  double* xi = A + (size_t)K * ldm;         // n x 3
  int* cols = (int*)(xi + 3 * n);           // n (stencil positions)
  int* piv = cols + n;                      // K
  int8_t* ex = (int8_t*)(piv + K);          // M*3

  for (int t = lane; t < 3 * M; t += 64) ex[t] = P.ex[t];

  const bool explicit_rows = P.rows != nullptr;
  const int64_t total = explicit_rows ? P.n_rows : *P.n_centers;
  for (int64_t ci = blockIdx.x; ci < total; ci += gridDim.x) {
    const int32_t c = explicit_rows ? P.rows[ci] : P.centers[ci];
    if ((uint32_t)c >= (uint64_t)P.N) {  // invalid row list entry
      if (lane == 0) report(P.st, ORBF_EINVAL, c);
      continue;
    }
    const int32_t* stn = P.knn + (int64_t)c * n;
    const double* nrm = nullptr;
    double nv[3] = {0, 0, 0};
    if (explicit_rows && P.op == ORBF_OP_NEUMANN) {
      for (int a = 0; a < d; ++a) nv[a] = P.normals[ci * d + a];
      nrm = nv;
    } else if (P.op >= ORBF_OP_DX && P.op <= ORBF_OP_DZ) {
      nv[P.op - ORBF_OP_DX] = 1.0;
      nrm = nv;
    }
    bool bad = false;
    for (int q = lane; q < n; q += 64) bad |= (uint32_t)stn[q] >= (uint64_t)P.N;
    if (__ballot(bad)) {  // stencil indices from a failed kNN
      if (lane == 0) report(P.st, ORBF_EINVAL, c);
      continue;
    }
    // columns: stencil positions whose row this stencil computes
    int ncol = 0;
    if (explicit_rows) {
      if (lane == 0) cols[0] = 0;
      ncol = 1;
    } else {
      for (int q0 = 0; q0 < n; q0 += 64) {
        const int q = q0 + lane;
        const bool mine = q < n && P.owner[stn[q]] == c;
        const unsigned long long b = __ballot(mine);
        if (mine) {
          const int r = __popcll(b & ((1ull << lane) - 1ull));
          cols[ncol + r] = q;
        }
        ncol += __popcll(b);
      }
    }
    // scaled coordinates
    const double r2c = P.rho2[c];
    const double rho = sqrt(r2c);
    const double* xc = P.xyz + (int64_t)c * d;
    for (int q = lane; q < n; q += 64) {
      const double* xq = P.xyz + (int64_t)stn[q] * d;
      for (int a = 0; a < 3; ++a)
        xi[3 * q + a] = (a < d) ? (xq[a] - xc[a]) / rho : 0.0;
    }
    wave_sync();
    // A_hat = [A Psi; Psi^T 0]
    for (int idx = lane; idx < K * K; idx += 64) {
      const int i = idx / K, j = idx - i * K;
      double v = 0.0;
      if (i < n && j < n) {
        const double dx = xi[3 * i] - xi[3 * j], dy = xi[3 * i + 1] - xi[3 * j + 1];
        const double dz = xi[3 * i + 2] - xi[3 * j + 2];
        v = odd_pow(dx * dx + dy * dy + dz * dz, P.m);
      } else if (i < n) {
        v = mono(xi + 3 * i, ex + 3 * (j - n), d);
      } else if (j < n) {
        v = mono(xi + 3 * j, ex + 3 * (i - n), d);
      }
      A[(size_t)i * ldm + j] = v;
    }
    wave_sync();
    bool singular = false;
    const double scale = (P.op == ORBF_OP_LAPLACIAN) ? r2c
                         : (P.op == ORBF_OP_IDENTITY) ? 1.0
                                                      : rho;
    for (int cb = 0; cb < ncol; cb += P.pcap) {
      const int nb = min(P.pcap, ncol - cb);
      double* B = A + K;  // columns K .. K+nb of each row
      for (int idx = lane; idx < K * nb; idx += 64) {
        const int i = idx / nb, e = idx - i * nb;
        const double* pe = xi + 3 * cols[cb + e];
        B[(size_t)i * ldm + e] = (i < n) ? phs_op(pe, xi + 3 * i, d, P.m, P.op, nrm)
                                         : mono_op(pe, ex + 3 * (i - n), d, P.op, nrm);
      }
      wave_sync();
      if (cb == 0) {
        // factor [A | B] in place
        for (int k = 0; k < K && !singular; ++k) {
          double best = -1.0;
          int bi = K;
          for (int r = k + lane; r < K; r += 64) {
            const double v = fabs(A[(size_t)r * ldm + k]);
            if (v > best) {
              best = v;
              bi = r;
            }
          }
#pragma unroll
          for (int o = 32; o >= 1; o >>= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) {
              best = ob;
              bi = oi;
            }
          }
          if (!(best > 0.0)) {
            singular = true;
            break;
          }
          if (lane == 0) piv[k] = bi;
          if (bi != k)
            for (int j = lane; j < K + nb; j += 64) {
              const double t = A[(size_t)k * ldm + j];
              A[(size_t)k * ldm + j] = A[(size_t)bi * ldm + j];
              A[(size_t)bi * ldm + j] = t;
            }
          wave_sync();
          const double pinv = 1.0 / A[(size_t)k * ldm + k];
          for (int r = k + 1 + lane; r < K; r += 64)
            A[(size_t)r * ldm + k] *= pinv;
          wave_sync();
          for (int j = k + 1 + lane; j < K + nb; j += 64) {
            const double u = A[(size_t)k * ldm + j];
            for (int r = k + 1; r < K; ++r)
              A[(size_t)r * ldm + j] -= A[(size_t)r * ldm + k] * u;
          }
          wave_sync();
        }
      } else if (!singular) {
        // apply the stored row interchanges, then L^{-1}
        for (int k = 0; k < K; ++k) {
          const int pk = piv[k];
          if (pk != k)
            for (int e = lane; e < nb; e += 64) {
              const double t = B[(size_t)k * ldm + e];
              B[(size_t)k * ldm + e] = B[(size_t)pk * ldm + e];
              B[(size_t)pk * ldm + e] = t;
            }
          wave_sync();
        }
        for (int e = lane; e < nb; e += 64)
          for (int k = 0; k < K; ++k) {
            const double yk = B[(size_t)k * ldm + e];
            for (int r = k + 1; r < K; ++r)
              B[(size_t)r * ldm + e] -= A[(size_t)r * ldm + k] * yk;
          }
        wave_sync();
      }
      if (singular) {
        if (lane == 0) report(P.st, ORBF_ESINGULAR, c);
      }
      // back substitution, one lane per right-hand side
      for (int e = lane; e < nb; e += 64) {
        for (int k = K - 1; k >= 0; --k) {
          double s = B[(size_t)k * ldm + e];
          for (int j = k + 1; j < K; ++j) s -= A[(size_t)k * ldm + j] * B[(size_t)j * ldm + e];
          B[(size_t)k * ldm + e] = s / A[(size_t)k * ldm + k];
        }
        const int32_t row = stn[cols[cb + e]];
        double lam = 0.0;
        for (int j = 0; j < n; ++j) {
          const double wv = singular ? NAN : B[(size_t)j * ldm + e] / scale;
          P.W[(int64_t)row * n + j] = wv;
          lam += fabs(wv);
        }
        if (P.lebesgue) P.lebesgue[row] = lam;
        if (explicit_rows && P.owner_out) P.owner_out[row] = row;
      }
      wave_sync();
    }
  }
}

// Sort the stencils of `centers` into three lists by retained-row count p
// (owner[j] == c over the stencil of c, as the weights kernels count it):
// p <= 8, p <= 16 and above, for 8, 16 and 24 right-hand sides per pass.
// A wavefront takes 64 stencils: their counts are formed sixteen lanes per
// stencil (n <= 128: eight positions per lane), four stencils at a time,
// and gathered in LDS; then one lane per stencil appends it to its list,
// with one atomic per class per 64 stencils (three counters only, so
// fewer, larger reservations are what keeps them from serialising).
__global__ __launch_bounds__(256) void stencil_class_kernel(
    const int32_t* __restrict__ centers, const int64_t* __restrict__ n_centers,
    const int32_t* __restrict__ knn, const int32_t* __restrict__ owner,
    int64_t N, int n, int32_t* __restrict__ lists,
    unsigned long long* __restrict__ counts) {
  __shared__ int p_s[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int pl = lane & 15, grp = lane >> 4;
  const int64_t total = *n_centers;
  for (int64_t b64 = ((int64_t)blockIdx.x * 4 + w) * 64; b64 < total;
       b64 += (int64_t)gridDim.x * 256) {
#pragma unroll 4
    for (int t = 0; t < 16; ++t) {
      const int64_t ci = b64 + 4 * t + grp;
      int p = 0;
      if (ci < total) {
        const int32_t c = centers[ci];
        if ((uint32_t)c < (uint64_t)N) {
          const int32_t* st = knn + (int64_t)c * n;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int q = pl + 16 * i;
            if (q < n) {
              const int32_t j = st[q];
              p += (uint32_t)j < (uint64_t)N && owner[j] == c;
            }
          }
        }
      }
      p += __shfl_xor(p, 1, 64);
      p += __shfl_xor(p, 2, 64);
      p += __shfl_xor(p, 4, 64);
      p += __shfl_xor(p, 8, 64);
      if (pl == 0) p_s[w][4 * t + grp] = p;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t ci = b64 + lane;
    const bool live = ci < total;
    const int p = p_s[w][lane];
    const int cls = p <= 8 ? 0 : (p <= 16 ? 1 : 2);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const unsigned long long m = __ballot(live && cls == k);
      if (m == 0ull) continue;
      const int lead = __ffsll((long long)m) - 1;
      unsigned long long at = 0;
      if (lane == lead)
        at = atomicAdd(&counts[k], (unsigned long long)__popcll(m));
      at = __shfl(at, lead, 64);
      if (live && cls == k)
        lists[(int64_t)k * N + at + __popcll(m & ((1ull << lane) - 1ull))] =
            centers[ci];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// The same lists from counts already known (the covering's), one thread
// per stencil; 1024-thread blocks gather their slots in LDS so that each
// block makes one atomic per class.
__global__ __launch_bounds__(1024) void stencil_class_from_p_kernel(
    const int32_t* __restrict__ centers, const int64_t* __restrict__ n_centers,
    const int32_t* __restrict__ pcount, int64_t N,
    int32_t* __restrict__ lists, unsigned long long* __restrict__ counts) {
  __shared__ int wave_n[3][16];
  __shared__ unsigned long long block_at[3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t total = *n_centers;
  for (int64_t b = (int64_t)blockIdx.x * 1024; b < total;
       b += (int64_t)gridDim.x * 1024) {
    const int64_t ci = b + threadIdx.x;
    const bool live = ci < total;
    const int p = live ? pcount[ci] : 0;
    const int cls = p <= 8 ? 0 : (p <= 16 ? 1 : 2);
    unsigned long long m[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      m[k] = __ballot(live && cls == k);
      if (lane == 0) wave_n[k][w] = __popcll(m[k]);
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      const int k = threadIdx.x;
      int sum = 0;
      for (int i = 0; i < 16; ++i) {
        const int v = wave_n[k][i];
        wave_n[k][i] = sum;  // exclusive prefix over the block's wavefronts
        sum += v;
      }
      block_at[k] = sum ? atomicAdd(&counts[k], (unsigned long long)sum) : 0ull;
    }
    __syncthreads();
    if (live)
      lists[(int64_t)cls * N + block_at[cls] + wave_n[cls][w] +
            __popcll(m[cls] & ((1ull << lane) - 1ull))] = centers[ci];
    __syncthreads();
  }
}

__global__ void zero3_u64_kernel(unsigned long long* c) {
  if (threadIdx.x < 3) c[threadIdx.x] = 0ull;
}

}  // namespace

orbf_status launch_weights(orbf_ctx* ctx, orbf_op op, int m, int l, int n,
                           double t2, const orbf_weights_args* a) {
  orbf_status st = ORBF_OK;
  const int d = a->d;
  int8_t ex[3 * 512] = {};
  int M = 0;
  for (int deg = 0; deg <= l; ++deg) {
    if (d == 2) {
      for (int e0 = deg; e0 >= 0; --e0) {
        ex[3 * M] = (int8_t)e0;
        ex[3 * M + 1] = (int8_t)(deg - e0);
        ex[3 * M + 2] = 0;
        ++M;
      }
    } else {
      for (int e0 = deg; e0 >= 0; --e0)
        for (int e1 = deg - e0; e1 >= 0; --e1) {
          ex[3 * M] = (int8_t)e0;
          ex[3 * M + 1] = (int8_t)e1;
          ex[3 * M + 2] = (int8_t)(deg - e0 - e1);
          ++M;
        }
    }
  }
  const int K = n + M;
  if (M > 80) return fail(ctx, ORBF_EINVAL, "compute_weights: M > 80");
  hipError_t e = hipSuccess;

  int max_lds = 65536;
  hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                        ctx->device);
  const bool explicit_rows = a->rows != nullptr;
  int pcap = (explicit_rows || t2 == 0.0) ? 1 : (n < 64 ? n : 64);
  auto lds_bytes = [&](int pc) {
    return (size_t)K * (K + pc) * 8 + (size_t)n * 24 + (size_t)(n + K) * 4 +
           3 * (size_t)M + 16;
  };
  while (pcap > 1 && lds_bytes(pcap) > (size_t)max_lds) pcap /= 2;
  if (lds_bytes(pcap) > (size_t)max_lds)
    return fail(ctx, ORBF_EINVAL, "compute_weights: n + M too large for LDS");
  if (lds_bytes(pcap) > 65536) {
    e = hipFuncSetAttribute((const void*)weights_lds_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes(pcap));
    if ((st = hip_check(ctx, e, "weights: LDS attribute"))) return st;
  }
  WeightsParams P;
  P.xyz = a->xyz;
  P.knn = a->knn;
  P.rho2 = a->rho2;
  P.centers = a->centers;
  P.n_centers = a->n_centers;
  P.rows = a->rows;
  P.n_rows = a->n_rows;
  P.owner = a->owner;
  P.N = a->N;
  P.owner_out = explicit_rows ? a->owner : nullptr;
  P.normals = a->normals;
  for (int t = 0; t < 3 * 80; ++t) P.ex[t] = t < 3 * M ? ex[t] : 0;
  P.W = a->W;
  P.lebesgue = a->lebesgue;
  P.ball = nullptr;
  P.accept = nullptr;
  P.tau = a->tau;
  P.ir_steps = nullptr;
  P.fb_list = nullptr;
  P.fb_count = nullptr;
  P.st = ctx->status;
  P.d = d;
  P.n = n;
  P.m = m;
  P.l = l;
  P.M = M;
  P.K = K;
  P.op = (int)op;
  P.pcap = pcap;
  P.ldm = K + pcap;
  if (!explicit_rows && !isinf(a->tau)) {
    // covering with the L-Lebesgue test first; rows below use its owners
    ctx->p_cache = PCache();  // these centers are not the cached covering's
    st = launch_lebesgue_cover(ctx, P, t2, a->eligible, a->centers,
                               a->n_centers, a->owner);
    if (st) return st;
  }
  const int64_t work = explicit_rows ? a->n_rows : a->N;
  // The stencil count is on the device, so the grid is sized from the
  // number of possible stencils, capped at 65536 blocks (32 per resident
  // wavefront slot at two wavefronts per SIMD); each block strides over the
  // stencils.  Below the cap every stencil has a block of its own and the
  // hardware dispatcher balances their uneven costs; the cap keeps blocks
  // that find no stencil from holding slots (1M-node ball, 121k stencils:
  // 6.21 ms capped against 6.42 ms with one block per node), while few
  // enough stencils per block keep the tail short (16384 blocks: 6.45 ms).
  constexpr int64_t kMaxGrid = 65536;
  const int64_t grid = work < kMaxGrid ? work : kMaxGrid;
  if (grid <= 0) return ORBF_OK;
  static const bool force_lds = getenv("ORBF_WEIGHTS_LDS") != nullptr;
  // FP64 kernels: the tuned schedule of (K, p-class) if there is one, else
  // one wavefront (K <= 72), one workgroup of four (K <= 144), else the
  // LDS-resident kernel.  p-class: expected kept rows n (1-delta)^d > 8.
  const double keep = explicit_rows ? 1.0 : n * pow(t2, 0.5 * d);
  const int sched = schedule_for(ctx, K, keep > 8.0 ? 1 : 0);
  // SPLIT: three lists by retained rows, one launch each
  auto split = [&](const WeightsParams& Q) -> bool {
    // the covering's own list only (not an FP32 fallback list)
    if (Q.rows != nullptr || Q.centers != a->centers || K > 72 || M > 35)
      return false;
    orbf_status s2 = ORBF_OK;
    auto* lists = (int32_t*)scratch(ctx, B_CLASS, (size_t)a->N * 12, &s2);
    auto* counts = (unsigned long long*)scratch(ctx, B_CLASS_N, 24, &s2);
    if (s2) return false;
    hipLaunchKernelGGL(zero3_u64_kernel, dim3(1), dim3(64), 0, ctx->stream,
                       counts);
    if (ctx->p_cache.matches(Q.centers, Q.owner, a->N, n)) {
      const int64_t cb = (work + 1023) / 1024;
      hipLaunchKernelGGL(stencil_class_from_p_kernel,
                         dim3((unsigned)(cb < 1024 ? cb : 1024)), dim3(1024),
                         0, ctx->stream, Q.centers, Q.n_centers,
                         ctx->p_cache.p, a->N, lists, counts);
    } else {
      const int64_t cb = (work + 255) / 256;  // 256 stencils per block
      hipLaunchKernelGGL(stencil_class_kernel,
                         dim3((unsigned)(cb < 8192 ? cb : 8192)), dim3(256),
                         0, ctx->stream, Q.centers, Q.n_centers, Q.knn,
                         Q.owner, a->N, n, lists, counts);
    }
    // one after the other, widest first, so the launch with the cheapest
    // stencils forms the tail (running them side by side on separate
    // streams measured slower: 6.18 against 5.95 ms)
    for (int k = 2; k >= 0; --k) {
      WeightsParams R = Q;
      R.centers = lists + (int64_t)k * a->N;
      R.n_centers = (int64_t*)(counts + k);
      launch_weights_reg(ctx, R, grid, k + 1);
    }
    return true;
  };
  // Without a tuned schedule, large node sets (where each of the three
  // lists fills the device) take SPLIT: on the 1M-node ball 5.91 ms against
  // 6.25 ms for one 16-wide launch, whose stencils with p > 16 need a
  // second full elimination.
  const bool split_default = sched == ORBF_SCHED_DEFAULT && a->N >= 65536;
  auto fp64 = [&](const WeightsParams& Q) {
    if ((sched == ORBF_SCHED_SPLIT || split_default) && split(Q)) return;
    if (sched == ORBF_SCHED_GROUP16 && launch_weights_wg(ctx, Q, work)) return;
    if (sched != ORBF_SCHED_GROUP16 &&
        launch_weights_reg(ctx, Q, grid, sched == ORBF_SCHED_WAVE8 ? 1 : 2))
      return;
    if (launch_weights_wg(ctx, Q, work)) return;
    hipLaunchKernelGGL(weights_lds_kernel, dim3((unsigned)grid), dim3(64),
                       lds_bytes(pcap), ctx->stream, Q);
  };
  // FP32 + refinement for covered rows; explicit rows, and systems beyond
  // the register variants, are solved in FP64 (their ir_steps stay -1)
  const bool use_ir = a->prec == ORBF_PREC_FP32_IR && !explicit_rows;
  int32_t* fb_list = nullptr;
  int64_t* fb_count = nullptr;
  if (use_ir) {
    fb_list = (int32_t*)scratch(ctx, B_IR_FALLBACK, (size_t)a->N * 4, &st);
    if (st) return st;
    fb_count = (int64_t*)scratch(ctx, B_IR_COUNT, 8, &st);
    if (st) return st;
    launch_ir_prepare(ctx, a->ir_steps, a->N, fb_count);
  }
  if (ctx->timing) hipEventRecord(ctx->ev[8], ctx->stream);
  bool ir_done = false;
  if (use_ir && !force_lds) {
    WeightsParams Q = P;
    Q.ir_steps = a->ir_steps;
    Q.fb_list = fb_list;
    Q.fb_count = fb_count;
    ir_done = launch_weights_ir(ctx, Q, grid);
  }
  if (ir_done) {
    if (ctx->timing) hipEventRecord(ctx->ev[9], ctx->stream);
    // stencils the refinement did not settle: FP64 from scratch
    WeightsParams F = P;
    F.centers = fb_list;
    F.n_centers = fb_count;
    fp64(F);
  } else {
    if (force_lds)
      hipLaunchKernelGGL(weights_lds_kernel, dim3((unsigned)grid), dim3(64),
                         lds_bytes(pcap), ctx->stream, P);
    else
      fp64(P);
    if (ctx->timing) hipEventRecord(ctx->ev[9], ctx->stream);
  }
  ctx->phase_valid[4] = ctx->timing;
  return hip_check(ctx, hipGetLastError(), "weights");
}

}  // namespace orbf
