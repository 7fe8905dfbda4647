// Local RBF-FD weights (Sec. 4.1, eqs. rbffd_linsys, orbffd_eq, orbffd_rhs):
// entry point and kernel dispatch.  Per stencil center k the kernels form
// the scaled coordinates xi_q = (x_{I_q} - x_k) / rho_k, the saddle matrix
// [A Psi; Psi^T 0] (K = n + M) and one right-hand side per computed row e,
// (L|xi - xi_j|^m, L psi_t) at xi_e, eliminate with row partial pivoting,
// unscale by rho_k^theta and drop W^psi; each row's L-Lebesgue value is
// Lambda = sum_j |w_j| (Sec. 4.2.1).  The one-wavefront register kernel
// serves K <= 72 (weights_reg.hip, also in FP32 + refinement:
// weights_ir.hip), the four-wavefront kernel K <= 144 (weights_wg.hip).
#include <math.h>

#include "orbf_internal.hpp"
#include "weights_common.hpp"

namespace orbf {

namespace {

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
  const bool explicit_rows = a->rows != nullptr;
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
  P.tau_mode = a->tau_mode;
  P.eligible = a->eligible;
  P.t2 = t2;
  P.ir_steps = nullptr;
  P.ir_max = ctx->ir_max_corrections;
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
  // false only if no kernel serves K (the entry point admits K <= 144)
  auto fp64 = [&](const WeightsParams& Q) -> bool {
    if (sched == ORBF_SCHED_MATRIX && launch_weights_mfma(ctx, Q, grid))
      return true;
    if ((sched == ORBF_SCHED_SPLIT || split_default) && split(Q)) return true;
    if (sched == ORBF_SCHED_GROUP16 && launch_weights_wg(ctx, Q, work))
      return true;
    if (sched != ORBF_SCHED_GROUP16 &&
        launch_weights_reg(ctx, Q, grid, sched == ORBF_SCHED_WAVE8 ? 1 : 2))
      return true;
    return launch_weights_wg(ctx, Q, work);
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
  if (use_ir) {
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
    if (!fp64(F)) return fail(ctx, ORBF_EINTERNAL, "no weights kernel for K");
  } else {
    if (!fp64(P)) return fail(ctx, ORBF_EINTERNAL, "no weights kernel for K");
    if (ctx->timing) hipEventRecord(ctx->ev[9], ctx->stream);
  }
  ctx->phase_valid[4] = ctx->timing;
  return hip_check(ctx, hipGetLastError(), "weights");
}

}  // namespace orbf
