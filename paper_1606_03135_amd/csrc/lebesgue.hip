// Greedy covering with the local L-Lebesgue test (Sec. 4.2.1, eq. calLstab
// with threshold tau): node j of stencil k is kept only if j is the center
// or Lambda(x_j) <= tau * Lambda(x_ref), x_ref the stencil node nearest the
// stencil centroid; a rejected node is left for a later stencil.
//
// Whether center c keeps j depends on c's stencil alone, so the sequential
// rule (ascending index) again has a parallel form.  With edges c -> j for
// eligible j > c in ball(c): j is a center iff every predecessor is a
// non-center or a center that rejects j; its owner is the smallest
// predecessor center that keeps it.  Rounds alternate
//   decide:  undecided nodes whose predecessors are all settled become
//            covered (some predecessor center keeps them) or centers;
//   solve:   the new centers solve their ball columns plus the reference
//            column and record which ball nodes pass the test,
// until every node is settled.  A final pass computes each row from its
// owner's stencil.
#include "orbf_internal.hpp"
#include "weights_common.hpp"

namespace orbf {

namespace {

constexpr int64_t kSolveGrid = 4096;  // accept-mode solve blocks per round

enum : int32_t {
  L_UNDECIDED = 0,
  L_PENDING = 1,   // center whose acceptance bits are not computed yet
  L_SOLVED = 2,    // center with acceptance bits
  L_COVERED = 3,   // kept by some earlier center
  L_INELIGIBLE = 4
};

// predecessor entries carry the stencil position: c | (q << 25)
__global__ __launch_bounds__(256) void lpred_kernel(
    const int32_t* __restrict__ knn, int64_t N, int n,
    const uint64_t* __restrict__ ball, const int64_t* __restrict__ start,
    int32_t* __restrict__ fill, uint32_t* __restrict__ pred) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= N) return;
  for (int h = 0; h < 2; ++h) {
    uint64_t b = ball[2 * c + h];
    while (b) {
      const int q = __ffsll((long long)b) - 1 + 64 * h;
      b &= b - 1;
      const int32_t j = knn[c * n + q];
      const int slot = atomicAdd(&fill[j], 1);
      pred[start[j] + slot] = (uint32_t)c | ((uint32_t)q << 25);
    }
  }
}

__device__ __forceinline__ bool kept(const uint64_t* acc, uint32_t e) {
  const uint32_t c = e & 0x1FFFFFFu, q = e >> 25;
  return (acc[2 * (int64_t)c + (q >> 6)] >> (q & 63)) & 1ull;
}

// counters: [0] undecided after the pass, [1] new centers; the new centers
// are also appended to list (count *npend), in no particular order: each
// is solved on its own
__global__ __launch_bounds__(256) void ldecide_kernel(
    const uint32_t* __restrict__ pred, const int64_t* __restrict__ start,
    const uint64_t* __restrict__ acc, int64_t N, int32_t* state,
    int32_t* __restrict__ counters, int32_t* __restrict__ list,
    int64_t* __restrict__ npend) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  if (state[j] != L_UNDECIDED) return;
  bool settled = true, covered = false;
  for (int64_t t = start[j]; t < start[j + 1]; ++t) {
    const uint32_t e = pred[t];
    const int32_t s = __atomic_load_n(&state[e & 0x1FFFFFFu], __ATOMIC_RELAXED);
    if (s == L_UNDECIDED || s == L_PENDING) {
      settled = false;
    } else if (s == L_SOLVED && kept(acc, e)) {
      covered = true;
      break;
    }
  }
  if (covered) {
    state[j] = L_COVERED;
  } else if (settled) {
    state[j] = L_PENDING;
    atomicAdd(&counters[1], 1);
    list[atomicAdd((unsigned long long*)npend, 1ull)] = (int32_t)j;
  } else {
    atomicAdd(&counters[0], 1);
  }
}

__global__ __launch_bounds__(256) void lcompact_kernel(
    const int32_t* __restrict__ flag, const int64_t* __restrict__ pos,
    int64_t N, int32_t* __restrict__ list, int64_t* __restrict__ count) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j == N) *count = pos[N];
  if (j < N && flag[j]) list[pos[j]] = (int32_t)j;
}

__global__ __launch_bounds__(256) void lsolved_kernel(
    const int32_t* __restrict__ list, const int64_t* __restrict__ count,
    int32_t* __restrict__ state) {
  const int64_t cnt = *count;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < cnt;
       t += (int64_t)gridDim.x * 256)
    state[list[t]] = L_SOLVED;
}

// start of a round: counters and the pending count
__global__ void lround_zero_kernel(int32_t* counters, int64_t* npend) {
  if (threadIdx.x < 2) counters[threadIdx.x] = 0;
  if (threadIdx.x == 0) *npend = 0;
}

__global__ __launch_bounds__(256) void lowner_kernel(
    const uint32_t* __restrict__ pred, const int64_t* __restrict__ start,
    const uint64_t* __restrict__ acc, const int32_t* __restrict__ state,
    int64_t N, int32_t* __restrict__ owner, int32_t* __restrict__ is_center) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  const int32_t s = state[j];
  int32_t o = -1;
  if (s == L_SOLVED) {
    o = (int32_t)j;
  } else if (s == L_COVERED) {
    o = INT32_MAX;
    for (int64_t t = start[j]; t < start[j + 1]; ++t) {
      const uint32_t e = pred[t];
      const int32_t c = (int32_t)(e & 0x1FFFFFFu);
      if (state[c] == L_SOLVED && kept(acc, e) && c < o) o = c;
    }
  }
  owner[j] = o;
  is_center[j] = s == L_SOLVED;
}

__global__ __launch_bounds__(256) void lzero_kernel(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    p[i] = 0;
}

}  // namespace

orbf_status launch_lebesgue_cover(orbf_ctx* ctx, const WeightsParams& P0,
                                  double t2, const uint8_t* eligible,
                                  int32_t* centers, int64_t* n_centers,
                                  int32_t* owner) {
  const int64_t N = P0.N;
  const int n = P0.n, d = P0.d;
  if (N >= (1 << 25) || n > 128)
    return fail(ctx, ORBF_EINVAL, "Lebesgue covering: N < 2^25, n <= 128");
  orbf_status st = ORBF_OK;
  auto* ball = (uint64_t*)scratch(ctx, B_BALL, (size_t)N * 16, &st);
  auto* indeg = (int32_t*)scratch(ctx, B_INDEG, (size_t)(N + 1) * 4, &st);
  auto* pstart = (int64_t*)scratch(ctx, B_PRED_START, (size_t)(N + 2) * 8, &st);
  auto* fill = (int32_t*)scratch(ctx, B_PRED_FILL, (size_t)(N + 1) * 4, &st);
  auto* state = (int32_t*)scratch(ctx, B_STATE, (size_t)N * 4, &st);
  auto* flag = (int32_t*)scratch(ctx, B_FLAGS, (size_t)(N + 1) * 4, &st);
  auto* pos = (int64_t*)scratch(ctx, B_CENTER_POS, (size_t)(N + 2) * 8, &st);
  auto* list = (int32_t*)scratch(ctx, B_ROWPTR_TMP, (size_t)(N + 1) * 4, &st);
  auto* acc = (uint64_t*)scratch(ctx, B_W_TMP, (size_t)N * 16, &st);
  auto* misc = (int64_t*)scratch(ctx, B_MISC2, 64, &st);
  if (st) return st;
  const size_t max_edges = (size_t)N * (size_t)(n > 1 ? n - 1 : 1);
  auto* pred = (uint32_t*)scratch(ctx, B_PRED, max_edges * 4, &st);
  if (st) return st;
  hipStream_t s = ctx->stream;
  const unsigned g = (unsigned)((N + 255) / 256);
  const unsigned g1 = (unsigned)((N + 256) / 256);
  const unsigned gz = g1 < 65535 ? g1 : 65535;
  int32_t* counters = (int32_t*)misc;   // 2 int32
  int64_t* npend = misc + 1;
  hipLaunchKernelGGL(lzero_kernel, dim3(gz), dim3(256), 0, s, indeg, N + 1);
  hipLaunchKernelGGL(lzero_kernel, dim3(gz), dim3(256), 0, s, fill, N + 1);
  hipLaunchKernelGGL(lzero_kernel, dim3(gz), dim3(256), 0, s, (int32_t*)acc,
                     4 * N);
  launch_ball(ctx, P0.xyz, P0.knn, P0.rho2, N, d, n, t2, eligible, ball,
              indeg, state, L_UNDECIDED, L_INELIGIBLE);
  if ((st = exclusive_scan_i32_to_i64(ctx, indeg, N, pstart))) return st;
  hipLaunchKernelGGL(lpred_kernel, dim3(g), dim3(256), 0, s, P0.knn, N, n,
                     ball, pstart, fill, pred);

  WeightsParams P = P0;
  P.eligible = eligible;
  P.t2 = t2;
  P.ball = ball;
  P.accept = acc;
  P.centers = list;
  P.n_centers = npend;
  P.owner = nullptr;
  P.W = nullptr;
  P.lebesgue = nullptr;
  // A round decides every node whose predecessors are settled, then solves
  // the new centers in accept mode and marks them solved.  The kernels read
  // the pending count on the device, so rounds run back to back and the
  // host reads the last round's counters only after each batch of rounds;
  // rounds after the last decision find nothing to do.
  const unsigned gs = (unsigned)(N < kSolveGrid ? N : kSolveGrid);
  const unsigned gm = (unsigned)((N + 255) / 256 < 1024 ? (N + 255) / 256 : 1024);
  int32_t hc[2];
  int64_t rounds = 0;
  for (int batch = 1;; batch = batch < 64 ? 2 * batch : 64) {
    for (int r = 0; r < batch; ++r, ++rounds) {
      hipLaunchKernelGGL(lround_zero_kernel, dim3(1), dim3(64), 0, s,
                         counters, npend);
      hipLaunchKernelGGL(ldecide_kernel, dim3(g), dim3(256), 0, s, pred,
                         pstart, acc, N, state, counters, list, npend);
      if (!launch_weights_reg(ctx, P, gs))
        return fail(ctx, ORBF_EINVAL,
                    "Lebesgue covering needs the register weights kernel "
                    "(n + M <= 72, M <= 35)");
      hipLaunchKernelGGL(lsolved_kernel, dim3(gm), dim3(256), 0, s, list,
                         npend, state);
    }
    hipError_t e = hipMemcpyAsync(hc, counters, sizeof hc,
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if ((st = hip_check(ctx, e, "Lebesgue covering round"))) return st;
    // the last round left no node undecided and made no new center
    if (hc[0] == 0 && hc[1] == 0) break;
    if (rounds > N + 2)
      return fail(ctx, ORBF_EINTERNAL, "Lebesgue covering did not settle");
  }
  hipLaunchKernelGGL(lowner_kernel, dim3(g), dim3(256), 0, s, pred, pstart,
                     acc, state, N, owner, flag);
  if ((st = exclusive_scan_i32_to_i64(ctx, flag, N, pos))) return st;
  hipLaunchKernelGGL(lcompact_kernel, dim3(g1), dim3(256), 0, s, flag, pos, N,
                     centers, n_centers);
  return hip_check(ctx, hipGetLastError(), "Lebesgue covering");
}

}  // namespace orbf
