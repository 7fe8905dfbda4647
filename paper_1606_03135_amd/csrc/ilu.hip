// ILU(0) of the implicit time-step matrix (Sec. 5; Secs. 7.1 and 7.2 solve
// the step with ILU(0)-preconditioned GMRES in 2D and BiCGSTAB in 3D).
//
// The step matrix A has the DM's sparsity (row e: alpha e_e + beta L_e for
// interior rows, e_e for Dirichlet rows, L_e for boundary-operator rows; see
// krylov.hip).  ILU(0) is Gaussian elimination restricted to that pattern:
// for each row i, for each k < i in the row (ascending), a_ik /= a_kk and
// a_ij -= a_ik a_kj for every j > k in both rows i and k.  L (unit lower)
// and U share A's storage.
//
// Row i needs the finished rows k < i of its pattern, and on these DMs the
// chains of such dependencies are hundreds of rows long, so level-by-level
// launches would cost hundreds of launches per solve.  Instead one launch
// runs the whole factorization (and each triangular solve): a wavefront
// claims the next row in order from a counter, waits for the rows it needs
// (a flag per row, set with release order after the row is written), and
// finishes its row.  A row only waits for rows claimed before it, by
// wavefronts already running, and the lowest unfinished claimed row waits
// for nothing, so the launch always drains.  Every wait is bounded: past the
// bound the kernel records EINTERNAL and moves on, so it ends regardless.
#include "orbf_internal.hpp"

namespace orbf {

namespace {

constexpr int kSpinLimit = 1 << 22;

// Wait for a flag that is the same for the whole wavefront: every lane polls
// it and the exit is taken on lane 0's reading (readfirstlane), so the loop
// is wave-uniform.
__device__ __forceinline__ bool wait_flag_uniform(const int32_t* flag) {
  for (int s = 0; s < kSpinLimit; ++s) {
    const int f =
        __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__builtin_amdgcn_readfirstlane(f)) return true;
  }
  return false;
}

// Wait for a flag of this lane's own (lanes leave the loop one by one).
__device__ __forceinline__ bool wait_flag_lane(const int32_t* flag) {
  for (int s = 0; s < kSpinLimit; ++s)
    if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return true;
  return false;
}

// The next row of the wavefront, as a wave-uniform (scalar) value.  All
// lanes execute the atomic (lane 0 adds one, the others zero) and the
// ticket is lane 0's result, taken with readfirstlane.  No part of the
// claim sits under a lane test: the loop that claims rows must exit as a
// whole wavefront, and a lane-0 branch here lets the compiler fuse it with
// the lane-0 work at the end of the previous row into a per-lane loop.
__device__ __forceinline__ int64_t claim(unsigned long long* next, int lane) {
  const unsigned long long v = atomicAdd(next, lane == 0 ? 1ull : 0ull);
  const unsigned lo =
      (unsigned)__builtin_amdgcn_readfirstlane((int)(v & 0xFFFFFFFFull));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((unsigned long long)hi << 32) | lo);
}

// values of the step matrix on the DM's pattern, and each row's diagonal
// position (-1 if the row has no diagonal entry); sixteen lanes per row
__global__ __launch_bounds__(256) void step_values_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const uint8_t* __restrict__ row_kind,
    double alpha, double beta, int64_t N, double* __restrict__ a,
    int32_t* __restrict__ diag, int32_t* __restrict__ flags) {
  const int pl = threadIdx.x & 15;
  for (int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4; e < N;
       e += (int64_t)gridDim.x * 16) {
    const int kind = row_kind ? row_kind[e] : 1;
    const int64_t s0 = row_ptr[e], s1 = row_ptr[e + 1];
    int dp = -1;
    for (int64_t t = s0 + pl; t < s1; t += 16) {
      const bool dg = col[t] == e;
      if (dg) dp = (int)(t - s0);
      a[t] = kind == 1 ? (dg ? fma(beta, val[t], alpha) : beta * val[t])
             : kind == 0 ? (dg ? 1.0 : 0.0)
                         : val[t];
    }
    for (int o = 1; o < 16; o <<= 1) dp = max(dp, __shfl_xor(dp, o, 64));
    if (pl == 0) {
      diag[e] = dp;
      flags[e] = 0;
    }
  }
}

// each row's diagonal position (-1 if none); sixteen lanes per row
__global__ __launch_bounds__(256) void diag_pos_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    int64_t N, int32_t* __restrict__ diag) {
  const int pl = threadIdx.x & 15;
  for (int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4; e < N;
       e += (int64_t)gridDim.x * 16) {
    const int64_t s0 = row_ptr[e], s1 = row_ptr[e + 1];
    int dp = -1;
    for (int64_t t = s0 + pl; t < s1; t += 16)
      if (col[t] == e) dp = (int)(t - s0);
    for (int o = 1; o < 16; o <<= 1) dp = max(dp, __shfl_xor(dp, o, 64));
    if (pl == 0) diag[e] = dp;
  }
}

__global__ void ilu_zero_counter_kernel(unsigned long long* c) {
  if (threadIdx.x == 0) *c = 0ull;
}

// position of column cj in row k's sorted columns [r0, r1), or -1
__device__ __forceinline__ int64_t find_col(const int32_t* __restrict__ col,
                                            int64_t r0, int64_t r1,
                                            int32_t cj) {
  int64_t lo = r0, hi = r1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (col[mid] < cj)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < r1 && col[lo] == cj) ? lo : -1;
}

// ILU(0) in place on a (the step values); a row holds at most 128 entries,
// two per lane.  done[] must be zero and *next zero at launch.
__global__ __launch_bounds__(64) void ilu0_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    double* a, const int32_t* __restrict__ diag, int64_t N, int32_t* done,
    unsigned long long* next, DevStatus* st) {
  const int lane = threadIdx.x;
  for (;;) {
    const int64_t i = claim(next, lane);
    if (i >= N) break;
    const int64_t s0 = row_ptr[i];
    const int len = (int)(row_ptr[i + 1] - s0);
    const int32_t c0 = lane < len ? col[s0 + lane] : INT32_MAX;
    const int32_t c1 = lane + 64 < len ? col[s0 + lane + 64] : INT32_MAX;
    double v0 = lane < len ? a[s0 + lane] : 0.0;
    double v1 = lane + 64 < len ? a[s0 + lane + 64] : 0.0;
    if (diag[i] < 0 && lane == 0) report(st, ORBF_EINVAL, (int)i);
    // entries left of the diagonal come first (columns ascend)
    const int nl = __popcll(__ballot(c0 < i)) + __popcll(__ballot(c1 < i));
    for (int p = 0; p < nl; ++p) {
      const int32_t k = __builtin_amdgcn_readlane(p < 64 ? c0 : c1, p & 63);
      if (!wait_flag_uniform(done + k) && lane == 0)
        report(st, ORBF_EINTERNAL, (int)i);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const int dk = diag[k];
      const int64_t r0 = row_ptr[k], r1 = row_ptr[k + 1];
      const double akk = dk >= 0 ? a[r0 + dk] : 0.0;
      const double pv = p < 64 ? v0 : v1;
      const int lo = __builtin_amdgcn_readlane(__double2loint(pv), p & 63);
      const int hi = __builtin_amdgcn_readlane(__double2hiint(pv), p & 63);
      if (akk == 0.0 && lane == 0) report(st, ORBF_ESINGULAR, (int)k);
      const double m = __hiloint2double(hi, lo) / akk;
      if (lane == (p & 63)) {
        if (p < 64)
          v0 = m;
        else
          v1 = m;
      }
      // a_ij -= m a_kj for the entries right of position p
      if (lane > p && lane < len) {
        const int64_t u = find_col(col, r0 + dk + 1, r1, c0);
        if (u >= 0) v0 = fma(-m, a[u], v0);
      }
      if (lane + 64 > p && lane + 64 < len) {
        const int64_t u = find_col(col, r0 + dk + 1, r1, c1);
        if (u >= 0) v1 = fma(-m, a[u], v1);
      }
    }
    if (lane < len) a[s0 + lane] = v0;
    if (lane + 64 < len) a[s0 + lane + 64] = v1;
    // every lane raises the (same) flag: no lane-0 branch at the loop's end
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(done + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// y = L^{-1} b (forward, unit lower) or x = U^{-1} y (backward): rows
// claimed in increasing (forward) or decreasing order.
template <bool FWD>
__global__ __launch_bounds__(64) void trsv_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const double* __restrict__ lu, const int32_t* __restrict__ diag,
    int64_t N, const double* __restrict__ in, double* out, int32_t* done,
    unsigned long long* next, DevStatus* st) {
  const int lane = threadIdx.x;
  for (;;) {
    const int64_t c = claim(next, lane);
    if (c >= N) break;
    const int64_t i = FWD ? c : N - 1 - c;
    const int64_t s0 = row_ptr[i];
    const int len = (int)(row_ptr[i + 1] - s0);
    double acc = 0.0;
    bool ok = true;
    for (int t = lane; t < len; t += 64) {
      const int32_t j = col[s0 + t];
      if (FWD ? j < i : j > i) {
        ok &= wait_flag_lane(done + j);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        acc = fma(lu[s0 + t], out[j], acc);
      }
    }
    if (__ballot(!ok) && lane == 0) report(st, ORBF_EINTERNAL, (int)i);
    // butterfly: every lane ends with the full sum and writes the same
    // value and flag, so no lane-0 branch closes the loop body
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    double v = in[i] - acc;
    if (!FWD) {
      const int dk = diag[i];
      v = dk >= 0 ? v / lu[s0 + dk] : v;
    }
    out[i] = v;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(done + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(256) void ilu_zero_flags_kernel(int32_t* f,
                                                             int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    f[i] = 0;
}

// resident wavefronts at most: claims happen only in running waves, so any
// grid drains; this keeps idle waves from queueing behind the spinning ones
unsigned ilu_grid(orbf_ctx* ctx, int64_t N) {
  const int64_t want = (int64_t)ctx->num_cus * 8;
  return (unsigned)(N < want ? N : want);
}

}  // namespace

size_t ilu_scratch_bytes(int64_t N) {
  // diagonal positions, flags, a counter, one intermediate vector
  return (size_t)N * 8 + 64 + (size_t)N * 8;
}

namespace {

struct IluScratch {
  int32_t* diag;
  int32_t* flags;
  unsigned long long* next;
  double* tmp;
};

IluScratch ilu_scratch(orbf_ctx* ctx, int64_t N, orbf_status* st) {
  auto* w = (char*)scratch(ctx, B_ILU, ilu_scratch_bytes(N), st);
  IluScratch r{nullptr, nullptr, nullptr, nullptr};
  if (*st) return r;
  r.diag = (int32_t*)w;
  r.flags = (int32_t*)(w + (size_t)N * 4);
  r.next = (unsigned long long*)(w + (size_t)N * 8);
  r.tmp = (double*)(w + (size_t)N * 8 + 64);
  return r;
}

}  // namespace

orbf_status launch_ilu0(orbf_ctx* ctx, int64_t N, const int64_t* row_ptr,
                        const int32_t* col, const double* val,
                        const uint8_t* row_kind, double alpha, double beta,
                        double* lu) {
  orbf_status st = ORBF_OK;
  const IluScratch w = ilu_scratch(ctx, N, &st);
  if (st) return st;
  hipStream_t s = ctx->stream;
  const int64_t rb = (N + 15) / 16;
  hipLaunchKernelGGL(step_values_kernel,
                     dim3((unsigned)(rb < 65536 ? rb : 65536)), dim3(256), 0,
                     s, row_ptr, col, val, row_kind, alpha, beta, N, lu,
                     w.diag, w.flags);
  hipLaunchKernelGGL(ilu_zero_counter_kernel, dim3(1), dim3(64), 0, s, w.next);
  hipLaunchKernelGGL(ilu0_kernel, dim3(ilu_grid(ctx, N)), dim3(64), 0, s,
                     row_ptr, col, lu, w.diag, N, w.flags, w.next,
                     ctx->status);
  return hip_check(ctx, hipGetLastError(), "ILU(0)");
}

orbf_status launch_ilu_prepare(orbf_ctx* ctx, int64_t N,
                               const int64_t* row_ptr, const int32_t* col) {
  orbf_status st = ORBF_OK;
  const IluScratch w = ilu_scratch(ctx, N, &st);
  if (st) return st;
  const int64_t rb = (N + 15) / 16;
  hipLaunchKernelGGL(diag_pos_kernel, dim3((unsigned)(rb < 65536 ? rb : 65536)),
                     dim3(256), 0, ctx->stream, row_ptr, col, N, w.diag);
  return hip_check(ctx, hipGetLastError(), "ILU(0) diagonal");
}

// out = U^{-1} L^{-1} in (launch_ilu_prepare first); in and out distinct
orbf_status launch_ilu_apply(orbf_ctx* ctx, int64_t N, const int64_t* row_ptr,
                             const int32_t* col, const double* lu,
                             const double* in, double* out) {
  orbf_status st = ORBF_OK;
  const IluScratch w = ilu_scratch(ctx, N, &st);
  if (st) return st;
  hipStream_t s = ctx->stream;
  const int64_t vb = (N + 255) / 256;
  const dim3 gz((unsigned)(vb < 65536 ? vb : 65536));
  const dim3 gs(ilu_grid(ctx, N));
  hipLaunchKernelGGL(ilu_zero_flags_kernel, gz, dim3(256), 0, s, w.flags, N);
  hipLaunchKernelGGL(ilu_zero_counter_kernel, dim3(1), dim3(64), 0, s, w.next);
  hipLaunchKernelGGL(trsv_kernel<true>, gs, dim3(64), 0, s, row_ptr, col, lu,
                     w.diag, N, in, w.tmp, w.flags, w.next, ctx->status);
  hipLaunchKernelGGL(ilu_zero_flags_kernel, gz, dim3(256), 0, s, w.flags, N);
  hipLaunchKernelGGL(ilu_zero_counter_kernel, dim3(1), dim3(64), 0, s, w.next);
  hipLaunchKernelGGL(trsv_kernel<false>, gs, dim3(64), 0, s, row_ptr, col, lu,
                     w.diag, N, w.tmp, out, w.flags, w.next, ctx->status);
  return hip_check(ctx, hipGetLastError(), "ILU(0) solve");
}

}  // namespace orbf
