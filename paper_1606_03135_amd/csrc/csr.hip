// Sparse DM in CSR (Sec. 4.1: L(R^k_i, I^k_j) = W^{phi,k}_{j,i}).
// Row pointers are a prefix sum of the row lengths (n for every row with an
// owner).  Each stencil's n indices (all distinct) are ranked once, by the
// wavefront of the row that owns itself (its center, or an explicit row);
// then one thread per entry writes each (index, weight) pair at its rank.
#include "orbf_internal.hpp"

namespace orbf {

namespace {

__global__ __launch_bounds__(256) void row_len_kernel(
    const int32_t* __restrict__ owner, int64_t N, int n,
    int32_t* __restrict__ len) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < N) len[e] = owner[e] >= 0 ? n : 0;
}

// Rank of every stencil position within its stencil, once per stencil.
// A wavefront reads the owners of 64 consecutive nodes in one load and
// ranks, one after the other, the stencils of those that own themselves
// (centers, explicit rows); lane q takes position q (and q + 64).
template <int PER_LANE>
__global__ __launch_bounds__(256) void stencil_rank_kernel(
    const int32_t* __restrict__ knn, const int32_t* __restrict__ owner,
    int64_t N, int n, uint8_t* __restrict__ crank) {
  const int lane = threadIdx.x & 63;
  const int64_t e0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64;
  if (e0 >= N) return;  // whole wavefront
  const int64_t me = e0 + lane;
  unsigned long long self = __ballot(me < N && owner[me] == me);
  while (self) {
    const int64_t e = e0 + __ffsll((long long)self) - 1;
    self &= self - 1;
    int32_t idx[PER_LANE];
#pragma unroll
    for (int h = 0; h < PER_LANE; ++h) {
      const int q = lane + 64 * h;
      idx[h] = q < n ? knn[e * n + q] : INT32_MAX;
    }
    int rank[PER_LANE];
#pragma unroll
    for (int h = 0; h < PER_LANE; ++h) rank[h] = 0;
#pragma unroll
    for (int g = 0; g < PER_LANE; ++g) {
      for (int s = 0; s < 64; ++s) {
        const int32_t v = __shfl(idx[g], s, 64);
#pragma unroll
        for (int h = 0; h < PER_LANE; ++h) rank[h] += v < idx[h];
      }
    }
#pragma unroll
    for (int h = 0; h < PER_LANE; ++h)
      if (lane + 64 * h < n) crank[e * n + lane + 64 * h] = (uint8_t)rank[h];
  }
}

// Row e: the owner's stencil at the recorded ranks, with row e's weights.
// A block step covers rpb = 256 / n whole rows, one thread per entry, so
// loads of W and stores of col/val stream through contiguous rows.
__global__ __launch_bounds__(256) void csr_scatter_kernel(
    const int32_t* __restrict__ knn, const int32_t* __restrict__ owner,
    const double* __restrict__ W, const uint8_t* __restrict__ crank,
    int64_t N, int n, int rpb, const int64_t* __restrict__ row_ptr,
    int32_t* __restrict__ col, double* __restrict__ val) {
  const int t = threadIdx.x;
  const int rl = t / n, q = t - rl * n;
  if (rl >= rpb) return;
  for (int64_t e = (int64_t)blockIdx.x * rpb + rl; e < N;
       e += (int64_t)gridDim.x * rpb) {
    const int32_t o = owner[e];
    if (o < 0 || o >= N) continue;
    const int64_t so = (int64_t)o * n + q;
    const int64_t at = row_ptr[e] + crank[so];
    col[at] = knn[so];
    val[at] = W[e * n + q];
  }
}

// y = L x for a CSR matrix: sixteen lanes per row, a grid-stride over rows;
// each row's products are summed in a fixed order (lane partials, then a
// butterfly over the sixteen lanes), so y is deterministic.
__global__ __launch_bounds__(256) void spmv_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ x, int64_t N,
    double* __restrict__ y) {
  const int pl = threadIdx.x & 15;
  for (int64_t e = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4; e < N;
       e += (int64_t)gridDim.x * 16) {
    const int64_t s0 = row_ptr[e], s1 = row_ptr[e + 1];
    double acc = 0.0;
    for (int64_t t = s0 + pl; t < s1; t += 16) acc = fma(val[t], x[col[t]], acc);
    for (int o = 1; o < 16; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (pl == 0) y[e] = acc;
  }
}

}  // namespace

orbf_status launch_spmv(orbf_ctx* ctx, int64_t N, const int64_t* row_ptr,
                        const int32_t* col, const double* val,
                        const double* x, double* y) {
  const int64_t want = (N + 15) / 16;
  const unsigned blocks = (unsigned)(want < 65536 ? want : 65536);
  hipLaunchKernelGGL(spmv_kernel, dim3(blocks), dim3(256), 0, ctx->stream,
                     row_ptr, col, val, x, N, y);
  return hip_check(ctx, hipGetLastError(), "spmv");
}

orbf_status launch_csr(orbf_ctx* ctx, int64_t N, int n, const int32_t* knn,
                       const int32_t* owner, const double* W,
                       int64_t* row_ptr, int32_t* col, double* val) {
  orbf_status st = ORBF_OK;
  auto* len = (int32_t*)scratch(ctx, B_INDEG, (size_t)(N + 1) * 4, &st);
  auto* crank = (uint8_t*)scratch(ctx, B_CSR_RANK, (size_t)N * n, &st);
  if (st) return st;
  hipStream_t s = ctx->stream;
  const unsigned g = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(row_len_kernel, dim3(g), dim3(256), 0, s, owner, N, n, len);
  st = exclusive_scan_i32_to_i64(ctx, len, N, row_ptr);
  if (st) return st;
  // one wavefront per 64 nodes, four per block
  const dim3 rgrid((unsigned)((N + 255) / 256));
  if (n <= 64)
    hipLaunchKernelGGL(stencil_rank_kernel<1>, rgrid, dim3(256), 0, s, knn,
                       owner, N, n, crank);
  else
    hipLaunchKernelGGL(stencil_rank_kernel<2>, rgrid, dim3(256), 0, s, knn,
                       owner, N, n, crank);
  const int rpb = 256 / n;  // n <= 128
  const int64_t steps = (N + rpb - 1) / rpb;
  const dim3 grid((unsigned)(steps < (1 << 16) ? steps : (1 << 16)));
  hipLaunchKernelGGL(csr_scatter_kernel, grid, dim3(256), 0, s, knn, owner, W,
                     crank, N, n, rpb, row_ptr, col, val);
  return hip_check(ctx, hipGetLastError(), "csr");
}

}  // namespace orbf
