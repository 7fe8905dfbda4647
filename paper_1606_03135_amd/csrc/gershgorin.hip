// Gershgorin disks of the DM rows (Sec. 4.2.1): row k's disk has center
// L_kk and radius g_k = sum_{j != k} |L_kj|, the row's L-Lebesgue value
// minus |L_kk|; every eigenvalue of L lies in the union of the disks, so no
// eigenvalue has a positive real part unless some disk reaches Re > 0.
//
// Sixteen lanes per row, a grid-stride over rows; each block writes its
// partial summary (rightmost edge L_kk + g_k, leftmost edge L_kk - g_k,
// number of rows whose edge passes 0) and one workgroup combines the
// partials in a fixed order, so the result does not depend on scheduling.
#include "orbf_internal.hpp"

namespace orbf {

namespace {

constexpr int kGershBlocks = 2048;

__global__ __launch_bounds__(256) void gersh_rows_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, int64_t N, double* __restrict__ diag,
    double* __restrict__ radius, double* __restrict__ part) {
  __shared__ double s_right[16], s_left[16], s_count[16];
  const int pl = threadIdx.x & 15, grp = threadIdx.x >> 4;
  double right = -INFINITY, left = INFINITY, count = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 16 + grp; e < N;
       e += (int64_t)gridDim.x * 16) {
    const int64_t s0 = row_ptr[e], s1 = row_ptr[e + 1];
    double dg = 0.0, off = 0.0;
    for (int64_t t = s0 + pl; t < s1; t += 16) {
      const double v = val[t];
      if (col[t] == e)
        dg = v;
      else
        off += fabs(v);
    }
    // the row's sixteen lanes: one holds the diagonal, all hold off-sums
    for (int o = 1; o < 16; o <<= 1) {
      dg += __shfl_xor(dg, o, 64);
      off += __shfl_xor(off, o, 64);
    }
    if (pl == 0) {
      if (diag) diag[e] = dg;
      if (radius) radius[e] = off;
      right = fmax(right, dg + off);
      left = fmin(left, dg - off);
      count += (dg + off > 0.0) ? 1.0 : 0.0;
    }
  }
  if (pl == 0) {
    s_right[grp] = right;
    s_left[grp] = left;
    s_count[grp] = count;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = -INFINITY, l = INFINITY, c = 0.0;
    for (int g = 0; g < 16; ++g) {
      r = fmax(r, s_right[g]);
      l = fmin(l, s_left[g]);
      c += s_count[g];
    }
    part[3 * blockIdx.x] = r;
    part[3 * blockIdx.x + 1] = l;
    part[3 * blockIdx.x + 2] = c;
  }
}

__global__ __launch_bounds__(64) void gersh_final_kernel(
    const double* __restrict__ part, int nparts, double* __restrict__ out) {
  const int lane = threadIdx.x;
  double r = -INFINITY, l = INFINITY, c = 0.0;
  for (int i = lane; i < nparts; i += 64) {
    r = fmax(r, part[3 * i]);
    l = fmin(l, part[3 * i + 1]);
    c += part[3 * i + 2];
  }
  for (int o = 32; o >= 1; o >>= 1) {
    r = fmax(r, __shfl_xor(r, o, 64));
    l = fmin(l, __shfl_xor(l, o, 64));
    c += __shfl_xor(c, o, 64);  // integers below 2^53: exact in any order
  }
  if (lane == 0) {
    out[0] = r;
    out[1] = l;
    out[2] = c;
  }
}

}  // namespace

size_t gershgorin_scratch_bytes() { return (size_t)kGershBlocks * 3 * 8; }

orbf_status launch_gershgorin(orbf_ctx* ctx, int64_t N,
                              const int64_t* row_ptr, const int32_t* col,
                              const double* val, double* diag, double* radius,
                              double* summary) {
  orbf_status st = ORBF_OK;
  auto* part =
      (double*)scratch(ctx, B_GERSH, gershgorin_scratch_bytes(), &st);
  if (st) return st;
  const int64_t want = (N + 15) / 16;
  const int blocks = (int)(want < kGershBlocks ? want : kGershBlocks);
  hipLaunchKernelGGL(gersh_rows_kernel, dim3(blocks), dim3(256), 0,
                     ctx->stream, row_ptr, col, val, N, diag, radius, part);
  hipLaunchKernelGGL(gersh_final_kernel, dim3(1), dim3(64), 0, ctx->stream,
                     part, blocks, summary);
  return hip_check(ctx, hipGetLastError(), "gershgorin");
}

}  // namespace orbf
