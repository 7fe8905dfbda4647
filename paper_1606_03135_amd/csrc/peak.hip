// Measurement helper (not a step of the method): the FP64 vector FMA rate
// this device actually reaches, reported beside the published peak that
// roofline fractions are taken against.
//
// Every thread runs eight independent FMA chains (enough to cover the FMA
// latency at full occupancy) for `iters` iterations on values that stay
// bounded and normal, and stores their sum so nothing is dead code.  The
// grid is 8 wavefronts per CU (2 per SIMD) times a multiple of the CU count.
#include "orbf_internal.hpp"

namespace orbf {
namespace {

__global__ __launch_bounds__(256) void fma_peak_kernel(double* out,
                                                       int iters) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  double a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = 1.0 + 1e-3 * (double)((t + i) & 255);
  const double x = 0.999999940395355, y = 5.9604644775390625e-8;
#pragma unroll 8
  for (int k = 0; k < iters; ++k) {
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = fma(a[i], x, y);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += a[i];
  out[t] = s;
}

}  // namespace
}  // namespace orbf

using namespace orbf;

extern "C" orbf_status orbf_measure_fp64_fma(orbf_ctx* ctx,
                                             double* tflops) {
  if (!ctx || !tflops) return ORBF_EINVAL;
  hipSetDevice(ctx->device);
  const int blocks = ctx->num_cus * 2 * 16;  // 2 blocks of 4 waves per CU, x16
  const int iters = 1 << 14;
  orbf_status st = ORBF_OK;
  auto* out = (double*)scratch(ctx, B_GERSH, (size_t)blocks * 256 * 8, &st);
  if (st) return st;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(ctx, ORBF_EHIP, "event");
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(ctx, ORBF_EHIP, "event");
  }
  float best = 1e30f;
  for (int rep = 0; rep < 4; ++rep) {  // the first launch warms up
    hipEventRecord(e0, ctx->stream);
    hipLaunchKernelGGL(fma_peak_kernel, dim3(blocks), dim3(256), 0,
                       ctx->stream, out, iters);
    hipEventRecord(e1, ctx->stream);
    hipEventSynchronize(e1);
    float ms = 0.0f;
    hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0 && ms < best) best = ms;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  const double flops = 2.0 * 8.0 * (double)iters * (double)blocks * 256.0;
  *tflops = flops / ((double)best * 1e-3) / 1e12;
  return hip_check(ctx, hipGetLastError(), "FP64 FMA rate");
}
