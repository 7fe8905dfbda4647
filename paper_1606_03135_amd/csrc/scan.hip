// Exclusive prefix sums used by the grid, the covering and the CSR row
// pointers.  Three-kernel scan: block-local scans of 1024 items, a recursive
// scan of the block totals, and a uniform add.
#include "orbf_internal.hpp"

namespace orbf {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

template <class T>
__global__ __launch_bounds__(kScanThreads) void scan_tile_kernel(
    const T* __restrict__ in, int64_t n, int64_t* __restrict__ out,
    int64_t* __restrict__ tile_sums) {
  __shared__ int64_t part[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t local = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? (int64_t)in[base + k] : 0;
    local += v[k];
  }
  part[threadIdx.x] = local;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread totals
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int64_t t = (threadIdx.x >= off) ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t run = part[threadIdx.x] - local;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) tile_sums[blockIdx.x] = part[threadIdx.x];
}

__global__ __launch_bounds__(kScanThreads) void scan_add_kernel(
    int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ offs) {
  const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
  const int64_t o = offs[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t j = i + (int64_t)k * kScanThreads;
    if (j < n) out[j] += o;
  }
}

__global__ void scan_total_kernel(int64_t* __restrict__ out, int64_t n,
                                  const int64_t* __restrict__ src) {
  out[n] = src[0];
}

__global__ void set_zero_kernel(int64_t* __restrict__ out) { out[0] = 0; }

// scratch layout: per recursion level, (tiles) sums followed by (tiles+1)
// scanned offsets
template <class T>
orbf_status scan_level(orbf_ctx* ctx, const T* in, int64_t n, int64_t* out,
                       int64_t* tmp) {
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;  // n >= 1
  int64_t* sums = tmp;
  int64_t* offs = tmp + tiles;
  hipLaunchKernelGGL(scan_tile_kernel<T>, dim3((unsigned)tiles),
                     dim3(kScanThreads), 0, ctx->stream, in, n, out, sums);
  if (tiles > 1) {
    orbf_status st = scan_level<int64_t>(ctx, sums, tiles, offs,
                                         offs + tiles + 1);
    if (st) return st;
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)tiles),
                       dim3(kScanThreads), 0, ctx->stream, out, n, offs);
    hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(1), 0, ctx->stream,
                       out, n, offs + tiles);
  } else {
    hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(1), 0, ctx->stream,
                       out, n, sums);
  }
  return hip_check(ctx, hipGetLastError(), "scan");
}

}  // namespace

size_t scan_tmp_elems(int64_t n) {
  size_t total = 16;
  while (n > 0) {
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    total += 2 * (size_t)tiles + 2;
    if (tiles <= 1) break;
    n = tiles;
  }
  return total;
}

orbf_status exclusive_scan_i32_to_i64(orbf_ctx* ctx, const int32_t* in,
                                      int64_t n, int64_t* out) {
  orbf_status st = ORBF_OK;
  int64_t* tmp = (int64_t*)scratch(ctx, B_SCAN_TMP,
                                   scan_tmp_elems(n) * sizeof(int64_t), &st);
  if (st) return st;
  return exclusive_scan_i32_to_i64_tmp(ctx, in, n, out, tmp);
}

orbf_status exclusive_scan_i32_to_i64_tmp(orbf_ctx* ctx, const int32_t* in,
                                          int64_t n, int64_t* out,
                                          int64_t* tmp) {
  if (n == 0) {
    hipLaunchKernelGGL(set_zero_kernel, dim3(1), dim3(1), 0, ctx->stream, out);
    return hip_check(ctx, hipGetLastError(), "scan");
  }
  return scan_level<int32_t>(ctx, in, n, out, tmp);
}

}  // namespace orbf
