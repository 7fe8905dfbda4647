// Exclusive prefix sums used by the grid, the covering and the CSR row
// pointers; out[n] receives the total.  Up to kOneBlock items: one block of
// 1024 threads walks the array in chunks with a carry (one launch).  Larger:
// block-local scans of 1024 items, a recursive scan of the block totals, and
// a uniform add.
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

// out[j] += offs[tile of j]; the last block also writes the total out[n]
__global__ __launch_bounds__(kScanThreads) void scan_add_kernel(
    int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ offs) {
  const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
  const int64_t o = offs[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t j = i + (int64_t)k * kScanThreads;
    if (j < n) out[j] += o;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = offs[gridDim.x];
}

constexpr int kBlockThreads = 1024;
constexpr int kBlockChunk = kBlockThreads * kScanItems;
constexpr int64_t kOneBlock = 4 * kBlockChunk;

// Exclusive scan of n <= kOneBlock items by one block, chunk by chunk: each
// thread sums kScanItems consecutive items, the per-thread sums are scanned
// within each wavefront by shuffles and across the 16 wavefronts by the
// first one, and the chunk total carries into the next chunk.
template <class T>
__global__ __launch_bounds__(kBlockThreads) void scan_block_kernel(
    const T* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
  __shared__ int64_t wsum[kBlockThreads / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += kBlockChunk) {
    const int64_t i0 = base + (int64_t)t * kScanItems;
    int64_t v[kScanItems];
    int64_t local = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      v[k] = (i0 + k < n) ? (int64_t)in[i0 + k] : 0;
      local += v[k];
    }
    int64_t x = local;  // inclusive scan over the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (w == 0) {
      int64_t y = lane < kBlockThreads / 64 ? wsum[lane] : 0;
#pragma unroll
      for (int o = 1; o < kBlockThreads / 64; o <<= 1) {
        const int64_t z = __shfl_up(y, o, 64);
        if (lane >= o) y += z;
      }
      if (lane < kBlockThreads / 64) wsum[lane] = y;
    }
    __syncthreads();
    int64_t run = carry + (w ? wsum[w - 1] : 0) + x - local;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (i0 + k < n) out[i0 + k] = run;
      run += v[k];
    }
    carry += wsum[kBlockThreads / 64 - 1];
    __syncthreads();  // wsum is rewritten by the next chunk
  }
  if (t == 0) out[n] = carry;
}

// scratch layout: per recursion level, (tiles) sums followed by (tiles+1)
// scanned offsets
template <class T>
orbf_status scan_level(orbf_ctx* ctx, const T* in, int64_t n, int64_t* out,
                       int64_t* tmp) {
  if (n <= kOneBlock) {
    hipLaunchKernelGGL(scan_block_kernel<T>, dim3(1), dim3(kBlockThreads), 0,
                       ctx->stream, in, n, out);
    return hip_check(ctx, hipGetLastError(), "scan");
  }
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;  // > 1
  int64_t* sums = tmp;
  int64_t* offs = tmp + tiles;
  hipLaunchKernelGGL(scan_tile_kernel<T>, dim3((unsigned)tiles),
                     dim3(kScanThreads), 0, ctx->stream, in, n, out, sums);
  orbf_status st = scan_level<int64_t>(ctx, sums, tiles, offs,
                                       offs + tiles + 1);
  if (st) return st;
  hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)tiles),
                     dim3(kScanThreads), 0, ctx->stream, out, n, offs);
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
  return scan_level<int32_t>(ctx, in, n, out, tmp);  // n = 0: out[0] = 0
}

}  // namespace orbf
