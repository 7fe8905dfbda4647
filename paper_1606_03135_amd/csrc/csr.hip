// Sparse DM in CSR (Sec. 4.1: L(R^k_i, I^k_j) = W^{phi,k}_{j,i}).
// Row pointers are a prefix sum of the row lengths (n for every row with an
// owner).  Each stencil's n indices (all distinct) are ranked once, by the
// wavefront of the row that owns itself (its center, or an explicit row);
// then one thread per entry writes each (index, weight) pair at its rank.
#include <mutex>

#include "orbf_internal.hpp"

namespace orbf {

namespace {

// Scratch of orbf_assemble_csr_noalloc: row lengths, the stencil ranks and
// the scan temporaries of one call, laid out at 256-byte offsets.  Every
// device the library runs on holds one copy until the process ends.  In
// host code this name is a stand-in, never a device address: the address
// comes from hipGetSymbolAddress (csr_noalloc_setup).
constexpr size_t kCsrScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char csr_noalloc_scratch[kCsrScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_csr_mu;
void* g_csr_scratch[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// byte offsets of the three parts for (N, n); total in *bytes
void csr_noalloc_layout(int64_t N, int n, size_t* off_rank, size_t* off_tmp,
                        size_t* bytes) {
  const size_t len = align256((size_t)(N + 1) * 4);
  const size_t rank = align256((size_t)N * (size_t)n);
  *off_rank = len;
  *off_tmp = len + rank;
  *bytes = len + rank + align256(scan_tmp_elems(N) * sizeof(int64_t));
}

__global__ __launch_bounds__(256) void row_len_kernel(
    const int32_t* __restrict__ owner, int64_t N, int n,
    int32_t* __restrict__ len) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < N) len[e] = owner[e] >= 0 ? n : 0;
}

// Rank of every stencil position within its stencil, once per stencil.
// A wavefront reads the owners of npw consecutive nodes (npw <= 64) in one
// load and ranks, one after the other, the stencils of those that own
// themselves (centers, explicit rows); lane q takes position q (and q + 64).
// Each other position's index is broadcast by readlane from a uniform lane,
// so a step is a scalar read and a compare, with no LDS round trip.
// threads of a rank block: one wavefront, so a wavefront with many
// centers holds no others' slots (1M-node ball, CSR phase: 0.363-0.364 ms
// against 0.370 at 256)
constexpr int kRankThreads = 64;

template <int PER_LANE>
__global__ __launch_bounds__(kRankThreads) void stencil_rank_kernel(
    const int32_t* __restrict__ knn, const int32_t* __restrict__ owner,
    int64_t N, int n, int npw, uint8_t* __restrict__ crank) {
  const int lane = threadIdx.x & 63;
  const int64_t e0 =
      ((int64_t)blockIdx.x * (kRankThreads / 64) + (threadIdx.x >> 6)) * npw;
  if (e0 >= N) return;  // whole wavefront
  const int64_t me = e0 + lane;
  unsigned long long self = __ballot(lane < npw && me < N && owner[me] == me);
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
      const int lim = n - 64 * g < 64 ? n - 64 * g : 64;  // uniform
      int s = 0;
      for (; s + 4 <= lim; s += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int32_t v = __builtin_amdgcn_readlane(idx[g], s + u);
#pragma unroll
          for (int h = 0; h < PER_LANE; ++h) rank[h] += v < idx[h];
        }
      }
      for (; s < lim; ++s) {
        const int32_t v = __builtin_amdgcn_readlane(idx[g], s);
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
    const int rk = crank[so];
    if (rk >= n) continue;  // a stale rank (owner o is not a ranked stencil)
    const int64_t at = row_ptr[e] + rk;
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

namespace {

// the CSR kernels on given scratch: len (N + 1 int32), crank (N * n bytes),
// scan temporaries (scan_tmp_elems(N) int64, or null: the context's)
orbf_status csr_kernels(orbf_ctx* ctx, int64_t N, int n, const int32_t* knn,
                        const int32_t* owner, const double* W,
                        int64_t* row_ptr, int32_t* col, double* val,
                        int32_t* len, uint8_t* crank, int64_t* scan_tmp) {
  orbf_status st = ORBF_OK;
  hipStream_t s = ctx->stream;
  const unsigned g = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(row_len_kernel, dim3(g), dim3(256), 0, s, owner, N, n, len);
  st = scan_tmp ? exclusive_scan_i32_to_i64_tmp(ctx, len, N, row_ptr, scan_tmp)
                : exclusive_scan_i32_to_i64(ctx, len, N, row_ptr);
  if (st) return st;
  // one wavefront per npw nodes: 64 nodes while that still
  // gives 65536 wavefronts, fewer (down to one) for smaller node sets, so
  // that each wavefront ranks few stencils in series (each one a dependent
  // load of its indices)
  int npw = 64;
  while (npw > 1 && (N + npw - 1) / npw < 65536) npw >>= 1;
  const int64_t waves = (N + npw - 1) / npw;
  constexpr int wpb = kRankThreads / 64;
  const dim3 rgrid((unsigned)((waves + wpb - 1) / wpb));
  if (n <= 64)
    hipLaunchKernelGGL(stencil_rank_kernel<1>, rgrid, dim3(kRankThreads), 0,
                       s, knn, owner, N, n, npw, crank);
  else
    hipLaunchKernelGGL(stencil_rank_kernel<2>, rgrid, dim3(kRankThreads), 0,
                       s, knn, owner, N, n, npw, crank);
  const int rpb = 256 / n;  // n <= 128
  const int64_t steps = (N + rpb - 1) / rpb;
  const dim3 grid((unsigned)(steps < (1 << 16) ? steps : (1 << 16)));
  hipLaunchKernelGGL(csr_scatter_kernel, grid, dim3(256), 0, s, knn, owner, W,
                     crank, N, n, rpb, row_ptr, col, val);
  return hip_check(ctx, hipGetLastError(), "csr");
}

}  // namespace

orbf_status launch_csr(orbf_ctx* ctx, int64_t N, int n, const int32_t* knn,
                       const int32_t* owner, const double* W,
                       int64_t* row_ptr, int32_t* col, double* val) {
  orbf_status st = ORBF_OK;
  auto* len = (int32_t*)scratch(ctx, B_INDEG, (size_t)(N + 1) * 4, &st);
  auto* crank = (uint8_t*)scratch(ctx, B_CSR_RANK, (size_t)N * n, &st);
  if (st) return st;
  return csr_kernels(ctx, N, n, knn, owner, W, row_ptr, col, val, len, crank,
                     nullptr);
}

// Once per device, with that device current (orbf_create): the device
// address of the file-scope array.  Later calls on the same device reuse it.
orbf_status csr_noalloc_setup(orbf_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return fail(ctx, ORBF_EINVAL, "device index beyond the no-alloc table");
  std::lock_guard<std::mutex> lock(g_csr_mu);
  if (!g_csr_scratch[ctx->device]) {
    void* ptr = nullptr;
    const hipError_t e =
        hipGetSymbolAddress(&ptr, HIP_SYMBOL(csr_noalloc_scratch));
    if (e != hipSuccess || !ptr)
      return hip_check(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol,
                       "hipGetSymbolAddress(csr no-alloc scratch)");
    g_csr_scratch[ctx->device] = ptr;
  }
  ctx->csr_scratch = g_csr_scratch[ctx->device];
  return ORBF_OK;
}

orbf_status launch_csr_noalloc(orbf_ctx* ctx, int64_t N, int n,
                               const int32_t* knn, const int32_t* owner,
                               const double* W, int64_t* row_ptr,
                               int32_t* col, double* val) {
  size_t off_rank, off_tmp, bytes;
  csr_noalloc_layout(N, n, &off_rank, &off_tmp, &bytes);
  if (bytes > kCsrScratchBytes)
    return fail(ctx, ORBF_EBUDGET,
                "assemble_csr_noalloc: N * (n + 4) bytes of scratch exceed "
                "its fixed 64 MiB (N * n <= about 6.4e7)");
  if (!ctx->csr_scratch)
    return fail(ctx, ORBF_EHIP, "assemble_csr_noalloc: no scratch address");
  auto* base = (unsigned char*)ctx->csr_scratch;
  return csr_kernels(ctx, N, n, knn, owner, W, row_ptr, col, val,
                     (int32_t*)base, base + off_rank,
                     (int64_t*)(base + off_tmp));
}

}  // namespace orbf
