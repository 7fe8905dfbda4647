// Stencils: the n nearest nodes of every node, itself first (Sec. 2 and
// Sec. 4.1, I^k_1 = k), ordered by the key (squared distance, index).
//
// The paper names a kd-tree; on the GPU a uniform bucket grid serves better:
//   1. bbox + grid parameters (cell side ~ the expected stencil radius),
//   2. per-node cell ids and per-cell counts (atomics), exclusive scan,
//   3. scatter into a cell-sorted copy of the coordinates,
//   4. one wavefront per query scans the (2R+1)^d block of cells around its
//      own cell, R = 1, 2, ... until the n-th key is provably inside the
//      scanned block; candidates below a threshold are compacted into LDS in
//      one pass and ranked exactly by (d^2, index).
// Each wavefront takes a run of consecutive queries in cell order: they
// share candidate cells (L2 reuse) and nearly the same stencil radius, which
// seeds the threshold of the next query.
#include <math.h>

#include "orbf_internal.hpp"

namespace orbf {

namespace {

// wavefronts per block in the query kernel (1M-node ball, kNN phase:
// 2.058-2.063 ms at 1, 2.085-2.094 at 2, 2.135-2.145 at 4, 2.44 at 8; at
// one per block, 2.048 ms with five wavefronts per SIMD, 2.30 with four,
// 2.107 with six)
constexpr int kWaves = 1;
constexpr int kKeep = 256;   // LDS capacity for ranked candidates per wave
// consecutive (cell-ordered) queries per wave: 8 in 3D, 4 in 2D (with the
// branch-free sort; 1M-node ball: 2.18 ms at 8, 2.20 at 16, 2.48 at 32;
// 100k-node disk: 0.208 ms at 4, 0.220 at 8); halved until the launch has
// 4096 wavefronts, down to one query per wave for sets of under 4096 nodes
__host__ __device__ constexpr int run_length(int d) { return d == 2 ? 4 : 8; }
// first threshold: kGrow x the previous query's n-th squared distance; small
// enough that about n (1 + 1.5 (kGrow - 1)) candidates pass, so most sets fit
// one key per lane, large enough that few queries need a second pass
// (1M-node ball, n = 50: 3.01 ms at 1.10, 3.04 at 1.12, 3.10 at 1.08, 3.16
// at 1.15, 3.56 at 1.20)
constexpr double kGrow = 1.10;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double readlane_f64_knn(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// (d, j) < (e, k) in the stencil order: squared distance, then index
__device__ __forceinline__ bool key_less(double d, int j, double e, int k) {
  return (d < e) | ((d == e) & (j < k));  // bitwise: no branches
}

// Value of lane ^ STRIDE.  Strides 1 and 2 are quad permutations and 8 is a
// rotation by 8 within each 16-lane row, all DPP moves (VALU latency); the
// others go through the LDS crossbar.  (Stride 4 from two rotations and a
// select measured no faster than the crossbar.)
template <int STRIDE>
__device__ __forceinline__ int xor_lane(int v) {
  if constexpr (STRIDE == 1)
    return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
  else if constexpr (STRIDE == 2)
    return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
  else if constexpr (STRIDE == 8)
    return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);
  else
    return __shfl_xor(v, STRIDE, 64);
}

template <int STRIDE>
__device__ __forceinline__ double xor_lane_f64(double v) {
  const int lo = xor_lane<STRIDE>(__double2loint(v));
  const int hi = xor_lane<STRIDE>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// One compare-exchange stage of a bitonic sort over the elements
// i = lane + 64 h held in registers (d[h], j[h]); partners at i ^ STRIDE
// (STRIDE < 64: another lane, same register).
template <int SIZE, int STRIDE, int NR>
__device__ __forceinline__ void bitonic_stage(double (&d)[NR], int (&j)[NR],
                                              int lane) {
#pragma unroll
  for (int h = 0; h < NR; ++h) {
    const int i = lane + 64 * h;
    const double pd = xor_lane_f64<STRIDE>(d[h]);
    const int pj = xor_lane<STRIDE>(j[h]);
    const bool keep_min = ((i & STRIDE) == 0) == ((i & SIZE) == 0);
    // keys are distinct except the identical padding keys, so "the
    // partner's key is the smaller" decides both directions; bitwise
    // operators keep it free of branches (a short-circuit form with one
    // comparison per direction compiled to about 30 exec-mask scalar
    // instructions and several branches per stage: 1M-node ball kNN
    // 2.86 -> 2.31 ms, the same stencils)
    const bool lt = (pd < d[h]) | ((pd == d[h]) & (pj < j[h]));
    const bool take = keep_min == lt;
    d[h] = take ? pd : d[h];
    j[h] = take ? pj : j[h];
  }
}

template <int SIZE, int STRIDE, int NR>
__device__ __forceinline__ void bitonic_merge(double (&d)[NR], int (&j)[NR],
                                              int lane) {
  if constexpr (STRIDE >= 1) {
    if constexpr (STRIDE == 64) {  // partner in the other register
      const bool take = key_less(d[1], j[1], d[0], j[0]);  // SIZE == 128
      const double t0 = d[0];
      const int u0 = j[0];
      d[0] = take ? d[1] : d[0];
      j[0] = take ? j[1] : j[0];
      d[1] = take ? t0 : d[1];
      j[1] = take ? u0 : j[1];
    } else {
      bitonic_stage<SIZE, STRIDE, NR>(d, j, lane);
    }
    bitonic_merge<SIZE, STRIDE / 2, NR>(d, j, lane);
  }
}

// Ascending sort of the 64 NR keys; padding keys are (inf, INT_MAX).
template <int NR, int SIZE = 2>
__device__ __forceinline__ void bitonic_sort(double (&d)[NR], int (&j)[NR],
                                             int lane) {
  if constexpr (SIZE <= 64 * NR) {
    bitonic_merge<SIZE, SIZE / 2, NR>(d, j, lane);
    bitonic_sort<NR, SIZE * 2>(d, j, lane);
  }
}

// Stencil of one query from `base` compacted candidates: sort, write the
// first n indices and squared distances, return the n-th squared distance
// (wave-uniform).
template <int NR>
__device__ __forceinline__ double rank_sorted(const double* kd, const int* kj,
                                              int base, int n, int lane,
                                              int32_t* knn_row,
                                              double* d2_row,
                                              double* rho2_q) {
  double d[NR];
  int j[NR];
#pragma unroll
  for (int h = 0; h < NR; ++h) {
    const int t = lane + 64 * h;
    d[h] = t < base ? kd[t] : INFINITY;
    j[h] = t < base ? kj[t] : 0x7FFFFFFF;
  }
  bitonic_sort<NR>(d, j, lane);
  double nth = 0.0;
#pragma unroll
  for (int h = 0; h < NR; ++h) {
    const int t = lane + 64 * h;
    if (t < n) {
      knn_row[t] = j[h];
      d2_row[t] = d[h];
    }
    if (t == n - 1) *rho2_q = d[h];
    const int src = (n - 1) - 64 * h;
    if (src >= 0 && src < 64) nth = readlane_f64_knn(d[h], src);
  }
  return nth;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The dimension is a template argument, so the axis loop unrolls and each
// thread keeps several grid-stride steps' loads in flight.
template <int D>
__global__ __launch_bounds__(256) void bbox_partial_kernel(
    const double* __restrict__ x, int64_t N, double* __restrict__ part,
    DevStatus* __restrict__ st) {
  __shared__ double s[6][256];
  bool bad = false;
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  const int64_t stride = (int64_t)gridDim.x * 256;
#pragma unroll 4
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += stride) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double v = x[i * D + a];
      bad |= !isfinite(v);
      mn[a] = fmin(mn[a], v);
      mx[a] = fmax(mx[a], v);
    }
  }
  if (bad) report(st, ORBF_EINVAL, -1);  // NaN or infinite coordinate
  for (int a = 0; a < 3; ++a) {
    s[a][threadIdx.x] = mn[a];
    s[3 + a][threadIdx.x] = mx[a];
  }
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = fmin(s[a][threadIdx.x], s[a][threadIdx.x + off]);
        s[3 + a][threadIdx.x] =
            fmax(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + off]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int a = 0; a < 6; ++a) part[blockIdx.x * 6 + a] = s[a][0];
}

// Finishes the bbox and fixes the grid: cell side alpha * r_est where
// r_est is the radius holding n nodes at the bounding-box mean density,
// enlarged if needed so that at most `cap` cells exist.
__global__ __launch_bounds__(256) void grid_params_kernel(
    const double* __restrict__ part, int nblk, int64_t N, int d, int n,
    int64_t cap, double alpha, GridParams* __restrict__ gp,
    DevStatus* __restrict__ st) {
  __shared__ double s[6][256];
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nblk; b += 256)
    for (int a = 0; a < 3; ++a) {
      v[a] = fmin(v[a], part[b * 6 + a]);
      v[3 + a] = fmax(v[3 + a], part[b * 6 + 3 + a]);
    }
  for (int a = 0; a < 6; ++a) s[a][threadIdx.x] = v[a];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = fmin(s[a][threadIdx.x], s[a][threadIdx.x + off]);
        s[3 + a][threadIdx.x] =
            fmax(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + off]);
      }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  GridParams g;
  double ext[3] = {0, 0, 0}, vol = 1.0, diag2 = 0.0;
  bool finite = true;
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = (a < d) ? s[a][0] : 0.0;
    ext[a] = (a < d) ? s[3 + a][0] - s[a][0] : 0.0;
    if (!isfinite(ext[a])) finite = false;
  }
  if (!finite) {
    report(st, ORBF_EINVAL, -1);  // NaN or infinite coordinates
    for (int a = 0; a < 3; ++a) {
      g.lo[a] = 0;
      g.nc[a] = 1;
    }
    g.s = g.inv_s = 1.0;
    g.diag2 = INFINITY;
    g.ncell = 1;
    *gp = g;
    return;
  }
  double emax = 0.0;
  for (int a = 0; a < d; ++a) emax = fmax(emax, ext[a]);
  if (emax <= 0.0) emax = 1.0;
  for (int a = 0; a < d; ++a) {
    vol *= (ext[a] > 0.0 ? ext[a] : emax * 1e-6);
    diag2 += ext[a] * ext[a];
  }
  const double vd = (d == 2) ? M_PI : 4.0 * M_PI / 3.0;
  double cell = alpha * pow((double)n * vol / ((double)N * vd), 1.0 / d);
  if (!(cell > 0.0)) cell = emax;
  // grow the cell until the grid has at most `cap` cells (product taken in
  // floating point so that a tiny first guess cannot overflow)
  int64_t ncell = 1;
  for (int it = 0; it < 4096; ++it) {
    double prod = 1.0;
    for (int a = 0; a < d; ++a) prod *= floor(ext[a] / cell) + 1.0;
    if (prod <= (double)cap) break;
    cell *= 1.25;
  }
  for (int a = 0; a < 3; ++a) {
    const int64_t c = (a < d) ? (int64_t)floor(ext[a] / cell) + 1 : 1;
    g.nc[a] = (int)c;
    ncell *= c;
  }
  g.s = cell;
  g.inv_s = 1.0 / cell;
  g.diag2 = diag2 * 1.001 + 1e-300;
  g.ncell = (int)ncell;
  *gp = g;
}

__device__ __forceinline__ int cell_coord(double v, const GridParams& g,
                                          int a) {
  int c = (int)((v - g.lo[a]) * g.inv_s);
  c = c < 0 ? 0 : c;
  return c >= g.nc[a] ? g.nc[a] - 1 : c;
}

// Cell index of coordinate v on axis a, clamped to the grid, for any finite
// v (the same truncation as cell_coord, so a node whose coordinate lies in
// [u, w] has its cell in [box_cell(u), box_cell(w)]).
__device__ __forceinline__ int box_cell(double v, const GridParams& g, int a) {
  double t = (v - g.lo[a]) * g.inv_s;
  t = fmin(fmax(t, 0.0), (double)(g.nc[a] - 1));
  return (int)t;
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* p, int64_t n,
                                                        int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256)
    p[i] = v;
}

__global__ __launch_bounds__(256) void cell_count_kernel(
    const double* __restrict__ x, int64_t N, int d,
    const GridParams* __restrict__ gp, int32_t* __restrict__ cell_of,
    int32_t* __restrict__ rank, int32_t* __restrict__ count) {
  const GridParams g = *gp;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    int c0 = cell_coord(x[i * d], g, 0), c1 = cell_coord(x[i * d + 1], g, 1);
    int c2 = (d == 3) ? cell_coord(x[i * d + 2], g, 2) : 0;
    int c = (c2 * g.nc[1] + c1) * g.nc[0] + c0;
    cell_of[i] = c;
    rank[i] = atomicAdd(&count[c], 1);
  }
}

__global__ __launch_bounds__(256) void cell_scatter_kernel(
    const double* __restrict__ x, int64_t N, int d,
    const int32_t* __restrict__ cell_of, const int32_t* __restrict__ rank,
    const int64_t* __restrict__ start, int32_t* __restrict__ perm,
    double* __restrict__ xs) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    int64_t pos = start[cell_of[i]] + rank[i];
    perm[pos] = (int32_t)i;
    for (int a = 0; a < d; ++a) xs[pos * d + a] = x[i * d + a];
  }
}

// One wavefront per query.  The scanned block is the box of cells around the
// ball of the expected stencil radius (the previous query's, x sqrt(kGrow)),
// so most queries prove their stencil in the first block (rings of whole
// cells around the query's own cell, 3^d and then 5^d: 3.01 ms against
// 2.89 ms on the 1M-node ball).  Candidates with d^2 < T are compacted into
// LDS in one pass and ordered exactly by (d^2, index) with an in-register
// bitonic sort (64 or 128 keys); T starts from the previous query's n-th
// distance (queries run in cell order, so neighbours have nearly the same
// stencil radius) and is corrected by bisection when the pass keeps fewer
// than n or more than 128 candidates.  T never exceeds the squared distance
// to the boundary of the scanned block, so the result is exact: every node
// outside the block is farther than every kept one.
__global__ __launch_bounds__(64 * kWaves)
__attribute__((amdgpu_waves_per_eu(5))) void knn_query_kernel(
    const double* __restrict__ xs, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ cstart, const GridParams* __restrict__ gpp,
    int64_t N, int d, int n, int run, int32_t* __restrict__ knn,
    double* __restrict__ rho2, double* __restrict__ d2,
    DevStatus* __restrict__ st) {
  __shared__ double kd[kWaves][kKeep];
  __shared__ int kj[kWaves][kKeep];
  __shared__ double kth[kWaves];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const GridParams g = *gpp;
  double est = 0.0;  // previous query's n-th squared distance (0: none)
  const int64_t q_begin = ((int64_t)blockIdx.x * kWaves + w) * run;
  const int64_t q_end = min(q_begin + run, N);

  for (int64_t qs = q_begin; qs < q_end; ++qs) {
    const int32_t qi = perm[qs];
    const double q0 = xs[qs * d], q1 = xs[qs * d + 1];
    const double q2 = (d == 3) ? xs[qs * d + 2] : 0.0;
    bool dup = false;
    bool done = false;

    // the block of cells that holds the ball of radius `rad` around the
    // query; rad starts from the expected stencil radius and grows by 1.5x
    // while the block cannot prove n neighbours
    double rad = sqrt(est > 0.0 ? est * kGrow : g.s * g.s);
    for (int grow = 0; !done && grow < 64; ++grow, rad *= 1.5) {
      const int lo0 = box_cell(q0 - rad, g, 0), hi0 = box_cell(q0 + rad, g, 0);
      const int lo1 = box_cell(q1 - rad, g, 1), hi1 = box_cell(q1 + rad, g, 1);
      const int lo2 = (d == 3) ? box_cell(q2 - rad, g, 2) : 0;
      const int hi2 = (d == 3) ? box_cell(q2 + rad, g, 2) : 0;
      bool whole = true;
      double b = INFINITY;
      if (lo0 > 0) { b = fmin(b, q0 - (g.lo[0] + (double)lo0 * g.s)); whole = false; }
      if (hi0 < g.nc[0] - 1) { b = fmin(b, (g.lo[0] + (double)(hi0 + 1) * g.s) - q0); whole = false; }
      if (lo1 > 0) { b = fmin(b, q1 - (g.lo[1] + (double)lo1 * g.s)); whole = false; }
      if (hi1 < g.nc[1] - 1) { b = fmin(b, (g.lo[1] + (double)(hi1 + 1) * g.s) - q1); whole = false; }
      if (d == 3) {
        if (lo2 > 0) { b = fmin(b, q2 - (g.lo[2] + (double)lo2 * g.s)); whole = false; }
        if (hi2 < g.nc[2] - 1) { b = fmin(b, (g.lo[2] + (double)(hi2 + 1) * g.s) - q2); whole = false; }
      }
      // unscanned nodes are at least b away; the margin absorbs rounding in
      // d^2, in b and in the cell assignment
      const double cut = whole ? g.diag2 : b * b * (1.0 - 1e-9);

      double tlo = 0.0, thi = cut;  // bisection bracket for T
      int shrink = 0;
      // first guess: kGrow x the previous query's n-th squared distance, or
      // the grid's expected one (the cell side is ~ the stencil radius)
      const double guess = est > 0.0 ? est * kGrow : g.s * g.s;
      double T = guess < cut ? guess : cut;
      for (int it = 0; it < 64; ++it) {
        // one pass: compact every candidate with d^2 < T.  A row of cells
        // (fixed y, z) is contiguous in cell order and holds a few dozen
        // nodes, so each half-wavefront scans one row: two rows per step.
        int base = 0;
        const int ny = hi1 - lo1 + 1;
        const int rows = ny * (hi2 - lo2 + 1);
        const int half = lane >> 5, hl = lane & 31;
        // (y, z) of this half's row, advanced by two rows per step without
        // a division (ny >= 1, so two wraps at most)
        int y = lo1 + half, z = lo2;
        if (y > hi1) { y -= ny; ++z; }
        for (int pr = 0; pr < rows; pr += 2) {
          const int row = pr + half;
          int64_t s0 = 0, s1 = 0;
          if (row < rows) {
            const int64_t crow = ((int64_t)z * g.nc[1] + y) * g.nc[0];
            s0 = cstart[crow + lo0];
            s1 = cstart[crow + hi0 + 1];
          }
          y += 2;
          if (y > hi1) { y -= ny; ++z; }
          if (y > hi1) { y -= ny; ++z; }
          for (int64_t t = s0 + hl; __ballot(t < s1) != 0ull; t += 32) {
            bool keep = false;
            double d2 = 0.0;
            int32_t pj = 0;
            if (t < s1) {
              const double* p = xs + t * d;
              // the node index is loaded with the coordinates, so one wait
              // covers both (loaded only for kept candidates it was a
              // second dependent round trip per step)
              pj = perm[t];
              d2 = exact_sqdist(q0, q1, q2, p[0], p[1], d == 3 ? p[2] : 0.0, d);
              if (d2 == 0.0 && t != qs) dup = true;
              keep = d2 < T;
            }
            const unsigned long long m = __ballot(keep);
            if (keep) {
              const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
              if (pos < kKeep) {
                kd[w][pos] = d2;
                kj[w][pos] = pj;
              }
            }
            base += __popcll(m);
          }
        }
        if (base < n) {
          if (T >= cut) break;  // too few inside the provable radius: grow R
          tlo = T;
          T = (thi < cut) ? 0.5 * (T + thi) : fmin(cut, T * 1.6);
          continue;
        }
        // more than the in-register sort holds: shrink T a few times, then
        // (ties on a lattice) fall back to pairwise ranking of <= kKeep
        if ((base > 128 && shrink < 8) || base > kKeep) {
          ++shrink;
          thi = T;
          T = 0.5 * (tlo + T);
          continue;
        }
        // exact order by (d^2, index); the first n are the stencil
        wave_sync();
        if (base <= 128) {
          est = (base <= 64)
                    ? rank_sorted<1>(kd[w], kj[w], base, n, lane,
                                     knn + (int64_t)qi * n,
                                     d2 + (int64_t)qi * n, rho2 + qi)
                    : rank_sorted<2>(kd[w], kj[w], base, n, lane,
                                     knn + (int64_t)qi * n,
                                     d2 + (int64_t)qi * n, rho2 + qi);
          wave_sync();
          done = true;
          break;
        }
        for (int t = lane; t < base; t += 64) {
          const double dt = kd[w][t];
          const int jt = kj[w][t];
          int r = 0;
          for (int u = 0; u < base; ++u) {
            const double du = kd[w][u];
            const int ju = kj[w][u];
            r += (du < dt) || (du == dt && ju < jt);
          }
          if (r < n) {
            knn[(int64_t)qi * n + r] = jt;
            d2[(int64_t)qi * n + r] = dt;
            if (r == n - 1) {
              rho2[qi] = dt;
              kth[w] = dt;  // n-th distance, the next query's first guess
            }
          }
        }
        wave_sync();
        est = kth[w];
        done = true;
        break;
      }
      if (!done && whole) {  // cannot happen with N >= n finite nodes
        if (lane == 0) report(st, ORBF_EINTERNAL, qi);
        break;
      }
      if (!done && T < cut) {  // bisection did not converge (ties)
        if (lane == 0) report(st, ORBF_EINTERNAL, qi);
        break;
      }
    }
    if (!done && lane == 0) report(st, ORBF_EINTERNAL, qi);
    if (__ballot(dup) && lane == 0) report(st, ORBF_EDUPLICATE, qi);
  }
}

}  // namespace

orbf_status launch_knn(orbf_ctx* ctx, const double* xyz, int64_t N, int d,
                       int n, int32_t* knn, double* rho2) {
  orbf_status st = ORBF_OK;
  const int64_t cap = N + 64;
  const int nblk = (int)((N + 255) / 256 < 1024 ? (N + 255) / 256 : 1024);
  auto* gp = (GridParams*)scratch(ctx, B_GRID_PARAMS, sizeof(GridParams), &st);
  auto* part = (double*)scratch(ctx, B_PARTIAL, (size_t)nblk * 6 * 8, &st);
  auto* cell_of = (int32_t*)scratch(ctx, B_CELL_OF, (size_t)N * 4, &st);
  auto* rank = (int32_t*)scratch(ctx, B_CELL_RANK, (size_t)N * 4, &st);
  auto* count = (int32_t*)scratch(ctx, B_FLAGS, (size_t)(cap + 1) * 4, &st);
  auto* cstart = (int64_t*)scratch(ctx, B_CELL_START, (size_t)(cap + 2) * 8, &st);
  auto* perm = (int32_t*)scratch(ctx, B_PERM, (size_t)N * 4, &st);
  auto* xs = (double*)scratch(ctx, B_XS, (size_t)N * d * 8, &st);
  // squared distance of every stencil member, kept for the covering, in
  // node order like knn (row i: node i's stencil), so that the covering
  // reads it as a stream
  auto* d2 = (double*)scratch(ctx, B_KNN_D2, (size_t)N * n * 8, &st);
  if (st) return st;
  const double alpha = 0.9;  // cell side in units of the mean stencil radius
  hipStream_t s = ctx->stream;
  const unsigned g1 = (unsigned)((N + 255) / 256);
  if (d == 2)
    hipLaunchKernelGGL(bbox_partial_kernel<2>, dim3(nblk), dim3(256), 0, s,
                       xyz, N, part, ctx->status);
  else
    hipLaunchKernelGGL(bbox_partial_kernel<3>, dim3(nblk), dim3(256), 0, s,
                       xyz, N, part, ctx->status);
  hipLaunchKernelGGL(grid_params_kernel, dim3(1), dim3(256), 0, s, part, nblk,
                     N, d, n, cap, alpha, gp, ctx->status);
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((cap + 256) / 256)),
                     dim3(256), 0, s, count, cap + 1, 0);
  hipLaunchKernelGGL(cell_count_kernel, dim3(g1), dim3(256), 0, s, xyz, N, d,
                     gp, cell_of, rank, count);
  st = exclusive_scan_i32_to_i64(ctx, count, cap + 1, cstart);
  if (st) return st;
  hipLaunchKernelGGL(cell_scatter_kernel, dim3(g1), dim3(256), 0, s, xyz, N, d,
                     cell_of, rank, cstart, perm, xs);
  // shorter runs for small node sets, so that they still fill the chip
  int run = run_length(d);
  while (run > 1 && (N + run - 1) / run < 4096) run >>= 1;
  const int64_t per_block = (int64_t)kWaves * run;
  const int64_t qblocks = (N + per_block - 1) / per_block;
  hipLaunchKernelGGL(knn_query_kernel, dim3((unsigned)qblocks),
                     dim3(64 * kWaves), 0, s, xs, perm, cstart, gp, N, d, n,
                     run, knn, rho2, d2, ctx->status);
  ctx->d2_cache = {xyz, knn, N, d, n, d2};
  return hip_check(ctx, hipGetLastError(), "knn");
}

}  // namespace orbf
