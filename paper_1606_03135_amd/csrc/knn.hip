// Stencils: the n nearest nodes of every node, itself first (Sec. 2 and
// Sec. 4.1, I^k_1 = k), ordered by the key (squared distance, index).
//
// The paper names a kd-tree; on the GPU a uniform bucket grid serves better:
//   1. bbox + grid parameters (cell side ~ the expected stencil radius),
//   2. per-node cell ids and per-cell counts (atomics), exclusive scan,
//   3. scatter into a cell-sorted copy of the coordinates,
//   4. one wavefront per query scans the (2R+1)^d block of cells around its
//      own cell, R = 1, 2, ... until the n-th key is provably inside the
//      scanned block; the candidates are staged in LDS through a 64-bin
//      histogram on d^2 that isolates the n nearest plus a few extra, which
//      are then ranked exactly by (d^2, index).
// Queries run in cell order so that neighbouring wavefronts reuse the same
// candidate cells from L2.
#include <math.h>

#include "orbf_internal.hpp"

namespace orbf {

namespace {

constexpr int kWaves = 4;    // wavefronts per block in the query kernel
constexpr int kBins = 64;    // histogram bins (one per lane)
constexpr int kKeep = 256;   // LDS capacity for ranked candidates per wave
constexpr int kLevels = 6;   // histogram refinements before giving up

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(256) void bbox_partial_kernel(
    const double* __restrict__ x, int64_t N, int d, double* __restrict__ part,
    DevStatus* __restrict__ st) {
  __shared__ double s[6][256];
  bool bad = false;
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * 256) {
    for (int a = 0; a < d; ++a) {
      double v = x[i * d + a];
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

// Histogram classification of a squared distance across refinement levels:
// returns -1 (below the selected bin: keep), 0 (in the selected bin of the
// deepest level), +1 (discard).  `lev` levels are fully decided; the
// deepest level's bin is returned through *bin.
struct Levels {
  double lo[kLevels];
  double scale[kLevels];
  int star[kLevels];
  int n;  // number of decided levels
};

__device__ __forceinline__ int bin_of(double d2, double lo, double scale) {
  double t = (d2 - lo) * scale;
  int b = (t > 0.0) ? (int)t : 0;
  return b >= kBins ? kBins - 1 : b;
}

// Classify d2 (already known < cut) against the decided levels.  Returns
// -1 keep, +1 drop, 0 undecided (then *bin holds the bin at the next level).
__device__ __forceinline__ int classify(double d2, const Levels& L, double lo,
                                        double scale, int* bin) {
#pragma unroll
  for (int k = 0; k < kLevels; ++k) {
    if (k < L.n) {
      int b = bin_of(d2, L.lo[k], L.scale[k]);
      if (b < L.star[k]) return -1;
      if (b > L.star[k]) return 1;
    }
  }
  *bin = bin_of(d2, lo, scale);
  return 0;
}

__global__ __launch_bounds__(256) void knn_query_kernel(
    const double* __restrict__ xs, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ cstart, const GridParams* __restrict__ gpp,
    int64_t N, int d, int n, int32_t* __restrict__ knn,
    double* __restrict__ rho2, DevStatus* __restrict__ st) {
  __shared__ int hist[kWaves][kBins];
  __shared__ double kd[kWaves][kKeep];
  __shared__ int kj[kWaves][kKeep];
  __shared__ int kcnt[kWaves];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const GridParams g = *gpp;

  for (int64_t qs = (int64_t)blockIdx.x * kWaves + w; qs < N;
       qs += (int64_t)gridDim.x * kWaves) {
    const int32_t qi = perm[qs];
    const double q0 = xs[qs * d], q1 = xs[qs * d + 1];
    const double q2 = (d == 3) ? xs[qs * d + 2] : 0.0;
    const double qv[3] = {q0, q1, q2};
    int cq[3];
    cq[0] = cell_coord(q0, g, 0);
    cq[1] = cell_coord(q1, g, 1);
    cq[2] = (d == 3) ? cell_coord(q2, g, 2) : 0;
    bool dup = false;

    for (int R = 1;; ++R) {
      int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
      bool whole = true;
      double b = INFINITY;
      for (int a = 0; a < d; ++a) {
        lo[a] = max(cq[a] - R, 0);
        hi[a] = min(cq[a] + R, g.nc[a] - 1);
        if (cq[a] - R > 0) {
          b = fmin(b, qv[a] - (g.lo[a] + (double)(cq[a] - R) * g.s));
          whole = false;
        }
        if (cq[a] + R < g.nc[a] - 1) {
          b = fmin(b, (g.lo[a] + (double)(cq[a] + R + 1) * g.s) - qv[a]);
          whole = false;
        }
      }
      // unscanned nodes are at least b away; the margin absorbs rounding in
      // d^2, in b and in the cell assignment
      const double cut = whole ? g.diag2 : b * b * (1.0 - 1e-9);

      // walk the candidate rows (runs of cells contiguous along x)
      auto for_candidates = [&](auto&& f) {
        for (int z = lo[2]; z <= hi[2]; ++z)
          for (int y = lo[1]; y <= hi[1]; ++y) {
            const int64_t crow = ((int64_t)z * g.nc[1] + y) * g.nc[0];
            const int64_t s0 = cstart[crow + lo[0]];
            const int64_t s1 = cstart[crow + hi[0] + 1];
            for (int64_t t = s0 + lane; t < s1; t += 64) f(t);
          }
      };
      auto dist = [&](int64_t t) {
        const double* p = xs + t * d;
        return exact_sqdist(q0, q1, q2, p[0], p[1], d == 3 ? p[2] : 0.0, d);
      };

      Levels L;
      L.n = 0;
      double hlo = 0.0, hscale = (double)kBins / cut;
      int base = 0;  // candidates below every selected bin so far
      int star = 0, kept = 0;
      bool ok = false;
      for (int lev = 0; lev <= kLevels; ++lev) {
        hist[w][lane] = 0;
        wave_sync();
        int cnt = 0;
        for_candidates([&](int64_t t) {
          double d2 = dist(t);
          if (lev == 0 && d2 == 0.0 && t != qs) dup = true;
          if (!(d2 < cut)) return;
          int bn;
          if (classify(d2, L, hlo, hscale, &bn) == 0) {
            atomicAdd(&hist[w][bn], 1);
            ++cnt;
          }
        });
        wave_sync();
        if (lev == 0) {
          if (wave_sum(cnt) < n) break;  // block too small: grow R
        }
        // inclusive prefix over the bins (bin = lane)
        int c = hist[w][lane];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          int u = __shfl_up(c, o, 64);
          if (lane >= o) c += u;
        }
        const int need = n - base;
        const unsigned long long m = __ballot(c >= need);
        star = __ffsll((long long)m) - 1;
        const int cum_star = __shfl(c, star, 64);
        const int below = (star > 0) ? __shfl(c, star - 1, 64) : 0;
        kept = base + cum_star;
        if (kept <= kKeep) {
          ok = true;
          break;
        }
        if (lev == kLevels) break;
        // refine inside the selected bin
        L.lo[lev] = hlo;
        L.scale[lev] = hscale;
        L.star[lev] = star;
        L.n = lev + 1;
        base += below;
        const double wbin = 1.0 / hscale;
        hlo = hlo + (double)star * wbin;
        hscale = (double)kBins / wbin;
      }
      if (!ok) {
        bool small = false;
        if (L.n == 0) {
          // fewer than n candidates inside the provable radius
          small = true;
        }
        if (small) {
          if (whole) {  // cannot happen with N >= n; guard the loop
            if (lane == 0) report(st, ORBF_EINTERNAL, qi);
            break;
          }
          continue;
        }
        if (lane == 0) report(st, ORBF_EINTERNAL, qi);
        break;
      }

      // stage the kept candidates in LDS
      if (lane == 0) kcnt[w] = 0;
      wave_sync();
      for_candidates([&](int64_t t) {
        double d2 = dist(t);
        if (!(d2 < cut)) return;
        int bn;
        int cl = classify(d2, L, hlo, hscale, &bn);
        if (cl < 0 || (cl == 0 && bn <= star)) {
          int slot = atomicAdd(&kcnt[w], 1);
          if (slot < kKeep) {
            kd[w][slot] = d2;
            kj[w][slot] = perm[t];
          }
        }
      });
      wave_sync();
      const int K = min(kcnt[w], kKeep);
      // exact rank by (d2, index); ranks below n are the stencil
      for (int t = lane; t < K; t += 64) {
        const double dt = kd[w][t];
        const int jt = kj[w][t];
        int r = 0;
        for (int u = 0; u < K; ++u) {
          const double du = kd[w][u];
          const int ju = kj[w][u];
          r += (du < dt) || (du == dt && ju < jt);
        }
        if (r < n) {
          knn[(int64_t)qi * n + r] = jt;
          if (r == n - 1) rho2[qi] = dt;
        }
      }
      wave_sync();
      break;
    }
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
  if (st) return st;
  double alpha = 0.9;
  if (const char* e = getenv("ORBF_KNN_ALPHA")) alpha = atof(e);
  hipStream_t s = ctx->stream;
  const unsigned g1 = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(bbox_partial_kernel, dim3(nblk), dim3(256), 0, s, xyz, N,
                     d, part, ctx->status);
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
  const int64_t qblocks = (N + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(knn_query_kernel,
                     dim3((unsigned)(qblocks < (1 << 20) ? qblocks : (1 << 20))),
                     dim3(64 * kWaves), 0, s, xs, perm, cstart, gp, N, d, n,
                     knn, rho2, ctx->status);
  return hip_check(ctx, hipGetLastError(), "knn");
}

}  // namespace orbf
