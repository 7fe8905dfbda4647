// Local RBF-FD weights for the larger saddle systems, 72 < K <= 144: one
// workgroup of four wavefronts per stencil center (Sec. 4.1, eqs.
// rbffd_linsys, orbffd_eq, orbffd_rhs).
//
// The elimination of the one-wavefront register kernel on a 16 x 16 thread
// grid: thread t = r + 16 c holds rows 16 ii + r (ii < L) and columns
// 16 jj + c (jj < L: A_hat; jj = L + jp: right-hand side 16 jp + c) of
// [A_hat | B_hat], K <= 16 L.  Column group c is one 16-lane DPP row inside
// wavefront c / 4, so the pivot search of step k reduces a 32-bit key
// (|a| high bits | local row) with DPP inside the wavefront that owns
// column k; that wavefront publishes the pivot slot through LDS (barrier 1);
// the pivot row and the multipliers follow (barrier 2); every thread then
// updates its L x (L + PL - kb) register block.  Rows stay in place (an
// activity mask retires pivot rows) and the sweep is Gauss-Jordan, so the
// row slot pivoted at step j ends holding u_jj x_j and no back substitution
// follows.  Padded slots (>= K) are inactive and hold zeros.
#include <math.h>

#include "orbf_internal.hpp"
#include "weights_common.hpp"

namespace orbf {

namespace {

// max of a 32-bit key over each 16-lane DPP row
__device__ __forceinline__ uint32_t group16_max(uint32_t k) {
  k = umax(k, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)k, 0xB1, 0xF, 0xF, false));
  k = umax(k, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)k, 0x4E, 0xF, 0xF, false));
  k = umax(k, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)k, 0x141, 0xF, 0xF, false));
  k = umax(k, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)k, 0x140, 0xF, 0xF, false));
  return k;
}

constexpr int kG = 16;            // thread grid side
constexpr int kThreads = kG * kG;  // four wavefronts
constexpr int kZeroPivot = 1 << 16;

template <int L, int PL>
__global__ __launch_bounds__(256, 2) void weights_wg_kernel(WeightsParams P) {
  constexpr int LC = L + PL;
  constexpr int S = kG * L;
  extern __shared__ double dyn_s[];  // psi | L psi | powers
  __shared__ double xi_s[3 * S];
  __shared__ int cols_s[S];
  __shared__ int8_t ex_s[3 * 36];
  __shared__ double ubuf[kG * LC];  // pivot row [c][jj]
  __shared__ double lbuf[kG * L];   // multipliers [r][ii]
  __shared__ double dinv[S];
  __shared__ int srank[S];
  __shared__ int piv_s[S];
  __shared__ int ncol_s;

  const int t0 = threadIdx.x;
  const int wave = t0 >> 6;
  const int n = P.n, K = P.K, d = P.d, M = P.M, m = P.m, op = P.op;
  const int l1 = P.l + 1;
  double* psi_s = dyn_s;
  double* lpsi_s = psi_s + n * M;
  double* pw_s = lpsi_s + kG * PL * M;
  for (int q = t0; q < 3 * M; q += kThreads) ex_s[q] = P.ex[q];
  // eliminations write only values in [0, K) here, so with this start no
  // rank read below can index out of range
  for (int q = t0; q < S; q += kThreads) srank[q] = 0;

  const bool explicit_rows = P.rows != nullptr;
  const int64_t total = explicit_rows ? P.n_rows : *P.n_centers;
  for (int64_t ci = blockIdx.x; ci < total; ci += gridDim.x) {
    // the thread index, opaque to the compiler in every iteration: values
    // derived from it are recomputed per stencil instead of being hoisted
    // out of the stencil loop and held (spilled) across it
    int t = t0;
    __asm__ volatile("" : "+v"(t));
    const int lane = t & 63;
    const int32_t ck = explicit_rows ? P.rows[ci] : P.centers[ci];
    if ((uint32_t)ck >= (uint64_t)P.N) {
      if (t == 0) report(P.st, ORBF_EINVAL, ck);
      continue;
    }
    const int32_t* stn = P.knn + (int64_t)ck * n;
    bool bad = false;
    for (int q = t; q < n; q += kThreads)
      bad |= (uint32_t)stn[q] >= (uint64_t)P.N;
    if (__syncthreads_or(bad)) {
      if (t == 0) report(P.st, ORBF_EINVAL, ck);
      continue;
    }
    double nrm[3] = {0.0, 0.0, 0.0};
    if (explicit_rows && op == ORBF_OP_NEUMANN) {
      nrm[0] = P.normals[ci * d];
      nrm[1] = P.normals[ci * d + 1];
      if (d == 3) nrm[2] = P.normals[ci * d + 2];
    }
    op_axis(op, nrm);
    if (wave == 0) {
      int ncol = 0;
      if (explicit_rows) {
        if (lane == 0) cols_s[0] = 0;
        ncol = 1;
      } else {
        for (int q0 = 0; q0 < n; q0 += 64) {
          const int q = q0 + lane;
          const bool mine = q < n && P.owner[stn[q]] == ck;
          const unsigned long long b = __ballot(mine);
          if (mine) cols_s[ncol + __popcll(b & ((1ull << lane) - 1ull))] = q;
          ncol += __popcll(b);
        }
      }
      if (lane == 0) ncol_s = ncol;
    }
    const double r2c = P.rho2[ck];
    const double rho = sqrt(r2c);
    const double inv_rho = 1.0 / rho;
    const double* xc = P.xyz + (int64_t)ck * d;
    for (int q = t; q < n; q += kThreads) {
      const double* xq = P.xyz + (int64_t)stn[q] * d;
      xi_s[3 * q] = (xq[0] - xc[0]) * inv_rho;
      xi_s[3 * q + 1] = (xq[1] - xc[1]) * inv_rho;
      xi_s[3 * q + 2] = (d == 3) ? (xq[2] - xc[2]) * inv_rho : 0.0;
    }
    __syncthreads();
    const int ncol = ncol_s;
    for (int q = t; q < 3 * n; q += kThreads) {
      const double v = xi_s[q];
      double* pw = pw_s + q * l1;
      double acc = 1.0;
      for (int e = 0; e < l1; ++e) {
        pw[e] = acc;
        acc *= v;
      }
    }
    __syncthreads();
    for (int q = t; q < n * M; q += kThreads) {
      const int qi = q / M, s = q - qi * M;
      psi_s[q] = monomial_pw(pw_s + 3 * qi * l1, l1, ex_s + 3 * s);
    }
    const double sinv = op_unscale(op, r2c, rho);

    for (int cb = 0; cb < ncol; cb += kG * PL) {
      const int nb = min(kG * PL, ncol - cb);
      // opaque again per pass, and the thread's grid coordinates derived
      // here: nothing thread-dependent is carried across the elimination
      // (K = 95 on 200k nodes: 4.50 -> 3.26 ms)
      int t = t0;
      __asm__ volatile("" : "+v"(t));
      const int lane = t & 63;
      const int r = t & 15, c = t >> 4;
      __syncthreads();
      for (int q = t; q < nb * M; q += kThreads) {
        const int e = q / M, s = q - e * M;
        lpsi_s[q] = monomial_op_pw(pw_s + 3 * cols_s[cb + e] * l1, l1,
                                   ex_s + 3 * s, op, nrm[0], nrm[1], nrm[2]);
      }
      __syncthreads();
      // ---- assemble [A_hat | B_hat] straight into the registers ----
      // (unrolled; a runtime loop through a per-thread LDS strip measured
      // 10.0 against 9.65 ms for K = 140 on a 200k ball)
      double a[L][LC];
      sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
        constexpr int ii = decltype(iic)::value;
        const int i = kG * ii + r;
        const bool ri = i < n;
        const double xi0 = ri ? xi_s[3 * i] : 0.0;
        const double xi1 = ri ? xi_s[3 * i + 1] : 0.0;
        const double xi2 = ri ? xi_s[3 * i + 2] : 0.0;
        sfor<0, LC>([&](auto jjc) __attribute__((always_inline)) {
          constexpr int jj = decltype(jjc)::value;
          double v = 0.0;
          if constexpr (jj < L) {
            const int j = kG * jj + c;
            if (i < n && j < n) {
              const double dx = xi0 - xi_s[3 * j], dy = xi1 - xi_s[3 * j + 1];
              const double dz = xi2 - xi_s[3 * j + 2];
              v = phs(dx * dx + dy * dy + dz * dz, m);
            } else if (i < n && j < K) {
              v = psi_s[i * M + (j - n)];
            } else if (j < n && i < K) {
              v = psi_s[j * M + (i - n)];
            }
          } else {
            const int e = kG * (jj - L) + c;
            if (e < nb && i < K) {
              const double* pe = xi_s + 3 * cols_s[cb + e];
              if (i < n) {
                const double dx = pe[0] - xi0, dy = pe[1] - xi1;
                const double dz = pe[2] - xi2;
                v = phs_op(dx, dy, dz, dx * dx + dy * dy + dz * dz, m, d, op,
                           nrm[0], nrm[1], nrm[2]);
              } else {
                v = lpsi_s[e * M + (i - n)];
              }
            }
          }
          a[ii][jj] = v;
        });
      });
      // ---- partial pivoting, rows in place, Gauss-Jordan sweep ----
      uint32_t act[L];
      sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
        constexpr int ii = decltype(iic)::value;
        act[ii] = (kG * ii + r < K) ? 0x7FFFFF80u : 0u;
      });
      bool singular = false;
      sfor<0, L>([&](auto kbc) __attribute__((always_inline)) {
        constexpr int kb = decltype(kbc)::value;
#pragma clang loop unroll(disable)
        for (int cc = 0; cc < kG; ++cc) {
          const int k = kG * kb + cc;
          if (k >= K) break;
          uint32_t key0 = 0;
          sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
            constexpr int ii = decltype(iic)::value;
            const uint32_t hi = (uint32_t)__double2hiint(a[ii][kb]);
            key0 = umax(key0, (hi & act[ii]) | (uint32_t)ii);
          });
          const uint32_t gm = group16_max(key0);
          if (wave == (cc >> 2)) {  // the wavefront holding column k
            const int base = 16 * (cc & 3);
            const uint32_t kmax = __builtin_amdgcn_readlane(gm, base);
            const unsigned long long who =
                __ballot(key0 == kmax) & (0xFFFFull << base);
            const int rp = (__ffsll((long long)who) - 1 - base) & 15;
            const int zero = ((kmax & 0x7FFFFF80u) == 0u) ? kZeroPivot : 0;
            if (lane == 0) piv_s[k] = (16 * (int)(kmax & 15u) + rp) | zero;
          }
          __syncthreads();
          const int pv = __builtin_amdgcn_readfirstlane(piv_s[k]);
          if (pv & kZeroPivot) singular = true;
          const int piv = pv & 0xFFFF;
          const int iip = piv >> 4, rp = piv & 15;
          sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
            constexpr int ii = decltype(iic)::value;
            act[ii] = (ii == iip && r == rp) ? 0u : act[ii];
          });
          sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
            constexpr int ii = decltype(iic)::value;
            if (iip == ii) {
              __asm__ volatile("; wg pivot row out %0" ::"i"(ii));
              if (r == rp) {
                sfor<kb, LC>([&](auto jjc) __attribute__((always_inline)) {
                  constexpr int jj = decltype(jjc)::value;
                  ubuf[c * LC + jj] = a[ii][jj];
                });
              }
            }
          });
          // multipliers of column k, the pivot row's written as zero
          if (c == cc) {
            sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
              constexpr int ii = decltype(iic)::value;
              lbuf[r * L + ii] = (ii == iip && r == rp) ? 0.0 : a[ii][kb];
            });
          }
          if (t == 0) srank[piv] = k;
          __syncthreads();
          const double upiv = ubuf[cc * LC + kb];
          if (!(upiv != 0.0)) singular = true;
          const double dk = singular ? 0.0 : recip(upiv);
          if (t == 0) dinv[k] = dk;
          double u[LC], lv[L];
          sfor<kb, LC>([&](auto jjc) __attribute__((always_inline)) {
            constexpr int jj = decltype(jjc)::value;
            u[jj] = ubuf[c * LC + jj];
          });
          sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
            constexpr int ii = decltype(iic)::value;
            lv[ii] = lbuf[r * L + ii];
          });
          sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
            constexpr int ii = decltype(iic)::value;
            const double lm = lv[ii] * dk;
            sfor<kb, LC>([&](auto jjc) __attribute__((always_inline)) {
              constexpr int jj = decltype(jjc)::value;
              a[ii][jj] = fma(-lm, u[jj], a[ii][jj]);
            });
          });
        }
      });
      __syncthreads();
      // Every step of a nonsingular system pivots a row still active, so
      // each of the K slots gets exactly one rank.  A singular system may
      // rank one slot twice and leave another with a stale rank; its slots
      // are then mapped to themselves, which writes each of its weights
      // exactly once, as NaN (and so makes Lambda NaN too).  The flag comes
      // from LDS, so the branch is uniform over the workgroup.
      if (singular) {
        for (int q = t; q < S; q += kThreads) srank[q] = q;
        __syncthreads();
      }
      int rank[L];
      double rdk[L];
      sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
        constexpr int ii = decltype(iic)::value;
        const bool live = kG * ii + r < K;
        rank[ii] = live ? srank[kG * ii + r] : 1 << 20;
        rdk[ii] = live ? dinv[rank[ii]] : 0.0;
      });
      if (singular && t == 0) report(P.st, ORBF_ESINGULAR, ck);
      // ---- unscale, write rows, Lebesgue values ----
      sfor<0, PL>([&](auto jpc) __attribute__((always_inline)) {
        constexpr int jp = decltype(jpc)::value;
        const int e = kG * jp + c;
        const bool live = e < nb;
        const int32_t row = live ? stn[cols_s[cb + e]] : 0;
        double lam = 0.0;
        sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
          constexpr int ii = decltype(iic)::value;
          const int j = rank[ii];
          if (live && j < n) {
            const double w =
                singular ? NAN : (a[ii][L + jp] * rdk[ii]) * sinv;
            P.W[(int64_t)row * n + j] = w;
            lam += fabs(w);
          }
        });
        lam += __shfl_xor(lam, 1, 64);
        lam += __shfl_xor(lam, 2, 64);
        lam += __shfl_xor(lam, 4, 64);
        lam += __shfl_xor(lam, 8, 64);
        if (live && r == 0) {
          if (P.lebesgue) P.lebesgue[row] = lam;
          if (explicit_rows && P.owner_out) P.owner_out[row] = row;
        }
      });
    }
    __syncthreads();
  }
}

template <int L, int PL>
bool launch_wg(orbf_ctx* ctx, const WeightsParams& P, int64_t work) {
  const size_t dyn = ((size_t)P.n * P.M + (size_t)kG * PL * P.M +
                      (size_t)3 * P.n * (P.l + 1)) * sizeof(double);
  static bool attr_set = false;  // set once, outside any graph capture
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)weights_wg_kernel<L, PL>,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            96 * 1024) != hipSuccess)
      return false;
    attr_set = true;
  }
  if (dyn > 96 * 1024) return false;
  const int64_t grid = work;  // one workgroup per possible stencil
  hipLaunchKernelGGL((weights_wg_kernel<L, PL>), dim3((unsigned)grid),
                     dim3(kThreads), dyn, ctx->stream, P);
  return true;
}

}  // namespace

// Launch the four-wavefront kernel for 72 < K <= 144 (plain rows, no
// acceptance mode); returns false when no variant applies.
bool launch_weights_wg(orbf_ctx* ctx, const WeightsParams& P, int64_t work) {
  if (P.M > 36 || P.K > 16 * 9 || P.accept != nullptr) return false;
  constexpr int PL = 1;
  if (work <= 0) return true;
  if (P.K <= 16 * 5) return launch_wg<5, PL>(ctx, P, work);
  if (P.K <= 16 * 6) return launch_wg<6, PL>(ctx, P, work);
  if (P.K <= 16 * 7) return launch_wg<7, PL>(ctx, P, work);
  if (P.K <= 16 * 8) return launch_wg<8, PL>(ctx, P, work);
  return launch_wg<9, PL>(ctx, P, work);
}

}  // namespace orbf
