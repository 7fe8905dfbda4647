// Local RBF-FD weights with the saddle system in FP64 matrix-core tiles
// (Sec. 4.1, eqs. rbffd_linsys, orbffd_eq, orbffd_rhs).
//
// One wavefront per stencil center, as in the register kernel, but the
// trailing updates of the elimination run on the matrix cores
// (v_mfma_f64_16x16x4f64) instead of as one vector FMA per entry and step.
//
// Layout.  [A_hat | B_hat] is held as NR x (NR + 1) tiles of 16 x 16 in the
// accumulator layout of that instruction: lane l = jc + 16 g, item t of tile
// (R, T) holds row 16 R + g + 4 t, column 16 T + jc (the last column tile
// holds up to 16 right-hand sides).  Operands: A (16 x 4) lane l holds
// A[l % 16][l / 16]; B (4 x 16) lane l holds B[l / 16][l % 16].
//
// Blocked Gauss-Jordan with row partial pivoting, rows kept in place.  For
// each panel of four columns:
//   1. the panel (every row, four columns) goes through LDS into a
//      row-per-lane copy (row i in lane i % 64, slot i / 64);
//   2. four pivot steps on that copy alone: pivot search by a wave max of a
//      32-bit key (|a| high bits of still-active rows | row), the pivot
//      row's four panel entries by readlane, multipliers m_s (zero on the
//      pivot row itself) and the update of the later panel columns;
//   3. the four steps applied to the rest of the matrix as one rank-4
//      update.  With P the four pivot rows as they stand before the panel
//      and L the unit lower 4 x 4 matrix L[s][s'] = m_s'(pivot row s), the
//      pivot rows after the steps before them are U = L^-1 P, so the four
//      sequential rank-1 updates sum to  A -= (M L^-1) P  (M: multipliers,
//      one column per step).  M L^-1 is formed per row in the row-per-lane
//      copy; the pivot rows P are read out of the tiles (one uniform case
//      per row position) -- both go through LDS into operand layout, and
//      one matrix instruction per (row tile, column tile) to the right of
//      the panel applies the update.
// Every row except the pivot row of a step is eliminated (Gauss-Jordan), so
// after the last panel the row slot pivoted at step j holds u_jj x_j in its
// right-hand-side columns and no back substitution is needed.  Columns left
// of the current panel are never read again; the tile containing the panel
// is updated whole, so its finished columns just hold rounding residue.
#include <math.h>

#include "orbf_internal.hpp"
#include "weights_common.hpp"

namespace orbf {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// max of a 32-bit key over the whole wavefront (DPP within each row of 16
// lanes, then the four row results by readlane)
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t k) {
  k = umax(k, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)k, 0xB1, 0xF, 0xF, false));
  k = umax(k, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)k, 0x4E, 0xF, 0xF, false));
  k = umax(k, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)k, 0x141, 0xF, 0xF, false));
  k = umax(k, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)k, 0x140, 0xF, 0xF, false));
  const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)k, 0);
  const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)k, 16);
  const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)k, 32);
  const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)k, 48);
  return umax(umax(a, b), umax(c, d));
}

// Pivot row `sel` = 4 R + t of the tiles (row 16 R + g_s + 4 t, held by the
// lanes with g = g_s), columns of tiles TP..NT-1, to dst[16 T + jc].
template <int NR, int NT, int TP>
__device__ __forceinline__ void pivot_row_out(const d4 (&acc)[NR][NT],
                                              int sel, bool mine, int jc,
                                              double* dst) {
#define ORBF_ROW_CASE(RR, TT)                                              \
  case 4 * RR + TT:                                                        \
    if constexpr (RR < NR) {                                               \
      /* distinct markers around each case keep the cases from being   */ \
      /* merged into one dynamically indexed read (which would move acc */ \
      /* to scratch memory)                                             */ \
      __asm__ volatile("; pivot row out %0" ::"i"(4 * RR + TT));           \
      if (mine) {                                                          \
        sfor<TP, NT>([&](auto Tc) __attribute__((always_inline)) {         \
          constexpr int T = decltype(Tc)::value;                           \
          dst[16 * T + jc] = acc[RR][T][TT];                               \
        });                                                                \
      }                                                                    \
      __asm__ volatile("; pivot row done %0" ::"i"(4 * RR + TT));          \
    }                                                                      \
    break;
  switch (sel) {
    ORBF_ROW_CASE(0, 0) ORBF_ROW_CASE(0, 1) ORBF_ROW_CASE(0, 2) ORBF_ROW_CASE(0, 3)
    ORBF_ROW_CASE(1, 0) ORBF_ROW_CASE(1, 1) ORBF_ROW_CASE(1, 2) ORBF_ROW_CASE(1, 3)
    ORBF_ROW_CASE(2, 0) ORBF_ROW_CASE(2, 1) ORBF_ROW_CASE(2, 2) ORBF_ROW_CASE(2, 3)
    ORBF_ROW_CASE(3, 0) ORBF_ROW_CASE(3, 1) ORBF_ROW_CASE(3, 2) ORBF_ROW_CASE(3, 3)
    ORBF_ROW_CASE(4, 0) ORBF_ROW_CASE(4, 1) ORBF_ROW_CASE(4, 2) ORBF_ROW_CASE(4, 3)
    default:
      break;
  }
#undef ORBF_ROW_CASE
}

template <int NR>
__global__ __launch_bounds__(64, 1) void weights_mfma_kernel(WeightsParams P) {
  static_assert(NR >= 3 && NR <= 5, "row tiles");
  constexpr int NT = NR + 1;  // column tiles: NR of A_hat, one of B_hat
  constexpr int S = 16 * NR;  // row / column slots of A_hat
  constexpr int NRHS = 16;    // right-hand sides per pass
  extern __shared__ double dyn_s[];  // L psi (16 x M), then powers
  __shared__ double xi_s[3 * S];
  __shared__ int cols_s[S];
  __shared__ int8_t ex_s[3 * 80];
  __shared__ double pbuf[4 * S];       // panel [c][row]
  __shared__ double mbuf[S * 4];       // -(M L^-1) [row][s]
  __shared__ double ubuf[4 * 16 * NT];  // pivot rows [s][column]
  __shared__ double dinv[S];
  __shared__ int srank[S];              // elimination step of each row slot
  __shared__ double strip[NT * 4 * 64];  // assembly staging, one row tile

  const int lane0 = threadIdx.x;
  const int n = P.n, K = P.K, d = P.d, M = P.M, m = P.m, op = P.op;
  double* lpsi_s = dyn_s;
  double* pw_s = lpsi_s + NRHS * M;
  for (int t = lane0; t < 3 * M; t += 64) ex_s[t] = P.ex[t];
  for (int t = lane0; t < S; t += 64) srank[t] = 0;

  const bool explicit_rows = P.rows != nullptr;
  const int64_t total = explicit_rows ? P.n_rows : *P.n_centers;
  for (int64_t ci = blockIdx.x; ci < total; ci += gridDim.x) {
    // the lane index, opaque to the compiler in every iteration, so values
    // derived from it are recomputed per stencil, not held across the loop
    int lane = lane0;
    __asm__ volatile("" : "+v"(lane));
    const int32_t ck = explicit_rows ? P.rows[ci] : P.centers[ci];
    if ((uint32_t)ck >= (uint64_t)P.N) {
      if (lane == 0) report(P.st, ORBF_EINVAL, ck);
      continue;
    }
    const int32_t* stn = P.knn + (int64_t)ck * n;
    bool bad = false;
    for (int q = lane; q < n; q += 64) bad |= (uint32_t)stn[q] >= (uint64_t)P.N;
    if (__ballot(bad)) {
      if (lane == 0) report(P.st, ORBF_EINVAL, ck);
      continue;
    }
    double nrm[3] = {0.0, 0.0, 0.0};
    if (explicit_rows && op == ORBF_OP_NEUMANN) {
      nrm[0] = P.normals[ci * d];
      nrm[1] = P.normals[ci * d + 1];
      if (d == 3) nrm[2] = P.normals[ci * d + 2];
    }
    op_axis(op, nrm);
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
    const double r2c = P.rho2[ck];
    const double rho = sqrt(r2c);
    const double inv_rho = 1.0 / rho;
    const double* xc = P.xyz + (int64_t)ck * d;
    for (int q = lane; q < n; q += 64) {
      const double* xq = P.xyz + (int64_t)stn[q] * d;
      xi_s[3 * q] = (xq[0] - xc[0]) * inv_rho;
      xi_s[3 * q + 1] = (xq[1] - xc[1]) * inv_rho;
      xi_s[3 * q + 2] = (d == 3) ? (xq[2] - xc[2]) * inv_rho : 0.0;
    }
    wsync();
    const int l1 = P.l + 1;
    for (int t = lane; t < 3 * n; t += 64) {
      const double v = xi_s[t];
      double* pw = pw_s + t * l1;  // pw_s[(3q + a) l1 + e]
      double acc = 1.0;
      for (int e = 0; e < l1; ++e) {
        pw[e] = acc;
        acc *= v;
      }
    }
    const double sinv = op_unscale(op, r2c, rho);

    for (int cb = 0; cb < ncol; cb += NRHS) {
      const int nb = min(NRHS, ncol - cb);
      int lane = lane0;
      __asm__ volatile("" : "+v"(lane));
      const int jc = lane & 15, g = lane >> 4;
      wsync();
      for (int t = lane; t < nb * M; t += 64) {
        const int e = t / M, s = t - e * M;
        lpsi_s[t] = monomial_op_pw(pw_s + 3 * cols_s[cb + e] * l1, l1,
                                   ex_s + 3 * s, op, nrm[0], nrm[1], nrm[2]);
      }
      wsync();
      // ---- assemble [A_hat | B_hat], one row tile at a time ----
      d4 acc[NR][NT];
      sfor<0, NR>([&](auto Rc) __attribute__((always_inline)) {
        constexpr int R = decltype(Rc)::value;
#pragma clang loop unroll(disable)
        for (int u = 0; u < 4 * NT; ++u) {
          const int T = u >> 2, t = u & 3;
          const int i = 16 * R + g + 4 * t;
          double v = 0.0;
          if (T < NR) {
            const int j = 16 * T + jc;
            if (i < n && j < n) {
              const double dx = xi_s[3 * i] - xi_s[3 * j];
              const double dy = xi_s[3 * i + 1] - xi_s[3 * j + 1];
              const double dz = xi_s[3 * i + 2] - xi_s[3 * j + 2];
              v = phs(dx * dx + dy * dy + dz * dz, m);
            } else if (i < n && j < K) {
              v = monomial_pw(pw_s + 3 * i * l1, l1, ex_s + 3 * (j - n));
            } else if (j < n && i < K) {
              v = monomial_pw(pw_s + 3 * j * l1, l1, ex_s + 3 * (i - n));
            }
          } else if (jc < nb && i < K) {
            const double* pe = xi_s + 3 * cols_s[cb + jc];
            if (i < n) {
              const double dx = pe[0] - xi_s[3 * i];
              const double dy = pe[1] - xi_s[3 * i + 1];
              const double dz = pe[2] - xi_s[3 * i + 2];
              v = phs_op(dx, dy, dz, dx * dx + dy * dy + dz * dz, m, d, op,
                         nrm[0], nrm[1], nrm[2]);
            } else {
              v = lpsi_s[jc * M + (i - n)];
            }
          }
          strip[u * 64 + lane] = v;
        }
        sfor<0, NT>([&](auto Tc) __attribute__((always_inline)) {
          constexpr int T = decltype(Tc)::value;
          sfor<0, 4>([&](auto tc) __attribute__((always_inline)) {
            constexpr int t = decltype(tc)::value;
            acc[R][T][t] = strip[(4 * T + t) * 64 + lane];
          });
        });
      });
      // ---- blocked Gauss-Jordan ----
      // row-per-lane activity masks (0 once a row has served as a pivot)
      uint32_t act0 = lane < K ? 0x7FFFFF80u : 0u;
      uint32_t act1 = (S > 64 && 64 + lane < K) ? 0x7FFFFF80u : 0u;
      bool singular = false;
      const int npan = (K + 3) >> 2;
      sfor<0, NR>([&](auto Tpc) __attribute__((always_inline)) {
        constexpr int TP = decltype(Tpc)::value;
#pragma clang loop unroll(disable)
        for (int q = 0; q < 4; ++q) {
          const int pan = 4 * TP + q;
          if (pan >= npan) break;
          // 1. the panel's four columns, row per lane
          wsync();
          if ((jc >> 2) == q) {
            sfor<0, NR>([&](auto Rc) __attribute__((always_inline)) {
              constexpr int R = decltype(Rc)::value;
              sfor<0, 4>([&](auto tc) __attribute__((always_inline)) {
                constexpr int t = decltype(tc)::value;
                pbuf[(jc & 3) * S + 16 * R + g + 4 * t] = acc[R][TP][t];
              });
            });
          }
          wsync();
          double p0[4], p1[4];
          sfor<0, 4>([&](auto cc) __attribute__((always_inline)) {
            constexpr int c = decltype(cc)::value;
            p0[c] = (S >= 64 || lane < S) ? pbuf[c * S + lane] : 0.0;
            p1[c] = (S > 64 && lane < S - 64) ? pbuf[c * S + 64 + lane] : 0.0;
          });
          // 2. four pivot steps on the panel
          double m0[4], m1[4];
          int prow[4];
          sfor<0, 4>([&](auto sc) __attribute__((always_inline)) {
            constexpr int s = decltype(sc)::value;
            const int k = 4 * pan + s;
            m0[s] = 0.0;
            m1[s] = 0.0;
            prow[s] = -1;
            if (k < K) {
              // rows that do not exist (slots >= S) take key 0, so even a
              // singular system's pivot is a row slot below S
              const uint32_t key0 =
                  (S >= 64 || lane < S)
                      ? ((uint32_t)__double2hiint(p0[s]) & act0) | (uint32_t)lane
                      : 0u;
              const uint32_t key1 =
                  (S > 64 && lane < S - 64)
                      ? ((uint32_t)__double2hiint(p1[s]) & act1) |
                            (uint32_t)(64 + lane)
                      : 0u;
              const uint32_t kmax = wave_max_u32(umax(key0, key1));
              if ((kmax & 0x7FFFFF80u) == 0u) singular = true;
              const int piv = (int)(kmax & 127u);
              const int pl = piv & 63;
              const bool ps = piv >= 64;
              double u[4];
              sfor<0, 4>([&](auto cc) __attribute__((always_inline)) {
                constexpr int c = decltype(cc)::value;
                u[c] = readlane_f64(ps ? p1[c] : p0[c], pl);
              });
              if (!(u[s] != 0.0)) singular = true;
              const double dk = singular ? 0.0 : recip(u[s]);
              const bool me0 = !ps && lane == pl, me1 = ps && lane == pl;
              act0 = me0 ? 0u : act0;
              act1 = me1 ? 0u : act1;
              m0[s] = me0 ? 0.0 : p0[s] * dk;
              m1[s] = me1 ? 0.0 : p1[s] * dk;
              sfor<s + 1, 4>([&](auto cc) __attribute__((always_inline)) {
                constexpr int c = decltype(cc)::value;
                p0[c] = fma(-m0[s], u[c], p0[c]);
                p1[c] = fma(-m1[s], u[c], p1[c]);
              });
              if (lane == 0) {
                srank[piv] = k;
                dinv[k] = dk;
              }
              prow[s] = piv;
            }
          });
          // 3. L[s][s'] = m_s'(pivot row s), s' < s; Ti = L^-1 (unit lower)
          double Lm[4][4];
          sfor<1, 4>([&](auto sc) __attribute__((always_inline)) {
            constexpr int s = decltype(sc)::value;
            const int pr = prow[s];
            const int pl = pr & 63;
            const bool ps = pr >= 64;
            sfor<0, s>([&](auto s2c) __attribute__((always_inline)) {
              constexpr int s2 = decltype(s2c)::value;
              const double v = readlane_f64(ps ? m1[s2] : m0[s2], pl);
              Lm[s][s2] = pr >= 0 ? v : 0.0;
            });
          });
          const double T10 = -Lm[1][0];
          const double T21 = -Lm[2][1];
          const double T20 = -Lm[2][0] - Lm[2][1] * T10;
          const double T32 = -Lm[3][2];
          const double T31 = -Lm[3][1] - Lm[3][2] * T21;
          const double T30 = -Lm[3][0] - Lm[3][1] * T10 - Lm[3][2] * T20;
          // 4. -(M L^-1), row per lane, into operand layout
          auto mlinv = [&](const double (&mm)[4], double (&o)[4])
                           __attribute__((always_inline)) {
            o[3] = mm[3];
            o[2] = fma(mm[3], T32, mm[2]);
            o[1] = fma(mm[3], T31, fma(mm[2], T21, mm[1]));
            o[0] = fma(mm[3], T30, fma(mm[2], T20, fma(mm[1], T10, mm[0])));
          };
          double o0[4], o1[4];
          mlinv(m0, o0);
          mlinv(m1, o1);
          sfor<0, 4>([&](auto sc) __attribute__((always_inline)) {
            constexpr int s = decltype(sc)::value;
            if (S >= 64 || lane < S) mbuf[lane * 4 + s] = -o0[s];
            if (S > 64 && lane < S - 64) mbuf[(64 + lane) * 4 + s] = -o1[s];
          });
          // 5. the pivot rows as they stand, columns right of the panel
          //    tile's start, into operand layout
          sfor<0, 4>([&](auto sc) __attribute__((always_inline)) {
            constexpr int s = decltype(sc)::value;
            const int pr = prow[s];
            double* dst = ubuf + s * 16 * NT;
            if (pr >= 0) {
              pivot_row_out<NR, NT, TP>(acc, 4 * (pr >> 4) + ((pr & 15) >> 2),
                                        g == (pr & 3), jc, dst);
            } else if (g == 0) {
              sfor<TP, NT>([&](auto Tc) __attribute__((always_inline)) {
                constexpr int T = decltype(Tc)::value;
                dst[16 * T + jc] = 0.0;
              });
            }
          });
          wsync();
          double aop[NR], bop[NT];
          sfor<0, NR>([&](auto Rc) __attribute__((always_inline)) {
            constexpr int R = decltype(Rc)::value;
            aop[R] = mbuf[(16 * R + jc) * 4 + g];
          });
          sfor<TP, NT>([&](auto Tc) __attribute__((always_inline)) {
            constexpr int T = decltype(Tc)::value;
            bop[T] = ubuf[g * 16 * NT + 16 * T + jc];
          });
          // 6. rank-4 update of every row, tiles from the panel's on
          sfor<TP, NT>([&](auto Tc) __attribute__((always_inline)) {
            constexpr int T = decltype(Tc)::value;
            sfor<0, NR>([&](auto Rc) __attribute__((always_inline)) {
              constexpr int R = decltype(Rc)::value;
              acc[R][T] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                  aop[R], bop[T], acc[R][T], 0, 0, 0);
            });
          });
        }
      });
      // ---- solution: the row slot pivoted at step j holds u_jj x_j ----
      // (a singular system maps its slots to themselves and writes NaN, as
      // the register kernel does)
      wsync();
      if (singular) {
        for (int t = lane; t < S; t += 64) srank[t] = t;
        wsync();
      }
      if (singular && lane == 0) report(P.st, ORBF_ESINGULAR, ck);
      const int e = jc;
      const bool live = e < nb;
      const int32_t row = live ? stn[cols_s[cb + e]] : 0;
      double lam = 0.0;
      sfor<0, NR>([&](auto Rc) __attribute__((always_inline)) {
        constexpr int R = decltype(Rc)::value;
        sfor<0, 4>([&](auto tc) __attribute__((always_inline)) {
          constexpr int t = decltype(tc)::value;
          const int i = 16 * R + g + 4 * t;
          if (live && i < K) {
            const int j = srank[i];
            if (j < n) {
              const double w =
                  singular ? NAN : (acc[R][NR][t] * dinv[j]) * sinv;
              P.W[(int64_t)row * n + j] = w;
              lam += fabs(w);
            }
          }
        });
      });
      lam += __shfl_xor(lam, 16, 64);
      lam += __shfl_xor(lam, 32, 64);
      if (live && g == 0) {
        if (P.lebesgue) P.lebesgue[row] = lam;
        if (explicit_rows && P.owner_out) P.owner_out[row] = row;
      }
      wsync();
    }
  }
}

}  // namespace

// Launch the matrix-core kernel if it covers the system: K <= 80 and no
// acceptance mode.  Returns false otherwise.
bool launch_weights_mfma(orbf_ctx* ctx, const WeightsParams& P,
                         int64_t grid) {
  if (P.accept || P.M > 80 || P.K > 80 || P.K <= 32) return false;
  const size_t dyn =
      ((size_t)16 * P.M + (size_t)3 * P.n * (P.l + 1)) * sizeof(double);
  if (P.K <= 48)
    hipLaunchKernelGGL(weights_mfma_kernel<3>, dim3((unsigned)grid), dim3(64),
                       dyn, ctx->stream, P);
  else if (P.K <= 64)
    hipLaunchKernelGGL(weights_mfma_kernel<4>, dim3((unsigned)grid), dim3(64),
                       dyn, ctx->stream, P);
  else
    hipLaunchKernelGGL(weights_mfma_kernel<5>, dim3((unsigned)grid), dim3(64),
                       dyn, ctx->stream, P);
  return true;
}

}  // namespace orbf
