// Local RBF-FD weights with an FP32 elimination and FP64 iterative
// refinement (Sec. 4.1, eqs. rbffd_linsys, orbffd_eq, orbffd_rhs).
//
// Lane layout as in the FP64 register kernel: lane = r + 8 c holds rows
// 8 ii + r and columns 8 jj + c of A_hat, here an L x L block of FP32 values.
// The Gauss-Jordan sweep with implicit partial pivoting keeps its multipliers
// in place: at step k every non-pivot row stores l_ik in column k and the
// pivot row keeps u_kk there; later steps update only the columns right of k.
// The recorded sweep (pivot slot and 1/u_kk of every step) can then be
// replayed on any right-hand side without factoring again.
//
// For each block of up to 8 PL retained columns (right-hand sides):
//   X = 0; repeat
//     R = B_hat - A_hat X   in FP64, one matrix row per lane, with A_hat and
//                           B_hat evaluated again in FP64 from the scaled
//                           coordinates (the FP32 copy is never used here);
//     D = replay(R)         in FP32;
//     X = X + D             in FP64;
//   until max_{j<n} |D_j| <= tol * max_{j<n} |X_j| in every column.
// The weights (first n unknowns), their unscaling and the Lebesgue sums are
// formed from X in FP64.  A stencil that meets an exact zero FP32 pivot, or
// whose block has not converged after the context's correction cap (8 by
// default, orbf_set_ir_max_corrections) is appended to a fallback list that
// the FP64 kernel then solves from scratch.
#include <math.h>

#include "orbf_internal.hpp"
#include "weights_common.hpp"

namespace orbf {

namespace {

constexpr double kRefineTol = 1e-11;

template <int L, int PL>
__global__ __launch_bounds__(64, 2) void weights_ir_kernel(WeightsParams P) {
  constexpr int S = 8 * L;
  constexpr int NB = 8 * PL;         // right-hand sides per block
  extern __shared__ double dyn_s[];  // psi (n x M) | L psi (NB x M) | powers
  __shared__ double xi_s[3 * S];
  __shared__ int cols_s[S];
  __shared__ int8_t ex_s[3 * 36];
  __shared__ float ubuf[8 * L];  // pivot row [c][jj]; replay: pivot rhs [c][jp]
  __shared__ float lbuf[8 * L];  // multipliers [r][ii]
  __shared__ float dinv_s[S];    // 1 / u_kk of step k
  __shared__ int piv_s[S];       // row slot pivoted at step k
  __shared__ int srank[S];       // step at which a row slot was pivoted
  __shared__ double xs[S * NB];  // X by unknown index (also assembly strip)
  __shared__ float rs[S * NB];   // residual by matrix row

  const int lane0 = threadIdx.x;
  const int n = P.n, K = P.K, d = P.d, M = P.M, m = P.m, op = P.op;
  double* psi_s = dyn_s;
  double* lpsi_s = dyn_s + n * M;
  double* pw_s = lpsi_s + NB * M;
  double* strip = xs;
  for (int t = lane0; t < 3 * M; t += 64) ex_s[t] = P.ex[t];
  // eliminations write only values in [0, K) here, so with this start no
  // rank read below can index out of range
  for (int t = lane0; t < S; t += 64) srank[t] = 0;

  const int64_t total = *P.n_centers;
  for (int64_t ci = blockIdx.x; ci < total; ci += gridDim.x) {
    // the lane's coordinates, opaque to the compiler in every iteration:
    // values derived from them are recomputed per stencil instead of being
    // hoisted out of the stencil loop and held (spilled) across it
    int lane = lane0;
    __asm__ volatile("" : "+v"(lane));
    const int r = lane & 7, c = lane >> 3;
    const int32_t ck = P.centers[ci];
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
    // retained columns: the stencil nodes this center owns
    int ncol = 0;
    for (int q0 = 0; q0 < n; q0 += 64) {
      const int q = q0 + lane;
      const bool mine = q < n && P.owner[stn[q]] == ck;
      const unsigned long long b = __ballot(mine);
      if (mine) cols_s[ncol + __popcll(b & ((1ull << lane) - 1ull))] = q;
      ncol += __popcll(b);
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
      double* pw = pw_s + t * l1;
      double acc = 1.0;
      for (int e = 0; e < l1; ++e) {
        pw[e] = acc;
        acc *= v;
      }
    }
    wsync();
    for (int t = lane; t < n * M; t += 64) {
      const int q = t / M, s = t - q * M;
      psi_s[t] = monomial_pw(pw_s + 3 * q * l1, l1, ex_s + 3 * s);
    }
    const double sinv = op_unscale(op, r2c, rho);
    double nrm[3] = {0.0, 0.0, 0.0};
    op_axis(op, nrm);
    wsync();

    // ---- assemble A_hat (FP64 entries, stored as FP32) ----
    // A_hat is symmetric: only its blocks jj >= ii are computed, the others
    // are taken from their mirror blocks below
    float a[L][L];
    sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
      constexpr int ii = decltype(iic)::value;
      const int i = 8 * ii + r;
      const bool ri = i < n;
      const double xi0 = ri ? xi_s[3 * i] : 0.0;
      const double xi1 = ri ? xi_s[3 * i + 1] : 0.0;
      const double xi2 = ri ? xi_s[3 * i + 2] : 0.0;
#pragma clang loop unroll(disable)
      for (int jj = ii; jj < L; ++jj) {
        const int j = 8 * jj + c;
        double v = 0.0;
        if (i < n && j < n) {
          const double dx = xi0 - xi_s[3 * j], dy = xi1 - xi_s[3 * j + 1];
          const double dz = xi2 - xi_s[3 * j + 2];
          v = phs(dx * dx + dy * dy + dz * dz, m);
        } else if (i < n && j < K) {
          v = psi_s[i * M + (j - n)];
        } else if (j < n && i < K) {
          v = psi_s[j * M + (i - n)];
        }
        strip[jj * 64 + lane] = v;
      }
      sfor<ii, L>([&](auto jjc) __attribute__((always_inline)) {
        constexpr int jj = decltype(jjc)::value;
        a[ii][jj] = (float)strip[jj * 64 + lane];
      });
    });
    // entry (8 ii + r, 8 jj + c) equals entry (8 jj + c, 8 ii + r), which
    // lane (c, r) holds in block (jj, ii)
    {
      const int tr = (c + 8 * r) << 2;
      sfor<1, L>([&](auto iic) __attribute__((always_inline)) {
        constexpr int ii = decltype(iic)::value;
        sfor<0, ii>([&](auto jjc) __attribute__((always_inline)) {
          constexpr int jj = decltype(jjc)::value;
          a[ii][jj] = __int_as_float(
              __builtin_amdgcn_ds_bpermute(tr, __float_as_int(a[jj][ii])));
        });
      });
    }

    // ---- FP32 Gauss-Jordan, multipliers kept in place ----
    uint32_t act[L];
    sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
      constexpr int ii = decltype(iic)::value;
      act[ii] = (8 * ii + r < K) ? 0x7FFFFFF0u : 0u;
    });
    bool zero_pivot = false;
    sfor<0, L>([&](auto kbc) __attribute__((always_inline)) {
      constexpr int kb = decltype(kbc)::value;
#pragma clang loop unroll(disable)
      for (int cc = 0; cc < 8; ++cc) {
        const int k = 8 * kb + cc;
        if (k >= K) break;
        uint32_t key0 = 0;
        sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
          constexpr int ii = decltype(iic)::value;
          key0 = umax(key0, (__float_as_uint(a[ii][kb]) & act[ii]) | (uint32_t)ii);
        });
        const uint32_t kmax = __builtin_amdgcn_readlane(group8_max(key0), 8 * cc);
        if ((kmax & 0x7FFFFFF0u) == 0u) zero_pivot = true;
        const int iip = (int)(kmax & 15u);
        const unsigned long long who =
            __ballot(key0 == kmax) & (0xFFull << (8 * cc));
        const int rp = (__ffsll((long long)who) - 1) & 7;
        const int piv = 8 * iip + rp;
        sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
          constexpr int ii = decltype(iic)::value;
          act[ii] = (ii == iip && r == rp) ? 0u : act[ii];
        });
        sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
          constexpr int ii = decltype(iic)::value;
          if (iip == ii) {
            __asm__ volatile("; ir pivot row out %0" ::"i"(ii));
            if (r == rp) {
              sfor<kb, L>([&](auto jjc) __attribute__((always_inline)) {
                constexpr int jj = decltype(jjc)::value;
                ubuf[c * L + jj] = a[ii][jj];
              });
            }
          }
        });
        if (c == cc) {
          sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
            constexpr int ii = decltype(iic)::value;
            lbuf[r * L + ii] = (ii == iip && r == rp) ? 0.0f : a[ii][kb];
          });
        }
        if (lane == 0) {
          srank[piv] = k;
          piv_s[k] = piv;
        }
        wsync();
        const float upiv = ubuf[cc * L + kb];
        if (!(upiv != 0.0f)) zero_pivot = true;
        const float dk = zero_pivot ? 0.0f : __builtin_amdgcn_rcpf(upiv);
        if (lane == 0) dinv_s[k] = dk;
        float u[L], lv[L];
        sfor<kb, L>([&](auto jjc) __attribute__((always_inline)) {
          constexpr int jj = decltype(jjc)::value;
          u[jj] = ubuf[c * L + jj];
        });
        sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
          constexpr int ii = decltype(iic)::value;
          lv[ii] = lbuf[r * L + ii];
        });
        sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
          constexpr int ii = decltype(iic)::value;
          const bool is_piv = ii == iip && r == rp;
          const float lm = lv[ii] * dk;
          // column block kb: columns right of k are updated, column k
          // receives the multiplier, columns left of k hold earlier ones
          const float upd = fmaf(-lm, u[kb], a[ii][kb]);
          a[ii][kb] = (c > cc) ? upd : ((c == cc && !is_piv) ? lm : a[ii][kb]);
          sfor<kb + 1, L>([&](auto jjc) __attribute__((always_inline)) {
            constexpr int jj = decltype(jjc)::value;
            a[ii][jj] = fmaf(-lm, u[jj], a[ii][jj]);
          });
        });
        wsync();
      }
    });

    // Without a zero pivot every step pivots a row still active, so each
    // of the K slots has exactly one rank; with one, the ranks are not used
    // (the stencil goes to the FP64 fallback).
    int rank[L];
    float rdk[L];
    sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
      constexpr int ii = decltype(iic)::value;
      const bool live = 8 * ii + r < K;
      rank[ii] = live ? srank[8 * ii + r] : 1 << 20;
      rdk[ii] = live ? dinv_s[rank[ii]] : 0.0f;
    });
    bool ok = !zero_pivot;

    for (int cb = 0; ok && cb < ncol; cb += NB) {
      const int nb = min(NB, ncol - cb);
      wsync();
      for (int t = lane; t < nb * M; t += 64) {
        const int e = t / M, s = t - e * M;
        lpsi_s[t] = monomial_op_pw(pw_s + 3 * cols_s[cb + e] * l1, l1,
                                   ex_s + 3 * s, op, nrm[0], nrm[1], nrm[2]);
      }
      double X[L][PL];
      sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
        constexpr int ii = decltype(iic)::value;
        sfor<0, PL>([&](auto jpc) __attribute__((always_inline)) {
          constexpr int jp = decltype(jpc)::value;
          X[ii][jp] = 0.0;
        });
      });
      int it = 0;
      for (;;) {
        // X -> LDS by unknown index
        wsync();
        sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
          constexpr int ii = decltype(iic)::value;
          if (rank[ii] < K) {
            sfor<0, PL>([&](auto jpc) __attribute__((always_inline)) {
              constexpr int jp = decltype(jpc)::value;
              xs[rank[ii] * NB + 8 * jp + c] = X[ii][jp];
            });
          }
        });
        wsync();
        // R = B_hat - A_hat X in FP64, matrix row i on lane i mod 64
#pragma clang loop unroll(disable)
        for (int i0 = 0; i0 < K; i0 += 64) {
          const int i = i0 + lane;
          const bool ri = i < K, in = i < n;
          const double x0 = in ? xi_s[3 * i] : 0.0;
          const double x1 = in ? xi_s[3 * i + 1] : 0.0;
          const double x2 = in ? xi_s[3 * i + 2] : 0.0;
          double acc[NB];
          sfor<0, NB>([&](auto ec) __attribute__((always_inline)) {
            constexpr int e = decltype(ec)::value;
            double b = 0.0;
            if (ri && e < nb) {
              if (in) {
                const double* pe = xi_s + 3 * cols_s[cb + e];
                const double dx = pe[0] - x0, dy = pe[1] - x1, dz = pe[2] - x2;
                b = phs_op(dx, dy, dz, dx * dx + dy * dy + dz * dz, m, d, op,
                           nrm[0], nrm[1], nrm[2]);
              } else {
                b = lpsi_s[e * M + (i - n)];
              }
            }
            acc[e] = b;
          });
#pragma clang loop unroll(disable)
          for (int j = 0; j < K; ++j) {
            double aij = 0.0;
            if (in && j < n) {
              const double dx = x0 - xi_s[3 * j], dy = x1 - xi_s[3 * j + 1];
              const double dz = x2 - xi_s[3 * j + 2];
              aij = phs(dx * dx + dy * dy + dz * dz, m);
            } else if (in) {
              aij = psi_s[i * M + (j - n)];
            } else if (ri && j < n) {
              aij = psi_s[j * M + (i - n)];
            }
            const double* xj = xs + j * NB;
            sfor<0, NB>([&](auto ec) __attribute__((always_inline)) {
              constexpr int e = decltype(ec)::value;
              acc[e] = fma(-aij, xj[e], acc[e]);
            });
          }
          if (ri) {
            sfor<0, NB>([&](auto ec) __attribute__((always_inline)) {
              constexpr int e = decltype(ec)::value;
              rs[i * NB + e] = (float)acc[e];
            });
          }
        }
        wsync();
        // D = replay of the recorded sweep on R (FP32)
        float rhs[L][PL];
        sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
          constexpr int ii = decltype(iic)::value;
          const int i = 8 * ii + r;
          sfor<0, PL>([&](auto jpc) __attribute__((always_inline)) {
            constexpr int jp = decltype(jpc)::value;
            rhs[ii][jp] = (i < K) ? rs[i * NB + 8 * jp + c] : 0.0f;
          });
        });
        sfor<0, L>([&](auto kbc) __attribute__((always_inline)) {
          constexpr int kb = decltype(kbc)::value;
#pragma clang loop unroll(disable)
          for (int cc = 0; cc < 8; ++cc) {
            const int k = 8 * kb + cc;
            if (k >= K) break;
            const int piv = __builtin_amdgcn_readfirstlane(piv_s[k]);
            const int iip = piv >> 3, rp = piv & 7;
            // stored multipliers of step k; the pivot row's slot holds
            // u_kk, which the replay must not apply
            if (c == cc) {
              sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
                constexpr int ii = decltype(iic)::value;
                lbuf[r * L + ii] = (ii == iip && r == rp) ? 0.0f : a[ii][kb];
              });
            }
            sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
              constexpr int ii = decltype(iic)::value;
              if (iip == ii) {
                __asm__ volatile("; ir replay pivot rhs %0" ::"i"(ii));
                if (r == rp) {
                  sfor<0, PL>([&](auto jpc) __attribute__((always_inline)) {
                    constexpr int jp = decltype(jpc)::value;
                    ubuf[c * PL + jp] = rhs[ii][jp];
                  });
                }
              }
            });
            wsync();
            float ur[PL], lv[L];
            sfor<0, PL>([&](auto jpc) __attribute__((always_inline)) {
              constexpr int jp = decltype(jpc)::value;
              ur[jp] = ubuf[c * PL + jp];
            });
            sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
              constexpr int ii = decltype(iic)::value;
              lv[ii] = lbuf[r * L + ii];
            });
            sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
              constexpr int ii = decltype(iic)::value;
              const float lm = lv[ii];
              sfor<0, PL>([&](auto jpc) __attribute__((always_inline)) {
                constexpr int jp = decltype(jpc)::value;
                rhs[ii][jp] = fmaf(-lm, ur[jp], rhs[ii][jp]);
              });
            });
            wsync();
          }
        });
        // X += D; convergence of the weights part, per column
        uint32_t dkey[PL], xkey[PL];
        sfor<0, PL>([&](auto jpc) __attribute__((always_inline)) {
          constexpr int jp = decltype(jpc)::value;
          dkey[jp] = 0u;
          xkey[jp] = 0u;
        });
        sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
          constexpr int ii = decltype(iic)::value;
          sfor<0, PL>([&](auto jpc) __attribute__((always_inline)) {
            constexpr int jp = decltype(jpc)::value;
            const float dj = rhs[ii][jp] * rdk[ii];
            X[ii][jp] += (double)dj;
            if (rank[ii] < n) {
              dkey[jp] = umax(dkey[jp], __float_as_uint(fabsf(dj)));
              xkey[jp] = umax(xkey[jp],
                              __float_as_uint(fabsf((float)X[ii][jp])));
            }
          });
        });
        bool col_ok = true;
        sfor<0, PL>([&](auto jpc) __attribute__((always_inline)) {
          constexpr int jp = decltype(jpc)::value;
          const float dmax = __uint_as_float(group8_max(dkey[jp]));
          const float xmax = __uint_as_float(group8_max(xkey[jp]));
          if (8 * jp + c < nb)
            col_ok &= (double)dmax <= kRefineTol * (double)xmax;
        });
        if (__ballot(!col_ok) == 0ull) break;
        if (++it > P.ir_max) {
          ok = false;
          break;
        }
      }
      if (!ok) break;
      // unscale, write rows, Lebesgue values
      sfor<0, PL>([&](auto jpc) __attribute__((always_inline)) {
        constexpr int jp = decltype(jpc)::value;
        const int e = 8 * jp + c;
        const bool live = e < nb;
        const int32_t row = live ? stn[cols_s[cb + e]] : 0;
        double lam = 0.0;
        sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
          constexpr int ii = decltype(iic)::value;
          const int j = rank[ii];
          if (live && j < n) {
            const double w = X[ii][jp] * sinv;
            P.W[(int64_t)row * n + j] = w;
            lam += fabs(w);
          }
        });
        lam += __shfl_xor(lam, 1, 64);
        lam += __shfl_xor(lam, 2, 64);
        lam += __shfl_xor(lam, 4, 64);
        if (live && r == 0) {
          if (P.lebesgue) P.lebesgue[row] = lam;
          if (P.ir_steps) P.ir_steps[row] = it;
        }
      });
    }
    if (!ok) {
      // rows of blocks that did settle were written with their counts;
      // the FP64 kernel solves the whole stencil again, so all its rows
      // report -1 (solved in FP64)
      if (P.ir_steps)
        for (int e = lane; e < ncol; e += 64) P.ir_steps[stn[cols_s[e]]] = -1;
      if (lane == 0) {
        const unsigned long long at =
            atomicAdd((unsigned long long*)P.fb_count, 1ull);
        P.fb_list[at] = ck;
      }
    }
  }
}

__global__ void fill_i32_ir(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void zero_i64_ir(int64_t* p) { *p = 0; }

}  // namespace

void launch_ir_prepare(orbf_ctx* ctx, int32_t* ir_steps, int64_t N,
                       int64_t* fb_count) {
  if (ir_steps && N > 0) {
    const int64_t blocks = (N + 255) / 256 < 4096 ? (N + 255) / 256 : 4096;
    hipLaunchKernelGGL(fill_i32_ir, dim3((unsigned)blocks), dim3(256), 0,
                       ctx->stream, ir_steps, N, -1);
  }
  hipLaunchKernelGGL(zero_i64_ir, dim3(1), dim3(1), 0, ctx->stream, fb_count);
}

// Launch the FP32 + refinement kernel if a variant covers K (covered rows
// only); returns false otherwise.
bool launch_weights_ir(orbf_ctx* ctx, const WeightsParams& P, int64_t grid) {
  if (P.M > 35 || P.rows != nullptr || P.K > 72) return false;
  constexpr int PL = 1;
  const size_t dyn = ((size_t)(P.n + 8 * PL) * P.M +
                      (size_t)3 * P.n * (P.l + 1)) * sizeof(double);
#define ORBF_IR_CASE(LL)                                                      \
  if (P.K <= 8 * LL) {                                                        \
    hipLaunchKernelGGL((weights_ir_kernel<LL, PL>), dim3((unsigned)grid),     \
                       dim3(64), dyn, ctx->stream, P);                        \
    return true;                                                              \
  }
  ORBF_IR_CASE(3)
  ORBF_IR_CASE(4)
  ORBF_IR_CASE(5)
  ORBF_IR_CASE(6)
  ORBF_IR_CASE(7)
  ORBF_IR_CASE(8)
  ORBF_IR_CASE(9)
#undef ORBF_IR_CASE
  return false;
}

}  // namespace orbf
