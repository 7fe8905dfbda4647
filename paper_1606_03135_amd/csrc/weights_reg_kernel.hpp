// Local RBF-FD weights with the saddle system held in registers
// (Sec. 4.1, eqs. rbffd_linsys, orbffd_eq, orbffd_rhs).
//
// One wavefront per stencil center.  The K x (K + P) augmented matrix
// [A_hat | B_hat] is distributed 2D block-cyclically over an 8 x 8 lane grid:
// lane = r + 8 c holds rows i = 8 ii + r (ii < L) and columns j = 8 jj + c
// (jj < L: A_hat; jj = L + jp: right-hand side e = 8 jp + c), K <= 8 L,
// P <= 8 PL.  The trailing update is an L x (L + PL) register block per lane,
// so all 64 lanes stay busy and every broadcast value is reused L times.
//
// Rows never move (implicit partial pivoting): a per-row mask retires a row
// once it has served as a pivot, so every register index is a compile-time
// constant.  Elimination step k = 8 kb + cc (kb unrolled, cc a uniform loop
// counter) makes one LDS round trip:
//   1. pivot search: the 8 lanes of column k reduce a 32-bit key
//      (|a| high bits | local row) with DPP; readlane and a ballot give the
//      pivot's row slot as wave-uniform values;
//   2. the pivot row (one scalar-branch case) goes to LDS, and the column
//      of multipliers from lane to lane (ds_bpermute);
//   3. every lane reads its pivot-row entries and applies the rank-1
//      update to its L x (L + PL - kb) register block.
// The elimination is Gauss-Jordan: the rows pivoted earlier are eliminated
// too (they are in the register block anyway), so when the last step is done
// the row slot pivoted at step j holds u_jj x_j in its right-hand-side
// columns and no back substitution is needed.  Multipliers are not kept.
// Padded slots (>= K) are inactive from the start and hold zeros.
#pragma once

#include <math.h>

#include "orbf_internal.hpp"
#include "weights_common.hpp"

namespace orbf {

namespace {

// v of lane addr / 4 (ds_bpermute through the LDS crossbar, no LDS memory)
__device__ __forceinline__ double bperm_f64(int addr, double v) {
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// ACC: acceptance mode (the stencil's ball nodes plus the reference node are
// the columns; Lambda and the accept bits are written instead of W)
template <int L, int PL, bool ACC>
__global__ __launch_bounds__(64, 2) void weights_reg_kernel(WeightsParams P) {
  constexpr int LC = L + PL;
  constexpr int S = 8 * L;  // row / column slots of A_hat
  extern __shared__ double dyn_s[];  // L psi (8 PL x M), then powers
  __shared__ double xi_s[3 * S];
  __shared__ int cols_s[S];
  __shared__ int8_t ex_s[3 * 36];
  __shared__ double ubuf[8 * LC];  // [c][jj] pivot row
  __shared__ double dinv[S];
  __shared__ int srank[S];         // elimination step of each row slot
  __shared__ double lam_s[S + 1];  // acceptance mode: Lambda per column
  __shared__ double dif_s[3 * S];  // acceptance mode: x_q - x_k
  __shared__ int refcol_s;
  // per-stencil uniforms parked here for the passes, so they are not held
  // in registers (and spilled) across the elimination: the operator
  // direction, the unscale factor, the center
  __shared__ double sv_s[4];
  __shared__ int ck_s;
  __shared__ unsigned long long accw_s[2];

  const int lane0 = threadIdx.x;
  const int n = P.n, K = P.K, d = P.d, M = P.M, m = P.m, op = P.op;
  // no table of psi_t(xi_q): monomials are formed from the power table
  // during assembly, which keeps LDS per wavefront small enough for two
  // wavefronts per SIMD
  double* lpsi_s = dyn_s;               // L psi_t at the evaluation points
  double* pw_s = lpsi_s + 8 * PL * M;   // powers of the scaled coordinates
  for (int t = lane0; t < 3 * M; t += 64) ex_s[t] = P.ex[t];
  // every elimination writes only values in [0, K) here, so with this
  // start no rank read below can ever index out of range
  for (int t = lane0; t < S; t += 64) srank[t] = 0;

  const bool explicit_rows = P.rows != nullptr;
  const int64_t total = explicit_rows ? P.n_rows : *P.n_centers;
  for (int64_t ci = blockIdx.x; ci < total; ci += gridDim.x) {
    // the lane index, opaque to the compiler in every iteration: values
    // derived from it are recomputed per stencil instead of being hoisted
    // out of the stencil loop and held (spilled) across it
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
    int ncol = 0, nball = 0;
    constexpr bool accept_mode = ACC;
    if (accept_mode) {
      // columns: the center, its ball, and the stencil node nearest the
      // stencil centroid (Sec. 4.2.1), found exactly as the sequential
      // rule does: offsets x_q - x_k summed in stencil order, squared
      // distances ((e0*e0)+(e1*e1))+(e2*e2), first minimum
      const double* xc = P.xyz + (int64_t)ck * d;
      for (int q = lane; q < n; q += 64) {
        const double* xq = P.xyz + (int64_t)stn[q] * d;
        dif_s[3 * q] = xq[0] - xc[0];
        dif_s[3 * q + 1] = xq[1] - xc[1];
        dif_s[3 * q + 2] = (d == 3) ? xq[2] - xc[2] : 0.0;
      }
      wsync();
      double cen[3] = {0.0, 0.0, 0.0};
      if (lane == 0) {
#pragma clang fp contract(off)
        for (int q = 0; q < n; ++q)
          for (int a = 0; a < 3; ++a) cen[a] = cen[a] + dif_s[3 * q + a];
        for (int a = 0; a < 3; ++a) cen[a] = cen[a] / (double)n;
      }
      for (int a = 0; a < 3; ++a) cen[a] = __shfl(cen[a], 0, 64);
      double bd = INFINITY;
      int bq = n;
      for (int q = lane; q < n; q += 64) {
        const double s = exact_sqdist(dif_s[3 * q], dif_s[3 * q + 1],
                                      dif_s[3 * q + 2], cen[0], cen[1],
                                      cen[2], d);
        if (s < bd) {
          bd = s;
          bq = q;
        }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(bd, o, 64);
        const int oq = __shfl_xor(bq, o, 64);
        if (ob < bd || (ob == bd && oq < bq)) {
          bd = ob;
          bq = oq;
        }
      }
      const uint64_t b0 = P.ball[2 * (int64_t)ck], b1 = P.ball[2 * (int64_t)ck + 1];
      // columns: the unclaimed-candidate ball (eligible nodes after the
      // center, from the covering's masks), or for the radial prefix the
      // whole eligible ball, tested here exactly as the covering tests it
      const bool prefix = P.tau_mode == 1;
      const double thr = prefix ? P.t2 * P.rho2[ck] : 0.0;
      auto in_cols = [&](int q) -> bool {
        if (q == 0) return true;
        if (!prefix) {
          const uint64_t word = (q < 64) ? b0 : b1;
          return (word >> (q & 63)) & 1ull;
        }
        const int32_t j = stn[q];
        if (P.eligible != nullptr && P.eligible[j] == 0) return false;
        const double* xq = P.xyz + (int64_t)j * d;
        return exact_sqdist(xc[0], xc[1], d == 3 ? xc[2] : 0.0, xq[0], xq[1],
                            d == 3 ? xq[2] : 0.0, d) <= thr;
      };
      for (int q0 = 0; q0 < n; q0 += 64) {
        const int q = q0 + lane;
        const bool mine = q < n && in_cols(q);
        const unsigned long long b = __ballot(mine);
        if (mine) cols_s[ncol + __popcll(b & ((1ull << lane) - 1ull))] = q;
        if (mine && q == bq) refcol_s = ncol + __popcll(b & ((1ull << lane) - 1ull));
        ncol += __popcll(b);
      }
      const bool ref_in = in_cols(bq);
      nball = ncol;
      if (!ref_in) {
        if (lane == 0) {
          cols_s[ncol] = bq;
          refcol_s = ncol;
        }
        ++ncol;
      }
      if (lane == 0) accw_s[0] = accw_s[1] = 0ull;
    } else if (explicit_rows) {
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
    // power table p_a^e, e <= l, of every stencil node (2D: p_2 = 0)
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
    if (lane == 0) {
      sv_s[0] = nrm[0];
      sv_s[1] = nrm[1];
      sv_s[2] = nrm[2];
      sv_s[3] = op_unscale(op, r2c, rho);
      ck_s = ck;
    }

    for (int cb = 0; cb < ncol; cb += 8 * PL) {
      const int nb = min(8 * PL, ncol - cb);
      // opaque again per pass, and the lane's grid coordinates derived
      // here: nothing lane-dependent is carried across the elimination
      // (1M-node ball: weights 5.87 -> 5.33 ms, per-lane scratch at L = 9
      // from 244-388 to 32-180 bytes)
      int lane = lane0;
      __asm__ volatile("" : "+v"(lane));
      const int r = lane & 7, c = lane >> 3;
      wsync();
      const double n0 = sv_s[0], n1 = sv_s[1], n2 = sv_s[2];
      for (int t = lane; t < nb * M; t += 64) {
        const int e = t / M, s = t - e * M;
        lpsi_s[t] = monomial_op_pw(pw_s + 3 * cols_s[cb + e] * l1, l1,
                                   ex_s + 3 * s, op, n0, n1, n2);
      }
      wsync();
      // ---- assemble [A_hat | B_hat] ----
      // Each entry is computed straight into its register (an unrolled
      // loop; a compact runtime loop through an LDS strip, written and read
      // back per entry, measured 4.69 against 4.45 ms on the 1M-node ball).
      // A_hat is symmetric, so only its blocks jj >= ii are computed; the
      // others are taken from their mirror blocks below.
      double a[L][LC];
      sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
        constexpr int ii = decltype(iic)::value;
        const int i = 8 * ii + r;
        const bool ri = i < n;
        const double xi0 = ri ? xi_s[3 * i] : 0.0;
        const double xi1 = ri ? xi_s[3 * i + 1] : 0.0;
        const double xi2 = ri ? xi_s[3 * i + 2] : 0.0;
        sfor<ii, LC>([&](auto jjc) __attribute__((always_inline)) {
          constexpr int jj = decltype(jjc)::value;
          double v = 0.0;
          if constexpr (jj < L) {
            const int j = 8 * jj + c;
            if (i < n && j < n) {
              const double dx = xi0 - xi_s[3 * j], dy = xi1 - xi_s[3 * j + 1];
              const double dz = xi2 - xi_s[3 * j + 2];
              v = phs(dx * dx + dy * dy + dz * dz, m);
            } else if (i < n && j < K) {
              v = monomial_pw(pw_s + 3 * i * l1, l1, ex_s + 3 * (j - n));
            } else if (j < n && i < K) {
              v = monomial_pw(pw_s + 3 * j * l1, l1, ex_s + 3 * (i - n));
            }
          } else {
            const int e = 8 * (jj - L) + c;
            if (e < nb && i < K) {
              const double* pe = xi_s + 3 * cols_s[cb + e];
              if (i < n) {
                const double dx = pe[0] - xi0, dy = pe[1] - xi1;
                const double dz = pe[2] - xi2;
                v = phs_op(dx, dy, dz, dx * dx + dy * dy + dz * dz, m, d, op,
                           n0, n1, n2);
              } else {
                v = lpsi_s[e * M + (i - n)];
              }
            }
          }
          a[ii][jj] = v;
        });
      });
      // the blocks below the diagonal: entry (8 ii + r, 8 jj + c) equals
      // entry (8 jj + c, 8 ii + r), which lane (c, r) holds in block (jj, ii)
      // (the same bits: the mirrored differences only change sign)
      {
        const int tr = (c + 8 * r) << 2;
        sfor<1, L>([&](auto iic) __attribute__((always_inline)) {
          constexpr int ii = decltype(iic)::value;
          sfor<0, ii>([&](auto jjc) __attribute__((always_inline)) {
            constexpr int jj = decltype(jjc)::value;
            a[ii][jj] = bperm_f64(tr, a[jj][ii]);
          });
        });
      }
      // ---- LU with row partial pivoting, rows kept in place ----
      // act[ii]: magnitude mask of local row ii (0 once the row has been
      // used as a pivot).  Pivoted rows keep their U entries and receive
      // zero multipliers from then on.
      uint32_t act[L];
      sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
        constexpr int ii = decltype(iic)::value;
        act[ii] = (8 * ii + r < K) ? 0x7FFFFF80u : 0u;
      });
      bool singular = false;
      sfor<0, L>([&](auto kbc) __attribute__((always_inline)) {
        constexpr int kb = decltype(kbc)::value;
#pragma clang loop unroll(disable)
        for (int cc = 0; cc < 8; ++cc) {
          const int k = 8 * kb + cc;
          if (k >= K) break;
          // 1. pivot search down column k among the rows still active
          uint32_t key0 = 0;
          sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
            constexpr int ii = decltype(iic)::value;
            const uint32_t hi = (uint32_t)__double2hiint(a[ii][kb]);
            key0 = umax(key0, (hi & act[ii]) | (uint32_t)ii);
          });
          const uint32_t kmax = __builtin_amdgcn_readlane(group8_max(key0), 8 * cc);
          if ((kmax & 0x7FFFFF80u) == 0u) singular = true;
          const int iip = (int)(kmax & 15u);
          const unsigned long long who =
              __ballot(key0 == kmax) & (0xFFull << (8 * cc));
          const int rp = (__ffsll((long long)who) - 1) & 7;
          const int piv = 8 * iip + rp;
          // 2. one uniform case per row block: retire the pivot row, write
          //    it to LDS, and zero the pivot element of column k in place
          //    (the column is finished after this step), so the column of
          //    multipliers taken below carries zero for the pivot row and
          //    the update needs no per-row test; the pivot value itself
          //    comes by readlane, so its reciprocal is under way while the
          //    broadcasts are in flight
          double upiv = 0.0;
          sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
            constexpr int ii = decltype(iic)::value;
            if (iip == ii) {
              __asm__ volatile("; pivot row out %0" ::"i"(ii));
              upiv = readlane_f64(a[ii][kb], 8 * cc + rp);
              act[ii] = (r == rp) ? 0u : act[ii];
              if (r == rp) {
                sfor<kb, LC>([&](auto jjc) __attribute__((always_inline)) {
                  constexpr int jj = decltype(jjc)::value;
                  ubuf[c * LC + jj] = a[ii][jj];
                });
                if (c == cc) a[ii][kb] = 0.0;
              }
            }
          });
          if (lane == 0) srank[piv] = k;
          if (!(upiv != 0.0)) singular = true;
          const double dk = singular ? 0.0 : recip(upiv);
          wsync();
          if (lane == 0) dinv[k] = dk;
          // 3. rank-1 update
          double u[LC], lv[L];
          sfor<kb, LC>([&](auto jjc) __attribute__((always_inline)) {
            constexpr int jj = decltype(jjc)::value;
            u[jj] = ubuf[c * LC + jj];
          });
          // the multipliers lane to lane: lane (r, c) takes column k from
          // lane (r, cc) by ds_bpermute (no LDS store and reload; 1M-node
          // ball: 5.30 -> 5.24 ms, the same bits)
          const int src_l = (r + 8 * cc) << 2;
          sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
            constexpr int ii = decltype(iic)::value;
            lv[ii] = bperm_f64(src_l, a[ii][kb]);
          });
          // Gauss-Jordan: every row but the pivot row is eliminated, the
          // rows pivoted earlier included, so no back substitution follows
          sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
            constexpr int ii = decltype(iic)::value;
            const double l = lv[ii] * dk;
            sfor<kb, LC>([&](auto jjc) __attribute__((always_inline)) {
              constexpr int jj = decltype(jjc)::value;
              a[ii][jj] = fma(-l, u[jj], a[ii][jj]);
            });
          });
          wsync();
        }
      });
      // ---- solution: the row slot pivoted at step j holds u_jj x_j ----
      // Every step of a nonsingular system pivots a row still active, so
      // each of the K slots gets exactly one rank.  A singular system may
      // rank one slot twice and leave another with a stale rank; its slots
      // are then mapped to themselves, which writes each of its weights
      // exactly once, as NaN (and so makes Lambda NaN too).
      if (singular) {
        for (int t = lane; t < S; t += 64) srank[t] = t;
        wsync();
      }
      int rank[L];
      double rdk[L];
      sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
        constexpr int ii = decltype(iic)::value;
        const bool live = 8 * ii + r < K;
        rank[ii] = live ? srank[8 * ii + r] : 1 << 20;
        rdk[ii] = live ? dinv[rank[ii]] : 0.0;
      });
      // ---- unscale, write rows, Lebesgue values ----
      // row slot with rank j holds the unknown x_j; weights are x_j, j < n
      const int32_t ckp = ck_s;
      const double sinv = sv_s[3];
      const int32_t* stnp = P.knn + (int64_t)ckp * n;
      if (singular && lane == 0) report(P.st, ORBF_ESINGULAR, ckp);
      sfor<0, PL>([&](auto jpc) __attribute__((always_inline)) {
        constexpr int jp = decltype(jpc)::value;
        const int e = 8 * jp + c;
        const bool live = e < nb;
        const int32_t row = live ? stnp[cols_s[cb + e]] : 0;
        double lam = 0.0;
        sfor<0, L>([&](auto iic) __attribute__((always_inline)) {
          constexpr int ii = decltype(iic)::value;
          const int j = rank[ii];
          if (live && j < n) {
            const double w = singular ? NAN : (a[ii][L + jp] * rdk[ii]) * sinv;
            if (!accept_mode) P.W[(int64_t)row * n + j] = w;
            lam += fabs(w);
          }
        });
        lam += __shfl_xor(lam, 1, 64);
        lam += __shfl_xor(lam, 2, 64);
        lam += __shfl_xor(lam, 4, 64);
        if (live && r == 0) {
          if (accept_mode) {
            lam_s[cb + e] = lam;
          } else {
            if (P.lebesgue) P.lebesgue[row] = lam;
            if (explicit_rows && P.owner_out) P.owner_out[row] = row;
          }
        }
      });
      wsync();
    }
    if (accept_mode) {
      // keep node e iff it is the center or Lambda_e <= tau * Lambda_ref
      // (eq. calLstab with the threshold tau)
      const double lref = lam_s[refcol_s];
      // radial prefix: nothing at or after the first failing ball node
      int efail = nball;
      if (P.tau_mode == 1) {
        for (int e0 = 0; e0 < nball; e0 += 64) {
          const int e = e0 + lane;
          const bool fails =
              e < nball && cols_s[e] != 0 && !(lam_s[e] <= P.tau * lref);
          const unsigned long long fb = __ballot(fails);
          if (fb) {
            efail = e0 + __ffsll((long long)fb) - 1;
            break;
          }
        }
      }
      for (int e = lane; e < nball; e += 64) {  // the appended reference
                                                // column is not a row
        const int q = cols_s[e];
        const bool acc = q == 0 || (e < efail && lam_s[e] <= P.tau * lref);
        // only candidate positions (the covering's masks) carry a bit
        const uint64_t word = P.ball[2 * (int64_t)ck_s + (q >> 6)];
        if (acc && q != 0 && ((word >> (q & 63)) & 1ull))
          atomicOr(&accw_s[q >> 6], 1ull << (q & 63));
      }
      wsync();
      if (lane == 0) {
        P.accept[2 * (int64_t)ck_s] = accw_s[0];
        P.accept[2 * (int64_t)ck_s + 1] = accw_s[1];
      }
      wsync();
    }
  }
}

// Launch the variant with L row blocks: acceptance mode (16 right-hand
// sides per pass) or pl = 1, 2, 3 blocks of eight right-hand sides.
template <int LL>
void launch_reg_variant(orbf_ctx* ctx, const WeightsParams& P, int64_t grid,
                        int pl, size_t dyn) {
  if (P.accept)
    hipLaunchKernelGGL((weights_reg_kernel<LL, 2, true>), dim3((unsigned)grid),
                       dim3(64), dyn, ctx->stream, P);
  else if (pl == 1)
    hipLaunchKernelGGL((weights_reg_kernel<LL, 1, false>), dim3((unsigned)grid),
                       dim3(64), dyn, ctx->stream, P);
  else if (pl == 3)
    hipLaunchKernelGGL((weights_reg_kernel<LL, 3, false>), dim3((unsigned)grid),
                       dim3(64), dyn, ctx->stream, P);
  else
    hipLaunchKernelGGL((weights_reg_kernel<LL, 2, false>), dim3((unsigned)grid),
                       dim3(64), dyn, ctx->stream, P);
}

}  // namespace

// the variants, instantiated in three translation units so they compile in
// parallel; each returns false if none of its variants covers K
bool launch_weights_reg_3_6(orbf_ctx* ctx, const WeightsParams& P,
                            int64_t grid, int pl, size_t dyn);
bool launch_weights_reg_7_8(orbf_ctx* ctx, const WeightsParams& P,
                            int64_t grid, int pl, size_t dyn);
bool launch_weights_reg_9(orbf_ctx* ctx, const WeightsParams& P,
                          int64_t grid, int pl, size_t dyn);

}  // namespace orbf
