// Shared pieces of the two weights kernels: launch parameters and the
// operator formulas of the local saddle system (Sec. 4.1, eqs.
// rbffd_linsys / orbffd_rhs) in scaled coordinates.
#pragma once

#include <math.h>

#include <type_traits>

#include "orbf_internal.hpp"

namespace orbf {

struct WeightsParams {
  const double* xyz;
  const int32_t* knn;
  const double* rho2;
  const int32_t* centers;   // covered rows: centers list (device)
  const int64_t* n_centers; // covered rows: number of centers (device)
  const int32_t* rows;      // explicit rows (each on its own stencil)
  int64_t n_rows;
  const int32_t* owner;     // covered rows: row e is computed by owner[e]
  int64_t N;
  int32_t* owner_out;       // explicit rows: owner[row] = row
  const double* normals;    // explicit rows, NEUMANN: n_rows * d
  // M * 3 monomial exponents, graded lex, passed by value (no host copy
  // on the stream, so a build can be captured in a graph); M <= 80 since
  // n >= M and n + M <= 160
  int8_t ex[3 * 80];
  double* W;                // N * n
  double* lebesgue;         // N or null
  // acceptance mode (Lebesgue covering): solve the ball columns of each
  // listed center plus its reference column and record which pass
  const uint64_t* ball;     // 2 words per node: ball positions q (j > c)
  uint64_t* accept;         // 2 words per node: accepted positions q
  double tau;
  // 0: each ball node kept or rejected on its own; 1: radial prefix (the
  // ball shrunk to just inside its first node that fails, claimed or not,
  // which needs the whole eligible ball: eligibility and (1-delta)^2)
  int tau_mode;
  const uint8_t* eligible;
  double t2;
  // FP32 + refinement: steps per row (or null), and the list of centers the
  // FP64 kernel must solve again (with its device counter)
  int32_t* ir_steps;
  int ir_max;               // corrections allowed before the FP64 fallback
  int32_t* fb_list;
  int64_t* fb_count;
  DevStatus* st;
  int d, n, m, l, M, K, op;
};

__device__ __forceinline__ double ipow_small(double v, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= v;
  return r;
}

// psi(p) = p0^e0 p1^e1 p2^e2
__device__ __forceinline__ double monomial(const double* p, const int8_t* e,
                                           int d) {
  double v = ipow_small(p[0], e[0]) * ipow_small(p[1], e[1]);
  if (d == 3) v *= ipow_small(p[2], e[2]);
  return v;
}

// sqrt(x) for x >= 0 from the hardware reciprocal-square-root estimate and
// two Newton steps on s^2 = x (accurate to a few ulp; 0 for x = 0)
__device__ __forceinline__ double sqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y;
  const double h = 0.5 * y;
  s = fma(fma(-s, s, x), h, s);
  s = fma(fma(-s, s, x), h, s);
  return x > 0.0 ? s : 0.0;
}

// |x|^m from r2 = |x|^2, m odd: r * r2^((m-1)/2)
__device__ __forceinline__ double phs(double r2, int m) {
  double p = sqrt_nr(r2);
  for (int i = 0; i < (m - 1) / 2; ++i) p *= r2;
  return p;
}

// L |x - x_j|^m at x, with (dx,dy,dz) = x - x_j and r2 = |x - x_j|^2:
// Laplacian m (m + d - 2) r^(m-2); identity r^m; a first derivative along
// the unit vector (n0, n1, n2) (normal, or e_a for d/dx_a):
// m r^(m-2) (x - x_j) . n
__device__ __forceinline__ double phs_op(double dx, double dy, double dz,
                                         double r2, int m, int d, int op,
                                         double n0, double n1, double n2) {
  double p = sqrt_nr(r2);  // r^(m-2), m - 2 odd
  for (int i = 0; i < (m - 3) / 2; ++i) p *= r2;
  if (op == ORBF_OP_LAPLACIAN) return (double)(m * (m + d - 2)) * p;
  if (op == ORBF_OP_IDENTITY) return p * r2;
  const double dot = dx * n0 + dy * n1 + dz * n2;
  return ((double)m * p) * dot;
}

// 1 / rho^theta: theta = 2 (Laplacian), 0 (identity), 1 (first derivatives)
__device__ __forceinline__ double op_unscale(int op, double rho2,
                                             double rho) {
  return op == ORBF_OP_LAPLACIAN ? 1.0 / rho2
         : op == ORBF_OP_IDENTITY ? 1.0
                                  : 1.0 / rho;
}

// direction of a d/dx_a operator: component a of e_a is 1
__device__ __forceinline__ void op_axis(int op, double (&nrm)[3]) {
  if (op >= ORBF_OP_DX && op <= ORBF_OP_DZ) nrm[op - ORBF_OP_DX] = 1.0;
}

// Monomials from a power table pw[a * (l + 1) + e] = p_a^e of one point.
__device__ __forceinline__ double monomial_pw(const double* pw, int l1,
                                              const int8_t* e) {
  return pw[e[0]] * pw[l1 + e[1]] * pw[2 * l1 + e[2]];
}

// L psi from the power table: Laplacian sum_a e_a (e_a - 1) p^(e - 2 eps_a),
// the identity p^e, or a first derivative sum_a n_a e_a p^(e - eps_a)
__device__ __forceinline__ double monomial_op_pw(const double* pw, int l1,
                                                 const int8_t* e, int op,
                                                 double n0, double n1,
                                                 double n2) {
  const int e0 = e[0], e1 = e[1], e2 = e[2];
  const double* p0 = pw;
  const double* p1 = pw + l1;
  const double* p2 = pw + 2 * l1;
  double s = 0.0;
  if (op == ORBF_OP_IDENTITY) {
    s = p0[e0] * p1[e1] * p2[e2];
  } else if (op == ORBF_OP_LAPLACIAN) {
    if (e0 >= 2) s += (double)(e0 * (e0 - 1)) * (p0[e0 - 2] * p1[e1] * p2[e2]);
    if (e1 >= 2) s += (double)(e1 * (e1 - 1)) * (p0[e0] * p1[e1 - 2] * p2[e2]);
    if (e2 >= 2) s += (double)(e2 * (e2 - 1)) * (p0[e0] * p1[e1] * p2[e2 - 2]);
  } else {
    if (e0 >= 1) s += n0 * ((double)e0 * (p0[e0 - 1] * p1[e1] * p2[e2]));
    if (e1 >= 1) s += n1 * ((double)e1 * (p0[e0] * p1[e1 - 1] * p2[e2]));
    if (e2 >= 1) s += n2 * ((double)e2 * (p0[e0] * p1[e1] * p2[e2 - 1]));
  }
  return s;
}

// ---- wavefront helpers shared by the register-resident kernels ----

// compile-time loop: f(integral_constant<B>), ..., f(integral_constant<E-1>)
template <int B, int E, class F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) {
  return a > b ? a : b;
}

// max of a 32-bit key over each aligned group of 8 lanes (DPP, no LDS)
__device__ __forceinline__ uint32_t group8_max(uint32_t k) {
  k = umax(k, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)k, 0xB1, 0xF, 0xF, false));
  k = umax(k, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)k, 0x4E, 0xF, 0xF, false));
  k = umax(k, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)k, 0x141, 0xF, 0xF, false));
  return k;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// reciprocal of a wave-uniform value: hardware estimate + 2 Newton steps
__device__ __forceinline__ double recip(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  y = fma(fma(-x, y, 1.0), y, y);
  return y;
}

bool launch_weights_reg(orbf_ctx* ctx, const WeightsParams& P, int64_t grid,
                        int pl = 2);
bool launch_weights_ir(orbf_ctx* ctx, const WeightsParams& P, int64_t grid);
bool launch_weights_wg(orbf_ctx* ctx, const WeightsParams& P, int64_t work);
bool launch_weights_mfma(orbf_ctx* ctx, const WeightsParams& P, int64_t grid);
void launch_ir_prepare(orbf_ctx* ctx, int32_t* ir_steps, int64_t N,
                       int64_t* fb_count);
orbf_status launch_lebesgue_cover(orbf_ctx* ctx, const WeightsParams& P0,
                                  double t2, const uint8_t* eligible,
                                  int32_t* centers, int64_t* n_centers,
                                  int32_t* owner);

}  // namespace orbf
