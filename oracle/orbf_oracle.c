/*
 * orbf_oracle.c -- CPU oracle for the overlapped RBF-FD differentiation
 * matrix (DM) build.  TEST INFRASTRUCTURE ONLY: it is called by the tests,
 * by the smoke check and by the CPU-baseline leg of the benchmark, never by
 * the product path, and it shares no code with the HIP library.
 *
 * Everything is FP64, plain loops, no BLAS, compiled with -ffp-contract=off
 * so that every product and sum is rounded separately.  Each function names
 * the passage of the paper it follows:
 *
 *   Sec. 2            stencils (n nearest nodes, center first), the augmented
 *                     local interpolant and its block system, degree rule;
 *   Sec. 4.1          the augmented RBF-FD system (eq. rbffd_linsys), the
 *                     stencil width rho_k, the retention distance
 *                     r_k = (1-delta) rho_k, the retention ball and set R_k,
 *                     the multi-RHS system (eqs. orbffd_eq, orbffd_rhs), the
 *                     scatter L(R_i, I_j) = W_{j,i} and the rule that a row
 *                     computed once is never recomputed;
 *   Sec. 4.2.1        local L-Lebesgue function = column 1-norm of W^phi and
 *                     the acceptance test (eq. calLstab);
 *   Sec. 5            interior/boundary split of the DM rows.
 *
 * Readings where the paper is silent are fixed as follows (also listed with
 * reasons in the design notes of the repository):
 *   - ties in the kNN order are broken by the global index;
 *   - the retention ball is closed: d^2 <= ((1-delta)*(1-delta))*rho^2;
 *   - nodes are traversed in ascending index;
 *   - the local system is solved in coordinates shifted by x_k and scaled by
 *     1/rho_k, then unscaled by rho_k^theta (theta = 2 for the Laplacian,
 *     1 for a normal derivative); the weights do not depend on this choice
 *     in exact arithmetic;
 *   - monomials are graded-lexicographic;
 *   - Gaussian elimination with row partial pivoting, first maximum wins;
 *   - Lebesgue test: keep node e iff e is the center or
 *     Lambda_e <= tau * Lambda_ref (tau = 1 is the paper's test), where ref
 *     is the stencil node nearest the stencil centroid (lowest position on
 *     ties), centroid and distances computed in coordinates relative to x_k.
 */
#include "orbf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */

/* squared distance ((dx*dx)+(dy*dy))+(dz*dz), left to right */
static double sqdist(const double* a, const double* b, int d) {
  double dx = a[0] - b[0];
  double s = dx * dx;
  double dy = a[1] - b[1];
  s = s + dy * dy;
  if (d == 3) {
    double dz = a[2] - b[2];
    s = s + dz * dz;
  }
  return s;
}

static int key_less(double da, int32_t ja, double db, int32_t jb) {
  return da < db || (da == db && ja < jb);
}

/* keep the n smallest keys (d2, j) in ascending order; cnt = current fill */
static void topn_insert(double* kd, int32_t* kj, int* cnt, int n, double d2,
                        int32_t j) {
  int c = *cnt;
  if (c == n) {
    if (!key_less(d2, j, kd[n - 1], kj[n - 1])) return;
    c = n - 1; /* drop the last */
  }
  int p = c;
  while (p > 0 && key_less(d2, j, kd[p - 1], kj[p - 1])) {
    kd[p] = kd[p - 1];
    kj[p] = kj[p - 1];
    p--;
  }
  kd[p] = d2;
  kj[p] = j;
  *cnt = c + 1;
}

int orc_num_monomials(int d, int l) {
  /* C(l+d, d) */
  long num = 1, den = 1;
  for (int i = 1; i <= d; i++) {
    num *= (l + i);
    den *= i;
  }
  return (int)(num / den);
}

/* Sec. 2: choose s with C(s+d,d) = n/2; take the largest s whose number of
 * monomials does not exceed n/2 (2D: floor((sqrt(4n+1)-3)/2)). */
void orc_degree_rule(int d, int n, int* s_out, int* M_out) {
  int s = 0;
  while (2 * orc_num_monomials(d, s + 1) <= n) s++;
  *s_out = s;
  *M_out = orc_num_monomials(d, s);
}

static int check_nodes(const double* x, int64_t N, int d) {
  for (int64_t i = 0; i < N * d; i++)
    if (!isfinite(x[i])) return ORC_EINVAL;
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* kNN (Sec. 2: stencil = node plus its n-1 nearest neighbours)         */
/* ------------------------------------------------------------------ */

int orc_knn_one(const double* x, int64_t N, int d, int n, int64_t q,
                int32_t* knn_q, double* rho2_q) {
  if ((d != 2 && d != 3) || n < 1 || n > N || q < 0 || q >= N)
    return ORC_EINVAL;
  double* kd = (double*)malloc(sizeof(double) * n);
  int32_t* kj = (int32_t*)malloc(sizeof(int32_t) * n);
  int cnt = 0, dup = 0;
  for (int64_t j = 0; j < N; j++) {
    double d2 = sqdist(x + q * d, x + j * d, d);
    if (d2 == 0.0 && j != q) dup = 1;
    topn_insert(kd, kj, &cnt, n, d2, (int32_t)j);
  }
  memcpy(knn_q, kj, sizeof(int32_t) * n);
  *rho2_q = kd[n - 1];
  free(kd);
  free(kj);
  return dup ? ORC_EDUPLICATE : ORC_OK;
}

int orc_knn_brute(const double* x, int64_t N, int d, int n, int32_t* knn,
                  double* rho2) {
  if ((d != 2 && d != 3) || n < 1 || n > N || N > INT32_MAX) return ORC_EINVAL;
  if (check_nodes(x, N, d)) return ORC_EINVAL;
  int err = ORC_OK;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < N; i++) {
    int r = orc_knn_one(x, N, d, n, i, knn + i * n, rho2 + i);
    if (r != ORC_OK) {
#pragma omp critical
      err = r;
    }
  }
  return err;
}

int orc_knn_grid(const double* x, int64_t N, int d, int n, int32_t* knn,
                 double* rho2) {
  if ((d != 2 && d != 3) || n < 1 || n > N || N > INT32_MAX) return ORC_EINVAL;
  if (check_nodes(x, N, d)) return ORC_EINVAL;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int a = 0; a < d; a++) lo[a] = hi[a] = x[a];
  for (int64_t i = 0; i < N; i++)
    for (int a = 0; a < d; a++) {
      if (x[i * d + a] < lo[a]) lo[a] = x[i * d + a];
      if (x[i * d + a] > hi[a]) hi[a] = x[i * d + a];
    }
  /* cell side: about two nodes per cell on average over the bounding box */
  double vol = 1.0;
  for (int a = 0; a < d; a++) vol *= (hi[a] - lo[a] > 0 ? hi[a] - lo[a] : 1.0);
  double s = pow(2.0 * vol / (double)N, 1.0 / d);
  int64_t nc[3] = {1, 1, 1}, ncell = 1;
  for (int a = 0; a < d; a++) {
    nc[a] = (int64_t)((hi[a] - lo[a]) / s) + 1;
    if (nc[a] < 1) nc[a] = 1;
    ncell *= nc[a];
  }
  int32_t* cell_of = (int32_t*)malloc(sizeof(int32_t) * N);
  int64_t* start = (int64_t*)calloc(ncell + 1, sizeof(int64_t));
  int32_t* sorted = (int32_t*)malloc(sizeof(int32_t) * N);
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ncell);
  for (int64_t i = 0; i < N; i++) {
    int64_t c = 0;
    for (int a = d - 1; a >= 0; a--) {
      int64_t ca = (int64_t)((x[i * d + a] - lo[a]) / s);
      if (ca >= nc[a]) ca = nc[a] - 1;
      if (ca < 0) ca = 0;
      c = c * nc[a] + ca;
    }
    cell_of[i] = (int32_t)c;
    start[c + 1]++;
  }
  for (int64_t c = 0; c < ncell; c++) start[c + 1] += start[c];
  memcpy(fill, start, sizeof(int64_t) * ncell);
  for (int64_t i = 0; i < N; i++) sorted[fill[cell_of[i]]++] = (int32_t)i;

  int err = ORC_OK;
#pragma omp parallel
  {
    double* kd = (double*)malloc(sizeof(double) * n);
    int32_t* kj = (int32_t*)malloc(sizeof(int32_t) * n);
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; i++) {
      const double* xi = x + i * d;
      int64_t ci[3] = {0, 0, 0};
      for (int a = 0; a < d; a++) {
        int64_t ca = (int64_t)((xi[a] - lo[a]) / s);
        if (ca >= nc[a]) ca = nc[a] - 1;
        if (ca < 0) ca = 0;
        ci[a] = ca;
      }
      int cnt = 0, dup = 0;
      for (int64_t R = 0;; R++) {
        /* scan the cells at Chebyshev cell distance exactly R */
        int64_t lo3[3] = {0, 0, 0}, hi3[3] = {0, 0, 0};
        for (int a = 0; a < d; a++) {
          lo3[a] = ci[a] - R;
          hi3[a] = ci[a] + R;
        }
        for (int64_t cz = (d == 3 ? lo3[2] : 0); cz <= (d == 3 ? hi3[2] : 0);
             cz++)
          for (int64_t cy = lo3[1]; cy <= hi3[1]; cy++)
            for (int64_t cx = lo3[0]; cx <= hi3[0]; cx++) {
              int64_t cc[3] = {cx, cy, cz};
              int onshell = 0, inside = 1;
              for (int a = 0; a < d; a++) {
                if (cc[a] < 0 || cc[a] >= nc[a]) inside = 0;
                if (cc[a] == lo3[a] || cc[a] == hi3[a]) onshell = 1;
              }
              if (!inside || !onshell) continue;
              int64_t c = (d == 3 ? (cz * nc[1] + cy) * nc[0] + cx
                                  : cy * nc[0] + cx);
              for (int64_t t = start[c]; t < start[c + 1]; t++) {
                int32_t j = sorted[t];
                double d2 = sqdist(xi, x + (int64_t)j * d, d);
                if (d2 == 0.0 && j != i) dup = 1;
                topn_insert(kd, kj, &cnt, n, d2, j);
              }
            }
        /* distance from x_i to the boundary of the scanned block; sides at
         * the edge of the grid hold no further nodes */
        double b = INFINITY;
        for (int a = 0; a < d; a++) {
          if (ci[a] - R > 0) {
            double f = lo[a] + (double)(ci[a] - R) * s;
            double g = xi[a] - f;
            if (g < b) b = g;
          }
          if (ci[a] + R < nc[a] - 1) {
            double f = lo[a] + (double)(ci[a] + R + 1) * s;
            double g = f - xi[a];
            if (g < b) b = g;
          }
        }
        if (isinf(b)) break; /* the whole grid has been scanned */
        /* the margin covers rounding in d2, in b and in the cell index */
        if (cnt == n && b > 0 && kd[n - 1] < b * b * (1.0 - 1e-9)) break;
      }
      memcpy(knn + i * n, kj, sizeof(int32_t) * n);
      rho2[i] = kd[n - 1];
      if (dup) {
#pragma omp critical
        err = ORC_EDUPLICATE;
      }
    }
    free(kd);
    free(kj);
  }
  free(cell_of);
  free(start);
  free(sorted);
  free(fill);
  return err;
}

/* ------------------------------------------------------------------ */
/* greedy covering (Sec. 4.1: retention ball, rows never recomputed)    */
/* ------------------------------------------------------------------ */

static int elig(const uint8_t* e, int64_t i) { return e == NULL || e[i] != 0; }

int orc_cover(const double* x, int64_t N, int d, int n, const int32_t* knn,
              const double* rho2, double delta, const uint8_t* eligible,
              int32_t* owner, int32_t* centers, int64_t* n_centers) {
  if ((d != 2 && d != 3) || n < 1 || n > N || !(delta >= 0.0 && delta <= 1.0))
    return ORC_EINVAL;
  for (int64_t i = 0; i < N; i++) owner[i] = -1;
  int64_t nc = 0;
  double t = 1.0 - delta;
  double t2 = t * t;
  for (int64_t k = 0; k < N; k++) {
    if (!elig(eligible, k) || owner[k] != -1) continue;
    centers[nc++] = (int32_t)k;
    double thr = t2 * rho2[k];
    for (int q = 0; q < n; q++) {
      int32_t j = knn[k * n + q];
      if (!elig(eligible, j) || owner[j] != -1) continue;
      if (sqdist(x + k * d, x + (int64_t)j * d, d) <= thr) owner[j] = (int32_t)k;
    }
  }
  *n_centers = nc;
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* local weights (Sec. 4.1, eqs. rbffd_linsys / orbffd_eq / orbffd_rhs)  */
/* ------------------------------------------------------------------ */

/* exponents of the monomials of degree <= l, graded lexicographic */
static int monomial_exponents(int d, int l, int* ex /* M*3 */) {
  int t = 0;
  for (int deg = 0; deg <= l; deg++) {
    if (d == 2) {
      for (int a = deg; a >= 0; a--) {
        ex[3 * t + 0] = a;
        ex[3 * t + 1] = deg - a;
        ex[3 * t + 2] = 0;
        t++;
      }
    } else {
      for (int a = deg; a >= 0; a--)
        for (int b = deg - a; b >= 0; b--) {
          ex[3 * t + 0] = a;
          ex[3 * t + 1] = b;
          ex[3 * t + 2] = deg - a - b;
          t++;
        }
    }
  }
  return t;
}

static double ipow(double v, int e) {
  double r = 1.0;
  for (int i = 0; i < e; i++) r = r * v;
  return r;
}

static double monomial(const double* p, const int* e, int d) {
  double r = ipow(p[0], e[0]) * ipow(p[1], e[1]);
  if (d == 3) r = r * ipow(p[2], e[2]);
  return r;
}

/* Laplacian of p^e: sum_a e_a (e_a - 1) p^(e - 2 eps_a) */
static double monomial_lap(const double* p, const int* e, int d) {
  double s = 0.0;
  for (int a = 0; a < d; a++) {
    if (e[a] < 2) continue;
    int f[3] = {e[0], e[1], e[2]};
    f[a] -= 2;
    s = s + (double)(e[a] * (e[a] - 1)) * monomial(p, f, d);
  }
  return s;
}

/* normal derivative of p^e: sum_a nrm_a e_a p^(e - eps_a) */
static double monomial_dn(const double* p, const int* e, const double* nrm,
                          int d) {
  double s = 0.0;
  for (int a = 0; a < d; a++) {
    if (e[a] < 1) continue;
    int f[3] = {e[0], e[1], e[2]};
    f[a] -= 1;
    s = s + nrm[a] * ((double)e[a] * monomial(p, f, d));
  }
  return s;
}

/* r^k for odd k >= 1 from r2 = r^2: r * (r2)^((k-1)/2) */
static double odd_power(double r2, int k) {
  return sqrt(r2) * ipow(r2, (k - 1) / 2);
}

/* Gaussian elimination with row partial pivoting (first maximum) of the
 * K x K matrix A (row-major, destroyed) applied to the K x R right-hand
 * sides B (row-major, overwritten by the solution). */
static int ge_solve(int K, int R, double* A, double* B) {
  for (int k = 0; k < K; k++) {
    int piv = k;
    double best = fabs(A[k * K + k]);
    for (int r = k + 1; r < K; r++)
      if (fabs(A[r * K + k]) > best) {
        best = fabs(A[r * K + k]);
        piv = r;
      }
    if (best == 0.0) return ORC_ESINGULAR;
    if (piv != k) {
      for (int c = 0; c < K; c++) {
        double tmp = A[k * K + c];
        A[k * K + c] = A[piv * K + c];
        A[piv * K + c] = tmp;
      }
      for (int c = 0; c < R; c++) {
        double tmp = B[k * R + c];
        B[k * R + c] = B[piv * R + c];
        B[piv * R + c] = tmp;
      }
    }
    for (int r = k + 1; r < K; r++) {
      double f = A[r * K + k] / A[k * K + k];
      for (int c = k + 1; c < K; c++) A[r * K + c] = A[r * K + c] - f * A[k * K + c];
      A[r * K + k] = 0.0;
      for (int c = 0; c < R; c++) B[r * R + c] = B[r * R + c] - f * B[k * R + c];
    }
  }
  for (int k = K - 1; k >= 0; k--)
    for (int c = 0; c < R; c++) {
      double s = B[k * R + c];
      for (int j = k + 1; j < K; j++) s = s - A[k * K + j] * B[j * R + c];
      B[k * R + c] = s / A[k * K + k];
    }
  return ORC_OK;
}

int orc_stencil_weights(int d, int m, int l, int op, int n, const double* P,
                        int ne, const double* E, const double* nrm,
                        double* W) {
  /* l = -1: no polynomial augmentation (M = 0), the unaugmented RBF-FD
   * system A w = L phi that Sec. 4.3 also counts */
  if ((d != 2 && d != 3) || m < 3 || (m % 2) == 0 || l < -1 || ne < 1)
    return ORC_EINVAL;
  if (op < ORC_OP_LAPLACIAN || op > ORC_OP_IDENTITY) return ORC_EINVAL;
  if (op == ORC_OP_NEUMANN && nrm == NULL) return ORC_EINVAL;
  if (op == ORC_OP_DZ && d != 3) return ORC_EINVAL;
  int M = orc_num_monomials(d, l);
  if (n < M || n < 1) return ORC_EINVAL;
  int K = n + M;

  /* stencil width (Sec. 4.1): largest distance from the center */
  double rho2 = 0.0;
  for (int j = 0; j < n; j++) {
    double r2 = sqdist(P, P + j * d, d);
    if (r2 > rho2) rho2 = r2;
  }
  if (!(rho2 > 0.0)) return ORC_EINVAL;
  double rho = sqrt(rho2);

  int* ex = (int*)malloc(sizeof(int) * 3 * M);
  monomial_exponents(d, l, ex);
  double* xi = (double*)malloc(sizeof(double) * n * 3);
  double* ev = (double*)malloc(sizeof(double) * ne * 3);
  double* A = (double*)calloc((size_t)K * K, sizeof(double));
  double* B = (double*)calloc((size_t)K * ne, sizeof(double));
  for (int j = 0; j < n; j++)
    for (int a = 0; a < d; a++) xi[j * 3 + a] = (P[j * d + a] - P[a]) / rho;
  for (int e = 0; e < ne; e++)
    for (int a = 0; a < d; a++) ev[e * 3 + a] = (E[e * d + a] - P[a]) / rho;

  /* A_hat = [A Psi; Psi^T 0] with A_ij = |xi_i - xi_j|^m */
  for (int i = 0; i < n; i++) {
    for (int j = 0; j < n; j++)
      A[i * K + j] = odd_power(sqdist(xi + i * 3, xi + j * 3, d), m);
    for (int t = 0; t < M; t++) {
      double v = monomial(xi + i * 3, ex + 3 * t, d);
      A[i * K + n + t] = v;
      A[(n + t) * K + i] = v;
    }
  }
  /* B_hat: column e is L applied to each basis function at point e; a
   * first derivative d/dx_a is the directional derivative along e_a */
  for (int e = 0; e < ne; e++) {
    const double* pe = ev + e * 3;
    double dir[3] = {0.0, 0.0, 0.0};
    if (op == ORC_OP_NEUMANN)
      for (int a = 0; a < d; a++) dir[a] = nrm[e * d + a];
    else if (op >= ORC_OP_DX && op <= ORC_OP_DZ)
      dir[op - ORC_OP_DX] = 1.0;
    for (int j = 0; j < n; j++) {
      double r2 = sqdist(pe, xi + j * 3, d);
      double v;
      if (op == ORC_OP_LAPLACIAN) {
        /* Laplacian of r^m in d dimensions: m (m + d - 2) r^(m-2) */
        v = (double)(m * (m + d - 2)) * odd_power(r2, m - 2);
      } else if (op == ORC_OP_IDENTITY) {
        v = odd_power(r2, m);
      } else {
        /* gradient of r^m is m r^(m-2) (x - x_j) */
        double dot = 0.0;
        for (int a = 0; a < d; a++)
          dot = dot + (pe[a] - xi[j * 3 + a]) * dir[a];
        v = ((double)m * odd_power(r2, m - 2)) * dot;
      }
      B[j * ne + e] = v;
    }
    for (int t = 0; t < M; t++)
      B[(n + t) * ne + e] =
          (op == ORC_OP_LAPLACIAN)   ? monomial_lap(pe, ex + 3 * t, d)
          : (op == ORC_OP_IDENTITY) ? monomial(pe, ex + 3 * t, d)
                                    : monomial_dn(pe, ex + 3 * t, dir, d);
  }

  int st = ge_solve(K, ne, A, B);
  if (st == ORC_OK) {
    /* undo the 1/rho scaling: theta = 2 (Laplacian), 1 (first derivatives)
     * or 0 (identity) */
    double sc = (op == ORC_OP_LAPLACIAN) ? rho2
                : (op == ORC_OP_IDENTITY) ? 1.0
                                          : rho;
    for (int e = 0; e < ne; e++)
      for (int j = 0; j < n; j++) W[e * n + j] = B[j * ne + e] / sc;
  }
  free(ex);
  free(xi);
  free(ev);
  free(A);
  free(B);
  return st;
}

/* ------------------------------------------------------------------ */
/* DM rows (Sec. 4.1 scatter; Sec. 4.2.1 Lebesgue acceptance)           */
/* ------------------------------------------------------------------ */

/* stencil node nearest the centroid of the stencil (Sec. 4.2.1), computed
 * in coordinates relative to the center, sums in stencil order */
static int centroid_ref(const double* x, int d, int n, const int32_t* st) {
  const double* xk = x + (int64_t)st[0] * d;
  double c[3] = {0, 0, 0};
  for (int q = 0; q < n; q++)
    for (int a = 0; a < d; a++) c[a] = c[a] + (x[(int64_t)st[q] * d + a] - xk[a]);
  for (int a = 0; a < d; a++) c[a] = c[a] / (double)n;
  int best = 0;
  double bd = INFINITY;
  for (int q = 0; q < n; q++) {
    double e[3];
    for (int a = 0; a < d; a++) e[a] = (x[(int64_t)st[q] * d + a] - xk[a]) - c[a];
    double s = e[0] * e[0];
    s = s + e[1] * e[1];
    if (d == 3) s = s + e[2] * e[2];
    if (s < bd) {
      bd = s;
      best = q;
    }
  }
  return best;
}

static double l1norm(const double* w, int n) {
  double s = 0.0;
  for (int j = 0; j < n; j++) s = s + fabs(w[j]);
  return s;
}

/* weights of stencil k for the stencil positions qs[0..ne) */
static int stencil_cols(const double* x, int d, int n, int m, int l, int op,
                        const int32_t* st, int ne, const int* qs,
                        const double* nrm, double* P, double* E, double* W) {
  for (int j = 0; j < n; j++)
    for (int a = 0; a < d; a++) P[j * d + a] = x[(int64_t)st[j] * d + a];
  for (int e = 0; e < ne; e++)
    for (int a = 0; a < d; a++) E[e * d + a] = P[qs[e] * d + a];
  return orc_stencil_weights(d, m, l, op, n, P, ne, E, nrm, W);
}

/* covering first, then every center's columns independently */
static int covered_rows(const double* x, int64_t N, int d, int n, int m,
                        int l, int op, const int32_t* knn, const double* rho2,
                        double delta, const uint8_t* eligible, int32_t* owner,
                        int32_t* centers, int64_t* n_centers, double* Wrows,
                        double* lam, int nthreads) {
  int err = orc_cover(x, N, d, n, knn, rho2, delta, eligible, owner, centers,
                      n_centers);
  if (err) return err;
  {
    int64_t nc = *n_centers;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
      int* qs = (int*)malloc(sizeof(int) * n);
      double* P = (double*)malloc(sizeof(double) * n * d);
      double* E = (double*)malloc(sizeof(double) * n * d);
      double* W = (double*)malloc(sizeof(double) * n * n);
#pragma omp for schedule(dynamic, 16)
      for (int64_t c = 0; c < nc; c++) {
        int32_t k = centers[c];
        const int32_t* st = knn + (int64_t)k * n;
        int ne = 0;
        for (int q = 0; q < n; q++)
          if (owner[st[q]] == k) qs[ne++] = q;
        int r = stencil_cols(x, d, n, m, l, op, st, ne, qs, NULL, P, E, W);
        if (r != ORC_OK) {
#pragma omp critical
          err = r;
          continue;
        }
        for (int e = 0; e < ne; e++) {
          int32_t j = st[qs[e]];
          memcpy(Wrows + (int64_t)j * n, W + e * n, sizeof(double) * n);
          if (lam) lam[j] = l1norm(W + e * n, n);
        }
      }
      free(qs);
      free(P);
      free(E);
      free(W);
    }
  }
  return err;
}

int orc_overlapped_rows_op(const double* x, int64_t N, int d, int n, int m,
                           int l, int op, const int32_t* knn,
                           const double* rho2, double delta,
                           const uint8_t* eligible, int32_t* owner,
                           int32_t* centers, int64_t* n_centers,
                           double* Wrows, double* lam, int nthreads) {
  if ((d != 2 && d != 3) || n < 1 || n > N || !(delta >= 0.0 && delta <= 1.0))
    return ORC_EINVAL;
  if (n < orc_num_monomials(d, l) || m < 3 || m % 2 == 0) return ORC_EINVAL;
  if (op != ORC_OP_LAPLACIAN && op != ORC_OP_DX && op != ORC_OP_DY &&
      op != ORC_OP_DZ && op != ORC_OP_IDENTITY)
    return ORC_EINVAL;
  if (op == ORC_OP_DZ && d != 3) return ORC_EINVAL;
  return covered_rows(x, N, d, n, m, l, op, knn, rho2, delta, eligible, owner,
                      centers, n_centers, Wrows, lam, nthreads);
}

int orc_overlapped_rows(const double* x, int64_t N, int d, int n, int m, int l,
                        const int32_t* knn, const double* rho2, double delta,
                        double tau, const uint8_t* eligible, int32_t* owner,
                        int32_t* centers, int64_t* n_centers, double* Wrows,
                        double* lam, double* min_margin, int nthreads) {
  return orc_overlapped_rows_mode(x, N, d, n, m, l, knn, rho2, delta, tau, 0,
                                  eligible, owner, centers, n_centers, Wrows,
                                  lam, min_margin, nthreads);
}

int orc_overlapped_rows_mode(const double* x, int64_t N, int d, int n, int m,
                             int l, const int32_t* knn, const double* rho2,
                             double delta, double tau, int prefix,
                             const uint8_t* eligible, int32_t* owner,
                             int32_t* centers, int64_t* n_centers,
                             double* Wrows, double* lam, double* min_margin,
                             int nthreads) {
  if ((d != 2 && d != 3) || n < 1 || n > N || !(delta >= 0.0 && delta <= 1.0))
    return ORC_EINVAL;
  if (!(tau >= 1.0)) return ORC_EINVAL; /* tau = +inf disables the test */
  if (prefix != 0 && prefix != 1) return ORC_EINVAL;
  if (n < orc_num_monomials(d, l) || m < 3 || m % 2 == 0) return ORC_EINVAL;
  int err = ORC_OK;
  double margin = INFINITY;
  if (isinf(tau)) {
    err = covered_rows(x, N, d, n, m, l, ORC_OP_LAPLACIAN, knn, rho2, delta,
                       eligible, owner, centers, n_centers, Wrows, lam,
                       nthreads);
    if (min_margin) *min_margin = margin;
    return err;
  }

  /* finite tau: the acceptance of each column depends on the stencil only,
   * but which nodes are still unclaimed depends on the earlier centers, so
   * the loop is sequential in the traversal order */
  for (int64_t i = 0; i < N; i++) owner[i] = -1;
  int* qs = (int*)malloc(sizeof(int) * (n + 1));
  double* P = (double*)malloc(sizeof(double) * n * d);
  double* E = (double*)malloc(sizeof(double) * (n + 1) * d);
  double* W = (double*)malloc(sizeof(double) * (n + 1) * n);
  int64_t nc = 0;
  double t = 1.0 - delta;
  double t2 = t * t;
  for (int64_t k = 0; k < N && err == ORC_OK; k++) {
    if (!elig(eligible, k) || owner[k] != -1) continue;
    centers[nc++] = (int32_t)k;
    const int32_t* st = knn + k * n;
    double thr = t2 * rho2[k];
    int ne = 0, ref_col = -1;
    int ref = centroid_ref(x, d, n, st);
    for (int q = 0; q < n; q++) {
      int32_t j = st[q];
      /* the radial prefix tests every eligible node of the ball, claimed
       * or not: its cut depends on the stencil alone */
      if (!elig(eligible, j) || (!prefix && owner[j] != -1)) continue;
      if (sqdist(x + k * d, x + (int64_t)j * d, d) <= thr) {
        if (q == ref) ref_col = ne;
        qs[ne++] = q;
      }
    }
    int ncols = ne;
    if (ref_col < 0) {
      ref_col = ncols;
      qs[ncols++] = ref;
    }
    err = stencil_cols(x, d, n, m, l, ORC_OP_LAPLACIAN, st, ncols, qs, NULL,
                       P, E, W);
    if (err) break;
    double lref = l1norm(W + ref_col * n, n);
    /* radial prefix (the ball shrunk for this stencil): nothing at or
     * beyond the first ball node that fails the test is kept */
    int cut = ne;
    for (int e = 0; e < ne; e++) {
      int32_t j = st[qs[e]];
      double le = l1norm(W + e * n, n);
      int accept = (qs[e] == 0);
      if (!accept && e < cut) {
        accept = le <= tau * lref;
        /* the reference node compares its own column with itself */
        if (qs[e] != ref) {
          double mg = fabs(le - tau * lref) / (tau * lref);
          if (mg < margin) margin = mg;
        }
        if (!accept && prefix) cut = e;
      }
      if (!accept || owner[j] != -1) continue;
      owner[j] = (int32_t)k;
      memcpy(Wrows + (int64_t)j * n, W + e * n, sizeof(double) * n);
      if (lam) lam[j] = le;
    }
  }
  *n_centers = nc;
  if (min_margin) *min_margin = margin;
  free(qs);
  free(P);
  free(E);
  free(W);
  return err;
}

int orc_center_rows(const double* x, int64_t N, int d, int n, int m, int l,
                    int op, const int32_t* knn, int64_t n_rows,
                    const int32_t* rows, const double* nrm, int32_t* owner,
                    double* Wrows, int nthreads) {
  if ((d != 2 && d != 3) || n < 1 || n > N) return ORC_EINVAL;
  if (op == ORC_OP_NEUMANN && nrm == NULL) return ORC_EINVAL;
  int err = ORC_OK;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
  {
    double* P = (double*)malloc(sizeof(double) * n * d);
    double* E = (double*)malloc(sizeof(double) * d);
    double* W = (double*)malloc(sizeof(double) * n);
    int q0 = 0;
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_rows; i++) {
      int32_t b = rows[i];
      const int32_t* st = knn + (int64_t)b * n;
      int r = stencil_cols(x, d, n, m, l, op, st, 1, &q0,
                           nrm ? nrm + i * d : NULL, P, E, W);
      if (r != ORC_OK) {
#pragma omp critical
        err = r;
        continue;
      }
      memcpy(Wrows + (int64_t)b * n, W, sizeof(double) * n);
      owner[b] = b;
    }
    free(P);
    free(E);
    free(W);
  }
  return err;
}

/* ------------------------------------------------------------------ */
/* CSR (Sec. 4.1: L(R^k_i, I^k_j) = W^{phi,k}_{j,i})                     */
/* ------------------------------------------------------------------ */

int orc_csr(int64_t N, int n, const int32_t* knn, const int32_t* owner,
            const double* Wrows, int64_t* row_ptr, int32_t* col, double* val) {
  row_ptr[0] = 0;
  for (int64_t e = 0; e < N; e++) {
    int64_t base = row_ptr[e];
    if (owner[e] < 0) {
      row_ptr[e + 1] = base;
      continue;
    }
    const int32_t* st = knn + (int64_t)owner[e] * n;
    /* insertion sort of (index, weight) pairs by index */
    for (int q = 0; q < n; q++) {
      int32_t c = st[q];
      double v = Wrows[e * n + q];
      int p = q;
      while (p > 0 && col[base + p - 1] > c) {
        col[base + p] = col[base + p - 1];
        val[base + p] = val[base + p - 1];
        p--;
      }
      col[base + p] = c;
      val[base + p] = v;
    }
    row_ptr[e + 1] = base + n;
  }
  return ORC_OK;
}
