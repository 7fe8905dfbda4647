/*
 * orbf_oracle.h -- CPU oracle for the overlapped RBF-FD differentiation-matrix
 * (DM) build (Shankar, "The Overlapped RBF-FD Method: A Generalization of
 * RBF-FD").
 *
 * TEST INFRASTRUCTURE ONLY.  This header and orbf_oracle.c exist so that the
 * tests, the smoke check and the CPU-baseline leg of the benchmark can check
 * the HIP library against a plain, slow, single-precision-free (FP64) CPU
 * implementation written directly from the paper.  The product path never
 * includes, links or calls anything declared here, and nothing here includes
 * the product's headers.
 *
 * Conventions shared by every function:
 *   - nodes are AoS FP64, x[i*d + a], d in {2,3};
 *   - a stencil of node k is the n nearest nodes (k first), ordered by the key
 *     (squared distance, global index) ascending (Sec. 2 and Sec. 4.1: the
 *     stencil P_k is x_k and its n-1 nearest neighbours, I^k_1 = k);
 *   - squared distances are ((dx*dx)+(dy*dy))+(dz*dz) in FP64, evaluated left
 *     to right without contraction;
 *   - return value: ORC_OK or one of the ORC_E* codes below.
 */
#ifndef ORBF_ORACLE_H
#define ORBF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_EINVAL = 1,     /* bad sizes / parameters / NaN input            */
  ORC_EDUPLICATE = 2, /* two distinct nodes at squared distance zero   */
  ORC_ESINGULAR = 3   /* exact zero pivot in a local saddle system     */
};

/* Operators L (Sec. 4.1: the right-hand sides are L applied to the RBF and
 * polynomial basis at the evaluation points; the scaled solve is divided by
 * rho^theta, theta the order of L).  NEUMANN: n . grad with a given unit
 * normal per point (theta 1); DX, DY, DZ: d/dx_a (theta 1); IDENTITY: the
 * value itself (interpolation, theta 0). */
enum {
  ORC_OP_LAPLACIAN = 0,
  ORC_OP_NEUMANN = 1,
  ORC_OP_DX = 2,
  ORC_OP_DY = 3,
  ORC_OP_DZ = 4,
  ORC_OP_IDENTITY = 5
};

/* Number of monomials of total degree <= l in d variables, C(l+d, d). */
int orc_num_monomials(int d, int l);

/* Polynomial degree rule of Sec. 2: the largest s with C(s+d,d) <= n/2
 * (in 2D the closed form floor((sqrt(4n+1)-3)/2)).  Writes s and M. */
void orc_degree_rule(int d, int n, int* s_out, int* M_out);

/* kNN by brute force over all N nodes.  knn: N*n int32, rho2: N (squared
 * distance of the n-th neighbour).  ORC_EDUPLICATE if any two nodes coincide. */
int orc_knn_brute(const double* x, int64_t N, int d, int n, int32_t* knn,
                  double* rho2);

/* Same result as orc_knn_brute (bit for bit), found with a uniform bucket
 * grid and ring expansion; for node sets too large for brute force. */
int orc_knn_grid(const double* x, int64_t N, int d, int n, int32_t* knn,
                 double* rho2);

/* Brute-force kNN of a single query node q (for sampled checks at sizes
 * where the full brute force is too slow). */
int orc_knn_one(const double* x, int64_t N, int d, int n, int64_t q,
                int32_t* knn_q, double* rho2_q);

/* Greedy overlapped covering without Lebesgue rejection (Sec. 4.1): nodes
 * are visited in ascending index; an eligible node that no earlier stencil
 * has claimed becomes a center and claims every eligible, unclaimed node of
 * its stencil inside the closed retention ball of radius (1-delta)*rho_k.
 * eligible may be NULL (all nodes eligible).  owner[N] (-1 for ineligible
 * nodes), centers[] ascending (capacity N), *n_centers. */
int orc_cover(const double* x, int64_t N, int d, int n, const int32_t* knn,
              const double* rho2, double delta, const uint8_t* eligible,
              int32_t* owner, int32_t* centers, int64_t* n_centers);

/* Local weights of one stencil (eqs. rbffd_linsys, orbffd_eq, orbffd_rhs).
 *   P   : n*d stencil coordinates, P[0] is the center x_k;
 *   E   : ne*d evaluation points (normally stencil nodes);
 *   nrm : ne*d unit normals (ORC_OP_NEUMANN) or NULL;
 *   W   : ne*n output, W[e*n + j] = weight of stencil node j for point e,
 *         in physical units (the scaled solve is divided by rho^theta).
 * m odd >= 3, l >= -1 (l = -1: no polynomial part, M = 0, the unaugmented
 * system of Sec. 4.3), n >= C(l+d,d). */
int orc_stencil_weights(int d, int m, int l, int op, int n, const double* P,
                        int ne, const double* E, const double* nrm,
                        double* W);

/* Full DM rows for an interior operator (Laplacian) with the greedy covering
 * and, when tau is finite, the local L-Lebesgue rejection of Sec. 4.2.1
 * (node e of stencil k is kept iff e is the center or
 *  Lambda(x_e) <= tau * Lambda(x_ref), x_ref = stencil node nearest the
 *  centroid).  Rows of nodes whose owner is k are written to Wrows[e*n..]
 * aligned with knn[k*n..]; lam[e] receives Lambda of the row (may be NULL).
 * owner/centers/n_centers as in orc_cover.  min_margin (may be NULL)
 * receives the smallest |Lambda_e - tau*Lambda_ref| / (tau*Lambda_ref) seen
 * over all decisions (INFINITY if tau is infinite). */
int orc_overlapped_rows(const double* x, int64_t N, int d, int n, int m, int l,
                        const int32_t* knn, const double* rho2, double delta,
                        double tau, const uint8_t* eligible, int32_t* owner,
                        int32_t* centers, int64_t* n_centers, double* Wrows,
                        double* lam, double* min_margin, int nthreads);

/* orc_overlapped_rows with a choice of how the threshold shrinks a
 * stencil's retained set: prefix = 0 is node-wise (as above); prefix = 1 is
 * the radial prefix: with q* the first stencil position of an eligible node
 * of the retention ball (claimed by an earlier center or not) that fails
 * Lambda <= tau * Lambda_ref, the center keeps only its unclaimed eligible
 * ball nodes before q* (its ball shrunk to just inside the first failure). */
int orc_overlapped_rows_mode(const double* x, int64_t N, int d, int n, int m,
                             int l, const int32_t* knn, const double* rho2,
                             double delta, double tau, int prefix,
                             const uint8_t* eligible, int32_t* owner,
                             int32_t* centers, int64_t* n_centers,
                             double* Wrows, double* lam, double* min_margin,
                             int nthreads);

/* The same rows (infinite tau only) for another operator: LAPLACIAN, DX,
 * DY, DZ (d = 3) or IDENTITY. */
int orc_overlapped_rows_op(const double* x, int64_t N, int d, int n, int m,
                           int l, int op, const int32_t* knn,
                           const double* rho2, double delta,
                           const uint8_t* eligible, int32_t* owner,
                           int32_t* centers, int64_t* n_centers,
                           double* Wrows, double* lam, int nthreads);

/* Standard (delta = 1) rows for an explicit list of nodes with operator op
 * (boundary pass of Sec. 5: normal-derivative rows at boundary nodes, each
 * on its own stencil).  nrm: n_rows*d (ORC_OP_NEUMANN) or NULL.  Row of
 * node rows[i] is written to Wrows[rows[i]*n..]; owner[rows[i]] = rows[i]. */
int orc_center_rows(const double* x, int64_t N, int d, int n, int m, int l,
                    int op, const int32_t* knn, int64_t n_rows,
                    const int32_t* rows, const double* nrm, int32_t* owner,
                    double* Wrows, int nthreads);

/* CSR of the DM: row e has the n global indices of stencil owner[e] in
 * ascending order with the matching weights.  Rows with owner -1 are empty.
 * row_ptr: N+1 int64; col: capacity N*n int32; val: capacity N*n. */
int orc_csr(int64_t N, int n, const int32_t* knn, const int32_t* owner,
            const double* Wrows, int64_t* row_ptr, int32_t* col, double* val);

#ifdef __cplusplus
}
#endif
#endif
