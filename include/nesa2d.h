/*
 * nesa2d.h -- C ABI of the 2D model problem of the same library (MI355X).
 *
 * The paper's own benchmark (Sec. "The model problem", Eq. (pot)): N charges
 * q_j at points x_j on a curve in the plane; the potential at the same points
 * is phi = K q with k_ij = -log |x_i - x_j| (i != j) and k_ii = 0.  The
 * library builds, once, the NESA form of K over a quadtree and applies it on
 * the GPU in real FP64: the near-field block product (Eq. (algnf)) between
 * neighbouring finest-level groups, then radiation (Eq. (algrad)), source
 * transfer (Eq. (algsou)), translation (Eq. (algtrans)), potential transfer
 * (Eq. (algpot)) and reception (Eq. (algrec)).
 *
 * Tree (same section): the coarsest level l0 = 2 has 4 groups along the
 * longest side of the points' bounding square (side = longest extent x
 * (1 + 2^-20), anchored at the bounding-box minimum); L is the deepest level
 * (at most 20) whose mean number of points per non-empty group is still >= P.
 * Near groups
 * of a finest-level group: itself and its 8 neighbours; far groups at level
 * l: non-neighbours whose parents are neighbours (at l0: all non-neighbours).
 *
 * Matrices (the paper names only equivalent charges on circles matched on a
 * test circle; readings): Q equivalent points on a circle of radius 0.75 a_l
 * around each box (angles 2 pi (k + 1/2) / Q), 2Q check points on each of two
 * circles of radius 1.05 a_l and 1.6 a_l (angles 2 pi k / (2Q)), fitting operator
 * R_l = Tikhonov pseudo-inverse of G(X_l, E_l) with lambda = tau sigma_max;
 * V_b = R_L G(X_L + c_b, x_b), C = R_{l-1} G(X_{l-1}, E_l + delta_quadrant),
 * D = G(E_l + c_a, E_l + c_b), U_a = V_a^T, B = C^T.
 *
 * Conventions as in nesa.h: status codes, nesa_last_error(), device pointers
 * owned by the caller, `stream` a hipStream_t (NULL = default stream).
 */
#ifndef NESA2D_H
#define NESA2D_H

#include <stdint.h>

#include "nesa.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nesa2d nesa2d;

/* P: target mean number of points per finest-level group (>= 1).
 * Q: equivalent charges per group (2..128).
 * tau: Tikhonov parameter relative to the largest singular value (> 0). */
typedef struct {
  int P;
  int Q;
  double tau;
} nesa2d_params;

#define NESA2D_MAX_LEVELS 24

typedef struct {
  int64_t n;                               /* points */
  int l0, L;                               /* coarsest and finest level */
  int Q;
  int64_t n_box[NESA2D_MAX_LEVELS];        /* non-empty groups per level, index l - l0 */
  int64_t n_far[NESA2D_MAX_LEVELS];        /* translation pairs per level */
  int64_t near_pairs;                      /* (target point, source point) near pairs */
  int64_t max_leaf;                        /* most points in one finest-level group */
} nesa2d_info;

/* Builds the tree and the NESA matrices on the host (FP64) and uploads them to
 * the current device.  xy: host array [n][2] of distinct points (n >= 2).
 * Errors: NESA_EINVAL (null pointer, n < 2, bad P, Q, tau, or more than
 * NESA2D_MAX_LEVELS levels), NESA_ENOMEM, NESA_EHIP. */
nesa_status nesa2d_create(const double* xy, int64_t n, const nesa2d_params* params, nesa2d** out);

/* Sizes of the built operator. */
nesa_status nesa2d_info_get(const nesa2d* h, nesa2d_info* out);

/* perm[k] = index of the point at position k of the group order (groups in
 * (i, j) order of the finest level, points by index inside a group).  Host
 * array of n entries. */
nesa_status nesa2d_perm(const nesa2d* h, int32_t* perm);

/* phi_dev = K_NESA q_dev: device arrays of n doubles in the caller's point
 * order, distinct buffers.  Enqueued on `stream`, returns without waiting. */
nesa_status nesa2d_matvec(nesa2d* h, const double* q_dev, double* phi_dev, void* stream);

/* Releases the operator (synchronises the device first). */
nesa_status nesa2d_free(nesa2d* h);

#ifdef __cplusplus
}
#endif

#endif /* NESA2D_H */
