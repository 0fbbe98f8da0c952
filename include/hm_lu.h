/*
 * hm_lu.h -- H-LU factorisation with accumulated updates on the GPU
 * (libhm.so).
 *
 * The operation (Sec. 4.1): A = L U without pivoting, for an H-matrix A
 * over a binary cluster tree (Sec. 2.1, Definitions "Cluster Tree", "Block
 * Tree"); L is unit lower triangular and U upper triangular, both with A's
 * block structure: a diagonal leaf holds the strict lower part of L and the
 * upper part of U, as a dense LU does; a leaf below the diagonal (in the
 * cluster order) belongs to L, one above it to U.  The recursion is the
 * block LU of the 2 x 2 structure (LU of A00, triangular solves for A01 and
 * A10, update of A11 by A10 A01, LU of A11), the triangular solves recursing
 * the same way; Sec. 2.2 states that solves and LU follow the pattern of
 * the multiplication of Algorithm 2.
 *
 * Updates reach a block through an accumulator and a set of pending
 * products (Algorithm 3, Sec. 2.2): a product with a leaf factor is
 * evaluated into the accumulator of the block it updates when the recursion
 * enters that block; the others are split over the block's sons with the
 * restriction of the accumulator; a leaf applies its accumulator once,
 * before its own step (dense LU of a diagonal leaf, a triangular solve of an
 * off-diagonal one).  Low-rank sums are truncated by Algorithm 1 (Sec. 2.2)
 * at eps: the smallest rank whose Frobenius tail of singular values is at
 * most eps times the whole.  With a storage format, each leaf of L and U is
 * compressed once final and every later read sees its decompressed values
 * (Algorithm 4's semi-on-the-fly conversion); accumulators stay FP64
 * (Sec. 4.1).
 *
 * Readings where the paper is silent: an addition to a low-rank
 * accumulator is a truncated low-rank addition, one truncation per
 * product; a pending product with no leaf factor that reaches a leaf is
 * evaluated by its sons' products, each placed at its offsets and added
 * with truncation; a dense product added to a low-rank accumulator enters
 * as a low-rank term of rank min(rows, columns).
 *
 * Conventions as in hm.h: plain pointers, a negative hm_status on error
 * (text via hm_last_error), stream-ordered work on the current device.
 * Vectors and index ranges are in cluster order.
 */
#ifndef HM_LU_H
#define HM_LU_H

#include "hm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* A truncation needed a sum wider than HM_LU_MAX_RANK columns (after the
 * sum is reduced to min(rows, columns) columns). */
#define HM_ERANK (-10)
/* Widest low-rank sum the truncation takes (its SVD works in the LDS of
 * one workgroup up to 92 columns, in device memory beyond). */
#define HM_LU_MAX_RANK 256
/* Largest diagonal leaf (rows) the dense kernels take. */
#define HM_LU_MAX_LEAF 64

typedef struct hm_lu hm_lu;

/* The binary cluster tree: n_clusters clusters, cluster 0 the root over
 * [0, n); cluster c spans [begin[c], end[c]) and has sons son0[c], son1[c]
 * (both -1 at a leaf) that split its range in order. */
typedef struct {
  int64_t n_clusters;
  const int64_t* begin;
  const int64_t* end;
  const int32_t* son0;
  const int32_t* son1;
} hm_lu_tree;

typedef struct {
  int64_t kernels;        /* kernels launched by hm_lu_factor */
  int64_t truncations;    /* Algorithm 1 calls */
  int32_t max_rank;       /* largest rank of a leaf of L or U */
  int32_t reserved;
  double factor_doubles;  /* values held by the leaves of L and U */
  double stored_bytes;    /* bytes of those values in the storage format */
  size_t arena_peak;      /* device-memory high-water mark of the arena */
  /* with hm_lu_profile on: the summed duration of the timed truncation
   * kernels (HIP events around each), their arithmetic (flops of the QR of
   * both factors, 2 (m + n) r^2, and of the application of Q to the k kept
   * columns, 4 (m + n) r k; the SVD sweeps are not counted), and how many
   * were timed (the first 2^21) */
  double trunc_ms;
  double trunc_flops;
  int64_t timed_truncations;
} hm_lu_stats;

/* Creates the factorisation object on the current device and uploads A.
 * n_leaves leaves (tau[i], sigma[i]) that tile [0, n)^2 as the block tree
 * of `tree` (a leaf wherever the recursion from (0, 0) stops); kind[i]:
 * HM_DENSE (h_a[i]: D, m x n column-major; h_b[i] unused) or HM_LOWRANK
 * (h_a[i]: U, m x rank[i]; h_b[i]: V, n x rank[i]; both column-major, the
 * block U V^T).  Diagonal leaves must be dense with at most HM_LU_MAX_LEAF
 * rows.  arena_bytes of device memory are allocated for the factors and
 * every temporary; HM_ENOMEM when that does not suffice (at create or
 * factor time).  Host arrays are read during the call only.
 * Errors: HM_EINVAL (NULL, sizes), HM_EPARTITION (leaves do not match the
 * tree), HM_ESHAPE (a diagonal leaf not dense or too large, bad rank),
 * HM_ENOMEM, HM_EDEVICE. */
hm_status hm_lu_create(const hm_lu_tree* tree, int64_t n_leaves, const int32_t* tau, const int32_t* sigma,
                       const int32_t* kind, const int32_t* rank, const double* const* h_a,
                       const double* const* h_b, size_t arena_bytes, hm_lu** out);

/* Factorises in place: afterwards the leaves hold L and U.  eps > 0: the
 * truncation accuracy; dtype: HM_F64 (no compression) or one of HM_DFL16 ..
 * HM_DFL48 (each final leaf rounded to that format, Sec. 3.2).  Enqueues on
 * `stream` and synchronizes it before returning (the ranks and the error
 * flag are read back).  Once only per object (HM_ESTATE after).
 * Errors: HM_EINVAL, HM_EDTYPE, HM_ENOMEM (arena exhausted; the object is
 * then unusable), HM_ERANK, HM_ESTATE, HM_EDEVICE. */
hm_status hm_lu_factor(hm_lu* F, double eps, int32_t dtype, void* stream);

/* x := (L U)^-1 x for nrhs columns of d_x (device, n x nrhs, leading
 * dimension ld >= n), by the two H-triangular solves; stream-ordered.
 * Needs a factorised object (HM_ESTATE otherwise). */
hm_status hm_lu_solve(hm_lu* F, double* d_x, int64_t ld, int64_t nrhs, void* stream);

/* Copies leaf i of the factors to the host (synchronous): dense, D (m x n)
 * into h_a; low-rank, *rank = k and U (m x k), V (n x k) into h_a, h_b;
 * a_doubles / b_doubles: the room at h_a / h_b (HM_ENOMEM when short; *rank
 * is set first, so a call with 0 room asks for it). */
hm_status hm_lu_leaf(hm_lu* F, int64_t i, int32_t* rank, double* h_a, size_t a_doubles, double* h_b,
                     size_t b_doubles);

hm_status hm_lu_stats_get(const hm_lu* F, hm_lu_stats* st);

/* on != 0: the next hm_lu_factor records HIP events around every
 * truncation kernel and the kernel's arithmetic, for the statistics above
 * (adds two event records per truncation). */
hm_status hm_lu_profile(hm_lu* F, int32_t on);

void hm_lu_destroy(hm_lu* F);

#ifdef __cplusplus
}
#endif

#endif /* HM_LU_H */
