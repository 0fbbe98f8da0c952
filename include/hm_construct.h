/*
 * hm_construct.h -- GPU-side construction of H-matrix leaves (libhm.so).
 *
 * The leaves of the block tree (Sec. 2.1, Definition "Block Tree") are
 * filled on the GPU in FP64:
 *  - an inadmissible leaf tau x sigma holds the dense block
 *    D(i, j) = K(p_{rb+i}, p_{cb+j}) of the kernel function K;
 *  - an admissible leaf is approximated by partially pivoted adaptive cross
 *    approximation (ACA, named in Sec. 5.1 as the method that builds the
 *    low-rank blocks) at accuracy eps_aca, then truncated to accuracy eps by
 *    Algorithm 1 of Sec. 2.2 (QR of both factors, SVD of R_U R_V^T, the
 *    smallest rank k whose Frobenius tail of singular values is at most eps
 *    times the whole), giving W (m x k), X (n x k) with orthonormal columns
 *    and singular values s (k), M_b = W diag(s) X^T (Eq. (1)).
 * The paper does not state the ACA variant; the one here takes the leaf's
 * first row as the first pivot row, the largest entry of the residual row as
 * the column pivot, the largest entry of the newest column over the rows not
 * used yet as the next row (a zero residual row moves on to the lowest
 * unused row), and stops when |u_k| |v_k| <= eps_aca |S_k|_F or after
 * min(m, n) steps.
 *
 * Kernel functions (the point-kernel stand-ins of the model problems of
 * Sec. 5.1):
 *   HM_KERNEL_LAPLACE  K(x, y) = 1 / (4 pi |x - y|), K(x, x) = 1 / (4 pi h),
 *                      params[0] = h > 0;
 *   HM_KERNEL_EXP      K(x, y) = exp(-|x - y| / l), plus d on the diagonal,
 *                      params[0] = l > 0, params[1] = d.
 *
 * Conventions as in hm.h: plain pointers, caller-owned device memory, a
 * negative hm_status on error with nothing enqueued, stream-ordered work.
 */
#ifndef HM_CONSTRUCT_H
#define HM_CONSTRUCT_H

#include "hm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define HM_KERNEL_LAPLACE 0
#define HM_KERNEL_EXP 1
/* Largest number of ACA columns a leaf can reserve (cap). */
#define HM_CONSTRUCT_MAX_RANK 128

/* One leaf to construct.  Points are in cluster order; the leaf's rows are
 * points rb .. rb + m - 1, its columns points cb .. cb + n - 1.
 * adm: 1 admissible (low rank), 0 dense.  cap: ACA columns reserved
 * (admissible: 1 .. min(m, n, HM_CONSTRUCT_MAX_RANK); 0 in a call to
 * hm_construct_layout picks that maximum; dense: ignored).
 * out, scr: offsets, in doubles, of the leaf's output and scratch regions
 * (set by hm_construct_layout).  Output region: dense, D (m x n,
 * column-major); admissible, W (m x cap), then X (n x cap), then s (cap),
 * of which the first k columns / entries are the result.  Scratch region
 * (admissible only): the ACA factors and the used-row flags. */
typedef struct {
  int64_t rb, cb;
  int32_t m, n;
  int32_t adm, cap;
  int64_t out, scr;
} hm_cblock;

/* kernel: HM_KERNEL_LAPLACE or HM_KERNEL_EXP; params as above.
 * keep_sigma: 1 keeps s separately (W, X orthonormal); 0 folds it into the
 * first factor (U = W diag(s), V = X; s is still written).
 * eps_aca > 0: ACA stopping accuracy; eps > 0: truncation accuracy. */
typedef struct {
  int32_t kernel, keep_sigma;
  double params[2];
  double eps_aca, eps;
} hm_construct_opts;

/* Sets cap (where 0), out and scr of n_blocks leaves so that their regions
 * follow each other (16-byte aligned), and returns the doubles of output and
 * scratch they need.  Host only.  Errors: HM_EINVAL (NULL, bad m, n, adm or
 * cap). */
hm_status hm_construct_layout(hm_cblock* blocks, int64_t n_blocks, int64_t* out_doubles,
                              int64_t* scr_doubles);

/* Largest ACA rank whose truncation runs on the current device (its SVD
 * keeps two r x r FP64 matrices in the LDS of one workgroup).  Leaves whose
 * ACA rank exceeds it are returned with rank -2. */
hm_status hm_construct_rank_limit(int32_t* rmax);

/* Constructs n_blocks leaves on the current device.
 * d_points: n_points x 3 FP64 (x, y, z of each point, cluster order), device.
 * h_blocks: the leaves (host), laid out as by hm_construct_layout; the call
 *   copies them into d_desc (device, >= n_blocks * sizeof(hm_cblock) bytes),
 *   which must stay untouched until the work has run.
 * d_out (out_bytes), d_scr (scr_bytes): device memory for the regions.
 * d_rank: 2 * n_blocks int32, device: entries [0, n_blocks) receive the ACA
 *   ranks, entries [n_blocks, 2 n_blocks) the final ranks k: 0 for a dense
 *   leaf, k >= 0 for an admissible one, -1 where the ACA did not converge
 *   within cap columns, -2 where the ACA rank exceeds hm_construct_rank_limit
 *   (the caller constructs such leaves otherwise).
 * Validated synchronously (HM_EINVAL: arguments, a leaf outside the points,
 * a region outside its buffer; HM_ENOMEM: d_desc too small); the kernels are
 * enqueued on `stream` and the call returns after the descriptor copy has
 * been enqueued.  Read d_out and d_rank after synchronizing the stream. */
hm_status hm_construct(const double* d_points, int64_t n_points, const hm_cblock* h_blocks, int64_t n_blocks,
                       void* d_desc, size_t desc_bytes, const hm_construct_opts* opts, double* d_out,
                       size_t out_bytes, double* d_scr, size_t scr_bytes, int32_t* d_rank, void* stream);

/* Copies the results of hm_construct (after it has run: same stream, or
 * synchronized) into a dense packing, so that only the leaves' data need to
 * leave the device.  d_desc, n_blocks, d_rank, d_out: as passed to
 * hm_construct.  d_off: n_blocks int64 (device), the offset in doubles of
 * each leaf's data in d_packed; the data are, for a dense leaf, D (m x n);
 * for an admissible leaf of final rank k >= 0, W (m x k), then X (n x k),
 * then s (k); nothing when k < 0.  A leaf
 * whose data would end beyond packed_bytes is skipped (no write).
 * Errors: HM_EINVAL (NULL or negative size). */
hm_status hm_construct_pack(const void* d_desc, int64_t n_blocks, const int32_t* d_rank, const double* d_out,
                            const int64_t* d_off, double* d_packed, size_t packed_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HM_CONSTRUCT_H */
