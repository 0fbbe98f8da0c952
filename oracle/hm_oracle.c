/*
 * CPU oracle for the H-matrix-vector product.  TEST INFRASTRUCTURE ONLY:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code with the GPU library.
 *
 * Computes, in FP64 and in a fixed order, the definition
 *
 *     y := y + alpha * sum_{b=(tau,sigma) in L(T)}  E_tau M_b E_sigma^T x
 *
 * over the leaves of the block tree (Sec. 2.1, Definitions "Block Tree" and
 * "H-Matrix"), where M_b is the dense block D_b for an inadmissible leaf and
 * the low-rank product U_b V_b^T (Eq. (1)) for an admissible one, optionally
 * in the form W_b diag(s_b) X_b^T of Sec. 3.3.  The paper states the product
 * only as needing the decompressed blocks (Sec. 1, Sec. 5.4); the update
 * y += alpha*A*x follows the BLAS gemv convention.
 *
 * Loop order: blocks in the caller's order; dense blocks row by row with the
 * column sum ascending; low-rank blocks t = V^T x (ascending rows of V), then
 * t_l *= s_l, then y_i += alpha * sum_l U_il t_l (ascending l).
 *
 * Built with gcc -O2 (no -ffast-math, no OpenMP): plain and single-threaded.
 */
#include <stdint.h>
#include <stdlib.h>

/* Single right-hand side.  All arrays in cluster order; factors are FP64,
 * column-major: a[b] is D_b (m x n_b) for kind 0 and U_b (m x k) for kind 1,
 * bf[b] is V_b (n_b x k), s[b] is NULL or the k singular values. */
int oracle_hmvm(int64_t n_rows, int64_t n_cols, int64_t nblocks,
                const int64_t* rb, const int64_t* re, const int64_t* cb, const int64_t* ce,
                const int32_t* kind, const int32_t* rank,
                const double* const* a, const double* const* bf, const double* const* s,
                double alpha, const double* x, double* y)
{
    int64_t kmax = 0;
    for (int64_t b = 0; b < nblocks; ++b)
        if (kind[b] == 1 && rank[b] > kmax) kmax = rank[b];
    double* t = (double*)malloc(sizeof(double) * (size_t)(kmax > 0 ? kmax : 1));
    if (!t) return -5;
    for (int64_t b = 0; b < nblocks; ++b) {
        const int64_t r0 = rb[b], c0 = cb[b];
        const int64_t m = re[b] - r0, n = ce[b] - c0;
        if (r0 < 0 || re[b] > n_rows || c0 < 0 || ce[b] > n_cols || m <= 0 || n <= 0) {
            free(t);
            return -1;
        }
        if (kind[b] == 0) {
            const double* D = a[b];
            for (int64_t i = 0; i < m; ++i) {
                double acc = 0.0;
                for (int64_t j = 0; j < n; ++j) acc += D[j * m + i] * x[c0 + j];
                y[r0 + i] += alpha * acc;
            }
        } else {
            const int64_t k = rank[b];
            if (k == 0) continue;
            const double* U = a[b];
            const double* V = bf[b];
            for (int64_t l = 0; l < k; ++l) {
                double acc = 0.0;
                for (int64_t j = 0; j < n; ++j) acc += V[l * n + j] * x[c0 + j];
                t[l] = s && s[b] ? acc * s[b][l] : acc;
            }
            for (int64_t i = 0; i < m; ++i) {
                double acc = 0.0;
                for (int64_t l = 0; l < k; ++l) acc += U[l * m + i] * t[l];
                y[r0 + i] += alpha * acc;
            }
        }
    }
    free(t);
    return 0;
}

/* Several right-hand sides: the single-RHS definition applied column by
 * column.  X is n_cols x nrhs with leading dimension ldx, Y n_rows x nrhs
 * with leading dimension ldy, both column-major. */
int oracle_hmvm_multi(int64_t n_rows, int64_t n_cols, int64_t nblocks,
                      const int64_t* rb, const int64_t* re, const int64_t* cb, const int64_t* ce,
                      const int32_t* kind, const int32_t* rank,
                      const double* const* a, const double* const* bf, const double* const* s,
                      double alpha, int64_t nrhs, const double* X, int64_t ldx,
                      double* Y, int64_t ldy)
{
    for (int64_t c = 0; c < nrhs; ++c) {
        int rc = oracle_hmvm(n_rows, n_cols, nblocks, rb, re, cb, ce, kind, rank, a, bf, s,
                             alpha, X + c * ldx, Y + c * ldy);
        if (rc) return rc;
    }
    return 0;
}
