/*
 * All-cores timing variant of the CPU oracle.  TEST INFRASTRUCTURE ONLY:
 * only the tests and the benchmark's CPU-baseline leg may load it.  It
 * shares no code with the GPU library.  The pinned oracle is the plain
 * single-threaded loop of hm_oracle.c; this file computes the same sum
 * (Sec. 2.1, Definitions "Block Tree" and "H-Matrix", Eq. (1), the form
 * W_b diag(s_b) X_b^T of Sec. 3.3) with the same floating-point operations
 * in the same order per output entry, so its result is bitwise that of the
 * plain loop whatever the number of threads:
 *
 *   1. every low-rank block's t_b = (V_b^T x) .* s_b, one block per thread
 *      at a time, each entry summed over ascending rows of V_b exactly as
 *      the plain loop does;
 *   2. the rows cut into ranges of `rows_per_task`; one thread owns a range
 *      and, for every block that touches it, in the caller's block order,
 *      adds alpha * (D_b x_sigma)_i or alpha * (U_b t_b)_i to y_i for its
 *      rows i, each inner sum ascending.  Every y_i thus receives the same
 *      additions in the same order as in the plain loop, from one thread.
 *
 * Built with gcc -O2 -fopenmp (no -ffast-math), like hm_oracle.c otherwise.
 */
#include <stdint.h>
#include <stdlib.h>

#include <omp.h>

/* Same arguments as oracle_hmvm plus the thread count (<= 0: OpenMP's
 * default) and the rows per task.  Returns the number of threads used, or a
 * negative error (-1 bad block, -5 out of memory). */
int oracle_hmvm_omp(int64_t n_rows, int64_t n_cols, int64_t nblocks,
                    const int64_t* rb, const int64_t* re, const int64_t* cb, const int64_t* ce,
                    const int32_t* kind, const int32_t* rank,
                    const double* const* a, const double* const* bf, const double* const* s,
                    double alpha, const double* x, double* y, int32_t nthreads, int64_t rows_per_task)
{
    if (rows_per_task < 1) rows_per_task = 64;
    for (int64_t b = 0; b < nblocks; ++b) {
        const int64_t m = re[b] - rb[b], n = ce[b] - cb[b];
        if (rb[b] < 0 || re[b] > n_rows || cb[b] < 0 || ce[b] > n_cols || m <= 0 || n <= 0) return -1;
    }
    /* offsets of t_b */
    int64_t* toff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nblocks + 1));
    if (!toff) return -5;
    toff[0] = 0;
    for (int64_t b = 0; b < nblocks; ++b) toff[b + 1] = toff[b] + (kind[b] == 1 ? rank[b] : 0);
    double* t = (double*)malloc(sizeof(double) * (size_t)(toff[nblocks] > 0 ? toff[nblocks] : 1));
    /* per row range, the blocks touching it in block order (CSR) */
    const int64_t ntask = (n_rows + rows_per_task - 1) / rows_per_task;
    int64_t* cnt = (int64_t*)calloc((size_t)ntask + 1, sizeof(int64_t));
    if (!t || !cnt) { free(toff); free(t); free(cnt); return -5; }
    for (int64_t b = 0; b < nblocks; ++b)
        for (int64_t q = rb[b] / rows_per_task; q <= (re[b] - 1) / rows_per_task; ++q) cnt[q + 1]++;
    for (int64_t q = 0; q < ntask; ++q) cnt[q + 1] += cnt[q];
    int64_t* list = (int64_t*)malloc(sizeof(int64_t) * (size_t)(cnt[ntask] > 0 ? cnt[ntask] : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ntask > 0 ? ntask : 1));
    if (!list || !fill) { free(toff); free(t); free(cnt); free(list); free(fill); return -5; }
    for (int64_t q = 0; q < ntask; ++q) fill[q] = cnt[q];
    for (int64_t b = 0; b < nblocks; ++b)
        for (int64_t q = rb[b] / rows_per_task; q <= (re[b] - 1) / rows_per_task; ++q) list[fill[q]++] = b;

    if (nthreads > 0) omp_set_num_threads(nthreads);
    int used = 1;
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
        /* 1. t_b for every low-rank block */
#pragma omp for schedule(dynamic, 8)
        for (int64_t b = 0; b < nblocks; ++b) {
            if (kind[b] != 1) continue;
            const int64_t c0 = cb[b], n = ce[b] - cb[b], k = rank[b];
            const double* V = bf[b];
            double* tb = t + toff[b];
            for (int64_t l = 0; l < k; ++l) {
                double acc = 0.0;
                for (int64_t j = 0; j < n; ++j) acc += V[l * n + j] * x[c0 + j];
                tb[l] = s && s[b] ? acc * s[b][l] : acc;
            }
        }
        /* 2. rows: one thread per range, blocks in the caller's order */
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < ntask; ++q) {
            const int64_t lo = q * rows_per_task;
            const int64_t hi = lo + rows_per_task < n_rows ? lo + rows_per_task : n_rows;
            for (int64_t e = cnt[q]; e < cnt[q + 1]; ++e) {
                const int64_t b = list[e];
                const int64_t r0 = rb[b], c0 = cb[b];
                const int64_t m = re[b] - r0, n = ce[b] - c0;
                const int64_t i0 = (lo > r0 ? lo : r0) - r0;
                const int64_t i1 = (hi < re[b] ? hi : re[b]) - r0;
                if (kind[b] == 0) {
                    const double* D = a[b];
                    for (int64_t i = i0; i < i1; ++i) {
                        double acc = 0.0;
                        for (int64_t j = 0; j < n; ++j) acc += D[j * m + i] * x[c0 + j];
                        y[r0 + i] += alpha * acc;
                    }
                } else {
                    const int64_t k = rank[b];
                    if (k == 0) continue;
                    const double* U = a[b];
                    const double* tb = t + toff[b];
                    for (int64_t i = i0; i < i1; ++i) {
                        double acc = 0.0;
                        for (int64_t l = 0; l < k; ++l) acc += U[l * m + i] * tb[l];
                        y[r0 + i] += alpha * acc;
                    }
                }
            }
        }
    }
    free(toff); free(t); free(cnt); free(list); free(fill);
    return used;
}
