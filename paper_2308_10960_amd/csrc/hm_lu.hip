// HIP kernels (gfx950) of the H-LU factorisation with accumulated updates
// (hm_lu_host.cpp drives them; include/hm_lu.h is the C-ABI):
//
//  k_gemm     C := beta C + alpha op(A) op(B) in FP64, any dimension given
//             on the host or read from a rank on the device (the ranks of
//             low-rank blocks stay on the device during the factorisation);
//             64 x 64 tiles, 256 threads of 4 x 4 results, K in steps of 16
//             through LDS;
//  k_getrf    dense LU without pivoting of a diagonal leaf, in LDS;
//  k_trsm     a triangular solve with a dense diagonal leaf on a dense
//             panel: L^-1 Z (L unit lower), U^-T Z or U^-1 Z; the triangle
//             and 32 columns per workgroup in LDS;
//  k_trunc    Algorithm 1 (Sec. 2.2) on the sum of two low-rank terms placed
//             at row offsets of the target (zero elsewhere), one workgroup:
//             the factors are gathered into a scratch pair, reduced to
//             min(m, n) columns when wider, and truncated by the shared core
//             (QR of both, Jacobi SVD of R_U R_V^T in LDS, Frobenius tail
//             <= eps of the whole);
//  k_round    rounding of a matrix to a DFL format in place (Sec. 3.2: the
//             FP64 encoding cut to whole bytes, round to nearest even),
//             which is what a compressed block decompresses to;
//  k_eye, k_fill, k_axpy, k_transpose  small helpers.
#include <algorithm>
#include <cmath>

#include <hip/hip_runtime.h>

#include "hm_dense.hpp"
#include "hm_lu_internal.hpp"

namespace hm {
namespace lu {
namespace {

constexpr int kT = 256;
constexpr int kTT = dense::kWThreads;   // threads of the truncation kernel (the dense core's workgroup)

__device__ __forceinline__ int64_t dval(const Dim& d) {
  return d.p ? (int64_t)max(0, min(*d.p, (int32_t)d.cap)) : d.v;
}

// C (M x N, ldc) := beta C + alpha op(A) op(B); op(A) is M x K (A stored
// M x K, or K x M when ta), op(B) is K x N (B stored K x N, or N x K when
// tb).  beta == 0 writes C without reading it.
__global__ __launch_bounds__(kT) void k_gemm(Dim Md, Dim Nd, Dim Kd, double alpha, const double* __restrict__ A,
                                             int64_t lda, int ta, const double* __restrict__ B, int64_t ldb, int tb,
                                             double beta, double* __restrict__ C, int64_t ldc) {
  __shared__ double As[16][64 + 1];
  __shared__ double Bs[16][64 + 1];
  const int64_t M = dval(Md), N = dval(Nd), K = dval(Kd);
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  if (i0 >= M || j0 >= N) return;                   // uniform: the whole workgroup
  const int tid = threadIdx.x, ti = tid & 15, tj = tid >> 4;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += kT) {
      const int kk = e / 64, ii = e % 64;
      const int64_t gi = i0 + ii, gk = k0 + kk;
      double a = 0, b = 0;
      if (gi < M && gk < K) a = ta ? A[gi * lda + gk] : A[gk * lda + gi];
      const int64_t gj = j0 + ii;
      if (gj < N && gk < K) b = tb ? B[gk * ldb + gj] : B[gj * ldb + gk];
      As[kk][ii] = a;
      Bs[kk][ii] = b;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[kk][ti + 16 * u];
        b[u] = Bs[kk][tj + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gi = i0 + ti + 16 * u, gj = j0 + tj + 16 * v;
      if (gi < M && gj < N) {
        double* c = C + gj * ldc + gi;
        *c = beta == 0.0 ? alpha * acc[u][v] : beta * *c + alpha * acc[u][v];
      }
    }
}

// Dense LU without pivoting of D (m x m, ld), m <= kLeafMax, in place.
__global__ __launch_bounds__(kT) void k_getrf(double* __restrict__ D, int64_t ld, int m) {
  __shared__ double S[kLeafMax * kLeafMax];
  const int tid = threadIdx.x;
  for (int e = tid; e < m * m; e += kT) S[e] = D[(int64_t)(e / m) * ld + e % m];
  __syncthreads();
  for (int k = 0; k + 1 < m; ++k) {
    const double piv = S[k * m + k];
    for (int i = k + 1 + tid; i < m; i += kT) S[k * m + i] /= piv;
    __syncthreads();
    const int w = m - k - 1;
    for (int e = tid; e < w * w; e += kT) {
      const int i = k + 1 + e % w, j = k + 1 + e / w;
      S[j * m + i] -= S[k * m + i] * S[j * m + k];
    }
    __syncthreads();
  }
  for (int e = tid; e < m * m; e += kT) D[(int64_t)(e / m) * ld + e % m] = S[e];
}

// Triangular solve with the dense diagonal leaf D (m x m, ld) on Z
// (m x ncols, ldz) in place; mode 0: L^-1 Z with L the unit lower part of D;
// 1: U^-T Z with U the upper part; 2: U^-1 Z.  One workgroup per kTrsmCols
// columns: the triangle and the workgroup's columns sit in LDS, and each
// elimination step updates the remaining rows of all columns in parallel.
constexpr int kTrsmCols = 32;
__global__ __launch_bounds__(kT) void k_trsm(const double* __restrict__ D, int64_t ld, int m, int mode, double* Z,
                                             int64_t ldz, Dim ncd) {
  __shared__ double S[kLeafMax * kLeafMax];
  __shared__ double Zs[kLeafMax * kTrsmCols];
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * kTrsmCols;
  const int64_t nc = dval(ncd);
  if (c0 >= nc) return;                              // uniform: the whole workgroup
  const int w = (int)std::min<int64_t>(kTrsmCols, nc - c0);
  for (int e = tid; e < m * m; e += kT) S[e] = D[(int64_t)(e / m) * ld + e % m];
  for (int e = tid; e < m * w; e += kT) Zs[(e / m) * kLeafMax + e % m] = Z[(c0 + e / m) * ldz + e % m];
  __syncthreads();
  if (mode == 0) {
    for (int k = 0; k + 1 < m; ++k) {
      const int rows = m - k - 1;
      for (int e = tid; e < rows * w; e += kT) {
        const int i = k + 1 + e % rows, c = e / rows;
        Zs[c * kLeafMax + i] -= S[k * m + i] * Zs[c * kLeafMax + k];
      }
      __syncthreads();
    }
  } else if (mode == 1) {
    for (int k = 0; k < m; ++k) {
      if (tid < w) Zs[tid * kLeafMax + k] /= S[k * m + k];
      __syncthreads();
      const int rows = m - k - 1;
      for (int e = tid; e < rows * w; e += kT) {
        const int i = k + 1 + e % rows, c = e / rows;
        Zs[c * kLeafMax + i] -= S[i * m + k] * Zs[c * kLeafMax + k];      // U(k, i)
      }
      __syncthreads();
    }
  } else {
    for (int k = m - 1; k >= 0; --k) {
      if (tid < w) Zs[tid * kLeafMax + k] /= S[k * m + k];
      __syncthreads();
      for (int e = tid; e < k * w; e += kT) {
        const int i = e % k, c = e / k;
        Zs[c * kLeafMax + i] -= S[k * m + i] * Zs[c * kLeafMax + k];      // U(i, k)
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < m * w; e += kT) Z[(c0 + e / m) * ldz + e % m] = Zs[(e / m) * kLeafMax + e % m];
}

__device__ __forceinline__ double part_u(const Part& p, int64_t i, int64_t c) {
  const int64_t r = i - p.uoff;
  if (r < 0 || r >= p.urows) return 0.0;
  if (!p.U) return r == c ? 1.0 : 0.0;
  return p.U[c * p.ldu + r];
}

__device__ __forceinline__ double part_v(const Part& p, int64_t j, int64_t c) {
  const int64_t r = j - p.voff;
  if (r < 0 || r >= p.vrows) return 0.0;
  if (!p.V) return r == c ? 1.0 : 0.0;
  return p.vtrans ? p.V[r * p.ldv + c] : p.V[c * p.ldv + r];
}

// W X^T ~ s0 U0 V0^T + s1 U1 V1^T (parts at row offsets of the m x n
// target), Algorithm 1 at eps.  scr: (m + n) (k0cap + k1cap) doubles, then
// m n when k0cap + k1cap > min(m, n), then 2 r^2 for a sum of r columns
// whose SVD matrices exceed the LDS (see trunc_scratch).  W (m x capo, ld
// m), X (n x capo, ld n), rank_out = k.  A sum wider than kMaxTrunc after
// the reduction to min(m, n) columns sets *err = 1 and rank 0 (the host
// reports HM_ERANK).  Dynamic LDS: kTruncLds doubles.
__global__ __launch_bounds__(kTT) void k_trunc(Part p0, Part p1, int64_t m, int64_t n, double eps, double* scr,
                                              double* __restrict__ W, double* __restrict__ X,
                                              int32_t* __restrict__ rank_out, int32_t* __restrict__ err,
                                              double* __restrict__ flog) {
  extern __shared__ double dyn[];
  __shared__ dense::TruncShared sh;
  const int tid = threadIdx.x;
  const int64_t k0 = dval(p0.k), k1 = dval(p1.k);
  int64_t r = k0 + k1;
  double* U = scr;
  double* V = U + m * r;
  for (int64_t e = tid; e < m * r; e += kTT) {
    const int64_t i = e % m, c = e / m;
    U[e] = c < k0 ? p0.sign * part_u(p0, i, c) : p1.sign * part_u(p1, i, c - k0);
  }
  for (int64_t e = tid; e < n * r; e += kTT) {
    const int64_t j = e % n, c = e / n;
    V[e] = c < k0 ? part_v(p0, j, c) : part_v(p1, j, c - k0);
  }
  __syncthreads();
  if (r > m || r > n) {
    // the same matrix with min(m, n) columns: (I_m, V U^T) or (U V^T, I_n)
    double* P = V + n * r;
    if (m <= n) {
      for (int64_t e = tid; e < n * m; e += kTT) {
        const int64_t j = e % n, i = e / n;
        double s = 0;
        for (int64_t c = 0; c < r; ++c) s += V[c * n + j] * U[c * m + i];
        P[e] = s;
      }
      __syncthreads();
      for (int64_t e = tid; e < m * m; e += kTT) U[e] = (e % m) == (e / m) ? 1.0 : 0.0;
      for (int64_t e = tid; e < n * m; e += kTT) V[e] = P[e];
      r = m;
    } else {
      for (int64_t e = tid; e < m * n; e += kTT) {
        const int64_t i = e % m, j = e / m;
        double s = 0;
        for (int64_t c = 0; c < r; ++c) s += U[c * m + i] * V[c * n + j];
        P[e] = s;
      }
      __syncthreads();
      for (int64_t e = tid; e < m * n; e += kTT) U[e] = P[e];
      for (int64_t e = tid; e < n * n; e += kTT) V[e] = (e % n) == (e / n) ? 1.0 : 0.0;
      r = n;
    }
    __syncthreads();
  }
  if (r > kMaxTrunc) {
    if (tid == 0) { *err = 1; *rank_out = 0; if (flog) *flog = 0; }
    return;
  }
  double* gscr = V + n * (k0 + k1) + ((k0 + k1) > std::min(m, n) ? m * n : 0);   // after U, V and P
  if (r == 0) {
    if (tid == 0) { *rank_out = 0; if (flog) *flog = 0; }
    return;
  }
  const int k = dense::truncate_core(U, m, V, n, (int)r, eps, dyn, kTruncLds, gscr, sh, W, X, true, nullptr);
  if (tid == 0) {
    *rank_out = k;
    // the QR of both factors and the application of Q (the SVD sweeps not counted)
    if (flog) *flog = 2.0 * (m + n) * r * r + 4.0 * (m + n) * r * k;
  }
}

// Rounds the m x n matrix A (ld) to nearest even with `mbits` explicit
// mantissa bits kept (FP64's sign and exponent), in place.
__global__ __launch_bounds__(kT) void k_round(double* A, int64_t ld, int64_t m, Dim nd, int mbits) {
  const int64_t n = dval(nd);
  const int drop = 52 - mbits;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < m * n; e += (int64_t)gridDim.x * kT) {
    double* p = A + (e / m) * ld + e % m;
    uint64_t b = __double_as_longlong(*p);
    if (((b >> 52) & 0x7ff) == 0x7ff) continue;      // inf, NaN
    const uint64_t half = (uint64_t(1) << (drop - 1)) - 1 + ((b >> drop) & 1);
    b = (b + half) & ~((uint64_t(1) << drop) - 1);   // a carry into the exponent is the rounding up
    *p = __longlong_as_double(b);
  }
}

__global__ __launch_bounds__(kT) void k_fill(double* A, int64_t ld, int64_t m, int64_t n, double v) {
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < m * n; e += (int64_t)gridDim.x * kT)
    A[(e / m) * ld + e % m] = v;
}

// A (m x m, ld) := I.
__global__ __launch_bounds__(kT) void k_eye(double* A, int64_t ld, int64_t m) {
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < m * m; e += (int64_t)gridDim.x * kT)
    A[(e / m) * ld + e % m] = (e % m) == (e / m) ? 1.0 : 0.0;
}

// C (m x n, ldc) += alpha A (m x n, lda).
__global__ __launch_bounds__(kT) void k_axpy(int64_t m, int64_t n, double alpha, const double* __restrict__ A,
                                             int64_t lda, double* __restrict__ C, int64_t ldc) {
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < m * n; e += (int64_t)gridDim.x * kT)
    C[(e / m) * ldc + e % m] += alpha * A[(e / m) * lda + e % m];
}

// B (n x m, ldb) := A^T for A (m x n, lda).
__global__ __launch_bounds__(kT) void k_transpose(const double* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                  double* __restrict__ B, int64_t ldb) {
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < m * n; e += (int64_t)gridDim.x * kT) {
    const int64_t i = e % m, j = e / m;
    B[i * ldb + j] = A[j * lda + i];
  }
}

unsigned grid_for(int64_t count) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + kT - 1) / kT, 4096));
}

}  // namespace

hipError_t gemm(Dim M, Dim N, Dim K, int64_t mcap, int64_t ncap, double alpha, const double* A, int64_t lda, int ta,
                const double* B, int64_t ldb, int tb, double beta, double* C, int64_t ldc, hipStream_t s) {
  if (mcap <= 0 || ncap <= 0) return hipSuccess;
  const dim3 grid((unsigned)((mcap + 63) / 64), (unsigned)((ncap + 63) / 64));
  hipLaunchKernelGGL(k_gemm, grid, dim3(kT), 0, s, M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc);
  return hipGetLastError();
}

hipError_t getrf(double* D, int64_t ld, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_getrf, dim3(1), dim3(kT), 0, s, D, ld, m);
  return hipGetLastError();
}

hipError_t trsm(const double* D, int64_t ld, int m, int mode, double* Z, int64_t ldz, Dim nc, int64_t nccap,
                hipStream_t s) {
  if (nccap <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsm, dim3((unsigned)((nccap + kTrsmCols - 1) / kTrsmCols)), dim3(kT), 0, s, D, ld, m, mode,
                     Z, ldz, nc);
  return hipGetLastError();
}

hipError_t trunc(const Part& p0, const Part& p1, int64_t m, int64_t n, double eps, double* scr, double* W,
                 double* X, int32_t* rank_out, int32_t* err, double* flog, hipStream_t s) {
  const size_t lds = (size_t)8 * kTruncLds;
  hipLaunchKernelGGL(k_trunc, dim3(1), dim3(kTT), lds, s, p0, p1, m, n, eps, scr, W, X, rank_out, err, flog);
  return hipGetLastError();
}

// Lets k_trunc take the dynamic LDS of a kMaxTrunc-wide sum (on the
// current device).
hipError_t prepare_trunc() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_trunc), hipFuncAttributeMaxDynamicSharedMemorySize,
                             8 * kTruncLds);
}

hipError_t round_dfl(double* A, int64_t ld, int64_t m, Dim n, int64_t ncap, int mbits, hipStream_t s) {
  if (m * ncap <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_round, dim3(grid_for(m * ncap)), dim3(kT), 0, s, A, ld, m, n, mbits);
  return hipGetLastError();
}

hipError_t fill(double* A, int64_t ld, int64_t m, int64_t n, double v, hipStream_t s) {
  if (m * n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(m * n)), dim3(kT), 0, s, A, ld, m, n, v);
  return hipGetLastError();
}

hipError_t eye(double* A, int64_t ld, int64_t m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_eye, dim3(grid_for(m * m)), dim3(kT), 0, s, A, ld, m);
  return hipGetLastError();
}

hipError_t axpy(int64_t m, int64_t n, double alpha, const double* A, int64_t lda, double* C, int64_t ldc,
                hipStream_t s) {
  if (m * n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(m * n)), dim3(kT), 0, s, m, n, alpha, A, lda, C, ldc);
  return hipGetLastError();
}

hipError_t transpose(const double* A, int64_t lda, int64_t m, int64_t n, double* B, int64_t ldb, hipStream_t s) {
  if (m * n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose, dim3(grid_for(m * n)), dim3(kT), 0, s, A, lda, m, n, B, ldb);
  return hipGetLastError();
}

int trunc_lds_limit() {
  int dev = 0, lds = 0, optin = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess)
    lds = std::max(lds, optin);
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k_trunc)) != hipSuccess) return 0;
  return (int64_t)lds - (int64_t)fa.sharedSizeBytes >= 8 * (int64_t)kTruncLds ? kMaxTrunc : 0;
}

}  // namespace lu
}  // namespace hm
