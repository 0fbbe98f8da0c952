// Launchers of the H-LU kernels (hm_lu.hip) for the host driver
// (hm_lu_host.cpp); not part of the C-ABI.
#pragma once
#include <cstdint>

#include <hip/hip_runtime_api.h>

namespace hm {
namespace lu {

constexpr int kLeafMax = 64;     // largest diagonal leaf (rows) of the dense kernels
constexpr int kMaxTrunc = 256;   // widest sum Algorithm 1 truncates
constexpr int kTruncLds = 17152; // doubles of dynamic LDS of the truncation kernel

// Scratch doubles of one truncation of a sum of at most capsum columns over
// an m x n target: the gathered factors, the product when the sum is wider
// than min(m, n), and the two r x r SVD matrices when they exceed the LDS.
inline int64_t trunc_scratch(int64_t m, int64_t n, int64_t capsum) {
  const int64_t mn = m < n ? m : n;
  int64_t r = capsum < mn ? capsum : mn;
  if (r > kMaxTrunc) r = kMaxTrunc;
  return (m + n) * capsum + (capsum > mn ? m * n : 0) + (2 * r * r > kTruncLds ? 2 * r * r : 0);
}

// A dimension: the host value v, or the int32 at device address p (a rank
// that only the device knows during the factorisation), clamped to
// [0, cap], the capacity of the buffers sized for it.
struct Dim {
  int64_t v = 0;
  const int32_t* p = nullptr;
  int64_t cap = 0;
};

// A low-rank term s U V^T placed at rows [uoff, uoff + urows) and columns
// [voff, voff + vrows) of a target (zero elsewhere), with k columns.  U is
// urows x k (leading dimension ldu); a null U is the identity (k = urows).
// V is vrows x k (ldv), or k x vrows when vtrans; a null V is the identity.
struct Part {
  const double* U = nullptr;
  int64_t ldu = 0, uoff = 0, urows = 0;
  const double* V = nullptr;
  int64_t ldv = 0, voff = 0, vrows = 0;
  Dim k;
  double sign = 1.0;
  int32_t vtrans = 0;
};

hipError_t gemm(Dim M, Dim N, Dim K, int64_t mcap, int64_t ncap, double alpha, const double* A, int64_t lda, int ta,
                const double* B, int64_t ldb, int tb, double beta, double* C, int64_t ldc, hipStream_t s);
hipError_t getrf(double* D, int64_t ld, int m, hipStream_t s);
hipError_t trsm(const double* D, int64_t ld, int m, int mode, double* Z, int64_t ldz, Dim nc, int64_t nccap,
                hipStream_t s);
hipError_t prepare_trunc();
// flog: where the kernel writes its arithmetic (flops of the QR of both
// factors and of the application of Q), or null.
hipError_t trunc(const Part& p0, const Part& p1, int64_t m, int64_t n, double eps, double* scr, double* W,
                 double* X, int32_t* rank_out, int32_t* err, double* flog, hipStream_t s);
hipError_t round_dfl(double* A, int64_t ld, int64_t m, Dim n, int64_t ncap, int mbits, hipStream_t s);
hipError_t fill(double* A, int64_t ld, int64_t m, int64_t n, double v, hipStream_t s);
hipError_t eye(double* A, int64_t ld, int64_t m, hipStream_t s);
hipError_t axpy(int64_t m, int64_t n, double alpha, const double* A, int64_t lda, double* C, int64_t ldc,
                hipStream_t s);
hipError_t transpose(const double* A, int64_t lda, int64_t m, int64_t n, double* B, int64_t ldb, hipStream_t s);
int trunc_lds_limit();

}  // namespace lu
}  // namespace hm
