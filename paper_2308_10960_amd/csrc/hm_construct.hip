// HIP kernels (gfx950) that construct the leaves of an H-matrix on the GPU,
// in FP64, and their launcher (hm_construct):
//
//  k_dense_fill   inadmissible leaves: D(i, j) = K(p_{rb+i}, p_{cb+j}),
//                 column-major, one workgroup per leaf.
//  k_aca          admissible leaves: partially pivoted adaptive cross
//                 approximation U V^T (Sec. 5.1), one workgroup per leaf:
//                 the first pivot row is the leaf's first row; the column
//                 pivot is the argmax of the residual row, the next row the
//                 argmax of the newest column over the rows not used yet (a
//                 zero residual row moves on to the lowest unused row); it
//                 stops when |u_k| |v_k| <= eps_aca |S_k|_F, |S_k|_F updated
//                 recursively, or at min(m, n) steps.
//  k_recompress   admissible leaves: truncation by QR and SVD (Sec. 2.2,
//                 Algorithm 1): Householder QR of U and of V, B = R_U R_V^T,
//                 one-sided Jacobi SVD of B, the smallest rank k whose
//                 Frobenius tail of singular values is <= eps times the
//                 whole, W = Q_U U_s(:,1:k), X = Q_V V_s(:,1:k), s = S(1:k)
//                 (s folded into W unless kept); one workgroup per leaf, in
//                 three launches by ACA rank (the SVD works in LDS).
//
// Kernel functions (the point-kernel stand-ins of the model problems of
// Sec. 5.1): Laplace 1/(4 pi r) with diagonal 1/(4 pi h), and the
// exponential exp(-r / l) with d added on the diagonal.
//
// Every reduction has a fixed order and its result is broadcast from one
// place, so control flow that depends on a reduced value is uniform across
// the workgroup.

#include <algorithm>
#include <cmath>

#include <hip/hip_runtime.h>

#include "../../include/hm_construct.h"
#include "hm_dense.hpp"
#include "hm_internal.hpp"

namespace hm {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kThreads = 256;
constexpr int kRecompressThreads = 512;   // the truncation core's workgroup for the recompression
constexpr int kWaves = kThreads / 64;

struct CKern {
  int32_t kind;   // HM_KERNEL_LAPLACE or HM_KERNEL_EXP
  double p0, p1;  // Laplace: h; exponential: length l, diagonal shift d
};

__device__ __forceinline__ double kval(const CKern& K, const double* __restrict__ pc, int64_t i, int64_t j) {
  const double dx = pc[3 * i] - pc[3 * j], dy = pc[3 * i + 1] - pc[3 * j + 1], dz = pc[3 * i + 2] - pc[3 * j + 2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  if (K.kind == HM_KERNEL_LAPLACE) return i == j ? 1.0 / (4.0 * kPi * K.p0) : 1.0 / (4.0 * kPi * r);
  const double v = exp(-r / K.p0);
  return i == j ? v + K.p1 : v;
}

using dense::block_sum;
using dense::wave_sum;

// Argmax of v over the workgroup with the lowest index on ties (index -1
// with value -1 where no thread has a candidate); the same result in every
// thread.  Each thread passes its own best (value, index), found scanning
// its indices upward with a strict comparison.
__device__ __forceinline__ void block_argmax(double& v, int64_t& idx, double* sv, int64_t* si) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int64_t oi = __shfl_xor(idx, o, 64);
    if (ov > v || (ov == v && oi >= 0 && (idx < 0 || oi < idx))) { v = ov; idx = oi; }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { sv[wave] = v; si[wave] = idx; }
  __syncthreads();
  v = sv[0];
  idx = si[0];
#pragma unroll
  for (int w = 1; w < kWaves; ++w)
    if (sv[w] > v || (sv[w] == v && si[w] >= 0 && (idx < 0 || si[w] < idx))) { v = sv[w]; idx = si[w]; }
  __syncthreads();
}

// One workgroup per leaf of the batch; admissible leaves return at once.
__global__ __launch_bounds__(kThreads) void k_dense_fill(const hm_cblock* __restrict__ blocks, const double* pc,
                                                          CKern K, double* __restrict__ out) {
  const hm_cblock B = blocks[blockIdx.x];
  if (B.adm) return;                                 // uniform: the whole workgroup
  const int64_t m = B.m, mn = (int64_t)B.m * B.n;
  double* D = out + B.out;
  for (int64_t e = threadIdx.x; e < mn; e += kThreads) D[e] = kval(K, pc, B.rb + e % m, B.cb + e / m);
}

// ACA of one admissible leaf into its scratch: U (m x cap) at scr, V
// (n x cap) after it, then m bytes of used-row flags.  One workgroup per
// leaf of the batch; dense leaves get rank 0.  aca_rank: the ACA rank, or -1
// when cap columns did not reach the stopping criterion (cap < min(m, n)).
// rank: 0 for a dense leaf or a zero ACA rank, -1 with aca_rank -1, else -2
// (to be set by k_recompress).
__global__ __launch_bounds__(kThreads) void k_aca(const hm_cblock* __restrict__ blocks, const double* pc, CKern K,
                                                   double eps, double* __restrict__ scr,
                                                   int32_t* __restrict__ aca_rank, int32_t* __restrict__ rank) {
  __shared__ double sv[kWaves];
  __shared__ int64_t si[kWaves];
  __shared__ double urow[HM_CONSTRUCT_MAX_RANK], vrow[HM_CONSTRUCT_MAX_RANK];
  __shared__ double sa[kWaves][HM_CONSTRUCT_MAX_RANK], sb[kWaves][HM_CONSTRUCT_MAX_RANK];
  const int64_t b = blockIdx.x;
  const hm_cblock B = blocks[b];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (!B.adm) {                                      // uniform: the whole workgroup
    if (tid == 0) aca_rank[b] = rank[b] = 0;
    return;
  }
  const int64_t m = B.m, n = B.n;
  const int cap = B.cap;
  double* U = scr + B.scr;
  double* V = U + m * cap;
  uint8_t* used = reinterpret_cast<uint8_t*>(V + n * cap);
  for (int64_t i = tid; i < m; i += kThreads) used[i] = 0;
  const int64_t kmax = std::min(m, n);
  int r = 0, status = 0;
  int64_t piv_row = 0, nused = 0;
  double normS2 = 0;
  __syncthreads();
  while (r < kmax && nused < m) {
    if (r == cap) { status = -1; break; }
    for (int l = tid; l < r; l += kThreads) urow[l] = U[(int64_t)l * m + piv_row];
    __syncthreads();
    // residual row of piv_row -> column r of V (unscaled)
    double* row = V + (int64_t)r * n;
    double best = -1;
    int64_t jp = -1;
    for (int64_t j = tid; j < n; j += kThreads) {
      double v = kval(K, pc, B.rb + piv_row, B.cb + j);
      for (int l = 0; l < r; ++l) v -= urow[l] * V[(int64_t)l * n + j];
      row[j] = v;
      if (fabs(v) > best) { best = fabs(v); jp = j; }
    }
    block_argmax(best, jp, sv, si);
    if (tid == 0) used[piv_row] = 1;
    ++nused;
    __syncthreads();
    if (best == 0) {
      // a zero residual row: take the lowest unused row
      double f = -1;
      int64_t nxt = -1;
      for (int64_t i = tid; i < m; i += kThreads)
        if (!used[i]) { f = 0; nxt = i; break; }
      block_argmax(f, nxt, sv, si);
      if (nxt < 0) break;
      piv_row = nxt;
      continue;
    }
    const double piv = row[jp];
    for (int l = tid; l < r; l += kThreads) vrow[l] = V[(int64_t)l * n + jp];
    __syncthreads();
    // residual column of jp -> column r of U; row scaled by the pivot
    double* col = U + (int64_t)r * m;
    double pu = 0, pv = 0;
    for (int64_t i = tid; i < m; i += kThreads) {
      double c = kval(K, pc, B.rb + i, B.cb + jp);
      for (int l = 0; l < r; ++l) c -= vrow[l] * U[(int64_t)l * m + i];
      col[i] = c;
      pu += c * c;
    }
    for (int64_t j = tid; j < n; j += kThreads) {
      const double v = row[j] / piv;
      row[j] = v;
      pv += v * v;
    }
    // |S_k|_F^2 = |S_{k-1}|_F^2 + 2 sum_l (u_k . u_l)(v_k . v_l) + |u_k|^2 |v_k|^2
    for (int l = 0; l < r; ++l) {
      double a = 0, c = 0;
      for (int64_t i = tid; i < m; i += kThreads) a += col[i] * U[(int64_t)l * m + i];
      for (int64_t j = tid; j < n; j += kThreads) c += row[j] * V[(int64_t)l * n + j];
      a = wave_sum(a);
      c = wave_sum(c);
      if (lane == 0) { sa[wave][l] = a; sb[wave][l] = c; }
    }
    const double nu = block_sum<kWaves>(pu, sv), nv = block_sum<kWaves>(pv, sv);   // synchronizes: sa, sb complete
    double cross = 0;
    for (int l = 0; l < r; ++l) {
      double a = 0, c = 0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) { a += sa[w][l]; c += sb[w][l]; }
      cross += a * c;
    }
    normS2 += 2.0 * cross + nu * nv;
    ++r;
    if (sqrt(nu * nv) <= eps * sqrt(fabs(normS2))) break;
    // next pivot row: the largest |u_k| over the unused rows
    double bu = -1;
    int64_t nxt = -1;
    for (int64_t i = tid; i < m; i += kThreads)
      if (!used[i] && fabs(col[i]) > bu) { bu = fabs(col[i]); nxt = i; }
    block_argmax(bu, nxt, sv, si);
    if (nxt < 0) break;
    piv_row = nxt;
  }
  if (tid == 0) {
    aca_rank[b] = status < 0 ? -1 : r;
    rank[b] = status < 0 ? -1 : (r == 0 ? 0 : -2);
  }
}

// Algorithm 1 on the ACA factors of one leaf whose ACA rank r lies in
// (rlo, rhi] (the other leaves of the launch return at once), one workgroup
// of kRecompressThreads threads per leaf.  LDS
// (dynamic): the r x r matrix being orthogonalized (B, then U_s diag(S)) and
// V_s, both column-major with leading dimension r.  Output: W (m x k) at
// out, X (n x k) at out + m cap, s (k) at out + (m + n) cap; rank = k.
__global__ __launch_bounds__(kRecompressThreads) void k_recompress(const hm_cblock* __restrict__ blocks, int rlo, int rhi,
                                                          double eps, int keep_sigma, double* __restrict__ out,
                                                          double* __restrict__ scr,
                                                          const int32_t* __restrict__ aca_rank,
                                                          int32_t* __restrict__ rank) {
  extern __shared__ double dyn[];
  __shared__ dense::TruncShared sh;
  const int64_t b = blockIdx.x;
  const int r = aca_rank[b];
  if (r <= rlo || r > rhi) return;                   // uniform: the whole workgroup
  const hm_cblock B = blocks[b];
  const int64_t m = B.m, n = B.n;
  const int cap = B.cap;
  double* U = scr + B.scr;
  double* V = U + m * cap;
  double* W = out + B.out;
  double* X = W + m * cap;
  double* sg = X + n * cap;
  const int k = dense::truncate_core(U, m, V, n, r, eps, dyn, 2 * (int64_t)rhi * rhi, nullptr, sh, W, X, !keep_sigma,
                                     sg);
  if (threadIdx.x == 0) rank[b] = k;
}

// Packs the result of every leaf densely: leaf b's data at packed + off[b]
// -- D (m x n), or W (m x k), X (n x k), s (k) of an admissible leaf of
// final rank k >= 0 -- skipping a leaf whose data would end beyond cap.
__global__ __launch_bounds__(kThreads) void k_pack(const hm_cblock* __restrict__ blocks,
                                                    const int32_t* __restrict__ rank, const double* __restrict__ out,
                                                    const int64_t* __restrict__ off, double* __restrict__ packed,
                                                    int64_t cap) {
  const int64_t b = blockIdx.x;
  const hm_cblock B = blocks[b];
  const int k = rank[b];
  const int64_t m = B.m, n = B.n, o = off[b];
  if (!B.adm) {
    if (o < 0 || o + m * n > cap) return;
    for (int64_t e = threadIdx.x; e < m * n; e += kThreads) packed[o + e] = out[B.out + e];
    return;
  }
  if (k < 0 || o < 0 || o + (m + n + 1) * k > cap) return;
  const double* W = out + B.out;
  const double* X = W + m * B.cap;
  const double* sg = X + n * B.cap;
  double* p = packed + o;
  for (int64_t e = threadIdx.x; e < m * k; e += kThreads) p[e] = W[e];
  for (int64_t e = threadIdx.x; e < n * k; e += kThreads) p[m * k + e] = X[e];
  for (int64_t e = threadIdx.x; e < k; e += kThreads) p[(m + n) * k + e] = sg[e];
}

}  // namespace

hipError_t launch_construct_pack(const hm_cblock* d_blocks, int64_t n_blocks, const int32_t* d_rank,
                                 const double* d_out, const int64_t* d_off, double* d_packed, int64_t cap,
                                 hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)n_blocks), dim3(kThreads), 0, s, d_blocks, d_rank, d_out, d_off,
                     d_packed, cap);
  return hipGetLastError();
}

// Largest ACA rank whose SVD fits the LDS of one workgroup on the current
// device (the static LDS of k_recompress plus two r x r FP64 matrices).
hipError_t construct_rank_limit(int* rmax) {
  int dev = 0, lds = 0, optin = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess)
    lds = std::max(lds, optin);
  hipFuncAttributes fa{};
  e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k_recompress));
  if (e != hipSuccess) return e;
  const int64_t room = (int64_t)lds - (int64_t)fa.sharedSizeBytes;
  int r = 0;
  while (r < HM_CONSTRUCT_MAX_RANK && 16 * (int64_t)(r + 1) * (r + 1) <= room) ++r;
  *rmax = r;
  return hipSuccess;
}

hipError_t launch_construct(const hm_cblock* d_blocks, int64_t n_blocks, const double* d_points,
                            const hm_construct_opts& o, double* d_out, double* d_scr, int32_t* d_aca_rank,
                            int32_t* d_rank, int r_lds_max, hipStream_t s) {
  const CKern K{o.kernel, o.params[0], o.params[1]};
  if (n_blocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)n_blocks);
  hipLaunchKernelGGL(k_dense_fill, grid, dim3(kThreads), 0, s, d_blocks, d_points, K, d_out);
  hipLaunchKernelGGL(k_aca, grid, dim3(kThreads), 0, s, d_blocks, d_points, K, o.eps_aca, d_scr, d_aca_rank,
                     d_rank);
  // launches by ACA rank: the SVD keeps two r x r matrices in LDS
  const int bounds[4] = {0, std::min(32, r_lds_max), std::min(64, r_lds_max), r_lds_max};
  const size_t lds_max = (size_t)16 * r_lds_max * r_lds_max;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_recompress),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
  if (e != hipSuccess) return e;
  for (int c = 0; c < 3; ++c) {
    const int lo = bounds[c], hi = bounds[c + 1];
    if (hi <= lo) continue;
    hipLaunchKernelGGL(k_recompress, grid, dim3(kRecompressThreads), (size_t)16 * hi * hi, s, d_blocks, lo, hi, o.eps,
                       o.keep_sigma, d_out, d_scr, d_aca_rank, d_rank);
  }
  return hipGetLastError();
}

}  // namespace hm
