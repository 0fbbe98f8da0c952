// Device building blocks of the FP64 dense linear algebra that the GPU
// construction (hm_construct.hip) and the H-LU (hm_lu.hip) share: workgroup
// reductions, Householder QR in place, the application of its reflectors,
// and the truncation core of Algorithm 1 (Sec. 2.2) on two factors whose
// small SVD runs in LDS.
//
// Every routine is called by all threads of one workgroup (a multiple of 64,
// at most kWThreads); every reduction has a fixed order and broadcasts its
// result, so control flow that depends on a reduced value is uniform across
// the workgroup.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace hm {
namespace dense {

constexpr int kWThreads = 1024;              // largest workgroup the routines below are called by
constexpr int kWWaves = kWThreads / 64;
constexpr int kMaxR = 256;    // widest factor pair the shared arrays hold
constexpr int kJacobiLanes = 8;   // lanes that rotate one column pair of the Jacobi step

// Threads and waves of the calling workgroup (at most kWThreads, a multiple
// of 64): the routines below run on workgroups of any such size.
__device__ __forceinline__ int nthreads() { return (int)blockDim.x; }
__device__ __forceinline__ int nwaves() { return (int)blockDim.x >> 6; }

// v of the lane that the DPP pattern CTRL names (rows in ROW_MASK; the lanes
// of the other rows get 0).  Both 32-bit halves move the same way.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over each row of 16 lanes, the row's total in all its lanes: pairs
// (quad_perm 1,0,3,2), quads (2,3,0,1), half rows (row_half_mirror), rows
// (row_mirror).  Row-local, so rows of a wave that are inactive do not
// matter.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_move<0xB1, 0xF>(v);
  v += dpp_move<0x4E, 0xF>(v);
  v += dpp_move<0x141, 0xF>(v);
  v += dpp_move<0x140, 0xF>(v);
  return v;
}

// Sum over the wave, the same value in every lane (a fixed order): the row
// sums, then rows 0 + 1 and 2 + 3 by row_bcast15, all four rows by
// row_bcast31 into lane 63, read back into every lane.  Every lane of the
// wave must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v = row16_sum(v);
  v += dpp_move<0x142, 0xA>(v);
  v += dpp_move<0x143, 0xC>(v);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over a workgroup of NW waves (NW = 0: all of the calling workgroup's),
// the same value in every thread.  sred: one double per wave of LDS; the call
// synchronizes twice.
template <int NW = 0>
__device__ __forceinline__ double block_sum(double v, double* sred) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  double s = 0;
  const int nw = NW > 0 ? NW : nwaves();            // NW = 0: the workgroup's waves
  for (int w = 0; w < nw; ++w) s += sred[w];
  __syncthreads();
  return s;
}

// Orders the memory accesses (LDS or global) of the calling wave's lanes:
// what a lane wrote before is seen by every lane of the wave after (no
// workgroup barrier).
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Householder QR of A (m x r, column-major, leading dimension lda, m >= r)
// in place, in LDS or global memory: R in the upper triangle, the
// reflectors v_j (v_j[j] = 1 implied) below the diagonal, and tau_j in tau
// (LDS), H_j = I - tau_j v_j v_j^T.  Step k:
// every wave forms the reflector of column k from the column's sum of
// squares (a wave sum over the rows, the same value in every wave); wave w
// applies it to the later columns j = k + 1 + w, k + 1 + w + kWWaves, ...,
// its lanes over the rows with a wave sum per column; after the step's
// barrier wave 0 scales column k to the reflector.  One barrier per step.
__device__ inline void qr_waves(double* A, int lda, int m, int r, double* tau) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int k = 0; k < r; ++k) {
    double* a = A + (int64_t)k * lda;
    double p = 0;
    for (int i = k + 1 + lane; i < m; i += 64) p += a[i] * a[i];
    p = wave_sum(p);
    const double akk = a[k];
    const double nrm = sqrt(akk * akk + p);
    double tk = 0, iv = 0, alpha = akk;
    if (nrm != 0) {
      alpha = akk > 0 ? -nrm : nrm;
      const double v0 = akk - alpha;
      iv = 1.0 / v0;
      tk = -v0 / alpha;
    }
    if (tk != 0)
      for (int j = k + 1 + w; j < r; j += nwaves()) {
        double* c = A + (int64_t)j * lda;
        double s = 0;
        for (int i = k + 1 + lane; i < m; i += 64) s += a[i] * c[i];
        s = (c[k] + wave_sum(s) * iv) * tk;
        for (int i = k + 1 + lane; i < m; i += 64) c[i] -= s * (a[i] * iv);
        if (lane == 0) c[k] -= s;
      }
    __syncthreads();
    if (w == 0) {
      if (tk != 0)
        for (int i = k + 1 + lane; i < m; i += 64) a[i] *= iv;
      if (lane == 0) {
        a[k] = alpha;
        tau[k] = tk;
      }
    }
  }
  __syncthreads();
}

// Z := H_0 ... H_{r-1} Z (Z m x k, leading dimension ldz; LDS or global
// memory) with the reflectors of qr_waves in A (leading dimension lda): wave w
// takes the columns w, w + kWWaves, ... of Z and applies the reflectors
// r - 1, ..., 0 to each, its lanes over the rows (no workgroup barrier
// between reflectors).  cols: when not null, column c of Z is column
// cols[c] of the array at Z (only those columns are transformed).
__device__ inline void apply_q_waves(const double* A, int lda, int m, int r, const double* tau, double* Z, int ldz,
                                     int k, const int* cols = nullptr) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c = w; c < k; c += nwaves()) {
    double* z = Z + (int64_t)(cols ? cols[c] : c) * ldz;
    for (int j = r - 1; j >= 0; --j) {
      const double tj = tau[j];
      if (tj == 0) continue;
      const double* v = A + (int64_t)j * lda;
      double s = 0;
      for (int i = j + 1 + lane; i < m; i += 64) s += v[i] * z[i];
      s = (z[j] + wave_sum(s)) * tj;
      for (int i = j + 1 + lane; i < m; i += 64) z[i] -= s * v[i];
      if (lane == 0) z[j] -= s;
      wave_fence();                                 // z as updated, for the next reflector
    }
  }
  __syncthreads();
}

// Copies a (rows x cols) between column-major arrays, workgroup-wide.
__device__ inline void copy_mat(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows, int64_t cols) {
  for (int64_t e = threadIdx.x; e < rows * cols; e += nthreads()) dst[(e / rows) * ldd + e % rows] = src[(e / rows) * lds + e % rows];
  __syncthreads();
}

// LDS the truncation core needs besides its two dynamic r x r matrices.
struct TruncShared {
  double sv[kWWaves];
  double tauU[kMaxR], tauV[kMaxR];
  double nrm[kMaxR], S[kMaxR];
  double offg[kWThreads / kJacobiLanes];
  double tauB[kMaxR];
  int ord[kMaxR];
  int perm[kMaxR];
  int keep;
  int more;
  int piv;
};

// Sum over the 8 lanes of a Jacobi lane group (half a DPP row; the group's
// lanes get the total): pairs, quads, then row_half_mirror.
__device__ __forceinline__ double group_sum(double v) {
  v += dpp_move<0xB1, 0xF>(v);
  v += dpp_move<0x4E, 0xF>(v);
  v += dpp_move<0x141, 0xF>(v);
  return v;
}

// Algorithm 1 on U (m x r) and V (n x r), both column-major with leading
// dimensions m and n, m >= r, n >= r, r <= kMaxR; U and V are overwritten
// by their QR factors.  lds: lds_doubles doubles of LDS, which hold a
// factor for its QR (qr_waves) when it fits, then the two r x r matrices
// of the SVD when they fit (else gscr, 2 r^2 doubles of global memory,
// holds them) and the reflectors of Q_B when a third fits (else X), then
// reflectors and result for the application of Q.  W must hold m x r doubles and X n x r (they also serve
// as scratch).  Householder QR
// of U and V, B = R_U R_V^T, the SVD of B by a QR with column pivoting
// (B P = Q_B R) and one-sided Jacobi on R^T (round-robin ordering: in each
// round 8-lane groups rotate disjoint column pairs in parallel; the
// pivoting grades R, so that few sweeps are needed), singular values
// sorted descending (stable), k the smallest rank whose Frobenius tail is
// <= eps times the whole; then W = Q_U U_s(:, 1:k) (times diag(S) when
// fold), X = Q_V V_s(:, 1:k) written to W (m x k, leading dimension m) and
// X (n x k, leading dimension n), S(1:k) to sg when sg is not null.
// Returns k (the same in every thread).
__device__ inline int truncate_core(double* U, int64_t m, double* V, int64_t n, int r, double eps, double* lds,
                                    int64_t lds_doubles, double* gscr, TruncShared& sh, double* W, double* X,
                                    bool fold, double* sg) {
  const int tid = threadIdx.x;
  // QR of U and of V: in LDS (qr_waves) when the factor fits
  auto qr = [&](double* F, int64_t rows, double* tau) {
    const int ld = (int)(rows | 1);
    if ((int64_t)ld * r <= lds_doubles && rows <= 4096) {
      copy_mat(F, rows, lds, ld, rows, r);
      qr_waves(lds, ld, (int)rows, r, tau);
      copy_mat(lds, ld, F, rows, rows, r);
    } else {
      qr_waves(F, (int)rows, (int)rows, r, tau);      // in global memory
    }
  };
  qr(U, m, sh.tauU);
  qr(V, n, sh.tauV);
  // the two r x r matrices of the SVD: in LDS when they fit, else in global scratch
  double* Am = 2 * (int64_t)r * r <= lds_doubles ? lds : gscr;
  double* Vs = Am + (int64_t)r * r;
  // R_U -> Am, R_V -> Vs (upper triangles), then B = R_U R_V^T into W (r x r)
  for (int e = tid; e < r * r; e += nthreads()) {
    const int i = e % r, l = e / r;
    Am[e] = i <= l ? U[(int64_t)l * m + i] : 0.0;
    Vs[e] = i <= l ? V[(int64_t)l * n + i] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += nthreads()) {
    const int i = e % r, j = e / r;
    double s = 0;
    for (int l = std::max(i, j); l < r; ++l) s += Am[l * r + i] * Vs[l * r + j];
    W[e] = s;
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += nthreads()) Am[e] = W[e];
  for (int j = tid; j < r; j += nthreads()) sh.perm[j] = j;
  __syncthreads();
  // QR with column pivoting of B (B P = Q_B R; in place in Am): the
  // largest remaining column first, the lowest index on ties.  Column norms
  // by wave sums (wave w the columns k + w, k + w + kWWaves, ...), the
  // argmax and the column swap by wave 0, then the step of qr_waves: three
  // barriers per step.  One-sided Jacobi on R^T
  // then converges in a few sweeps, R being graded.
  const int lane = tid & 63, wv = tid >> 6;
  for (int k = 0; k < r; ++k) {
    for (int j = k + wv; j < r; j += nwaves()) {
      double s2 = 0;
      for (int i = k + lane; i < r; i += 64) s2 += Am[j * r + i] * Am[j * r + i];
      s2 = wave_sum(s2);
      if (lane == 0) sh.nrm[j] = s2;
    }
    __syncthreads();
    if (wv == 0) {
      double best = -1.0;
      int bj = r;
      for (int j = k + lane; j < r; j += 64)
        if (sh.nrm[j] > best) { best = sh.nrm[j]; bj = j; }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oj = __shfl_xor(bj, o, 64);
        if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; }
      }
      // every lane holds the same (best, bj): max and the index rule are exact
      const int jb = bj < r ? bj : k;
      if (jb != k)
        for (int i = lane; i < r; i += 64) {
          const double t = Am[k * r + i];
          Am[k * r + i] = Am[jb * r + i];
          Am[jb * r + i] = t;
        }
      if (lane == 0) {
        sh.piv = jb;
        const int t = sh.perm[k];
        sh.perm[k] = sh.perm[jb];
        sh.perm[jb] = t;
      }
    }
    __syncthreads();
    const int jb = sh.piv;
    double* a = Am + k * r;
    const double nrm = sqrt(sh.nrm[jb]);
    const double akk = a[k];
    double tk = 0, iv = 0, alpha = akk;
    if (nrm != 0) {
      alpha = akk > 0 ? -nrm : nrm;
      const double v0 = akk - alpha;
      iv = 1.0 / v0;
      tk = -v0 / alpha;
    }
    if (tk != 0)
      for (int j = k + 1 + wv; j < r; j += nwaves()) {
        double* c = Am + j * r;
        double s = 0;
        for (int i = k + 1 + lane; i < r; i += 64) s += a[i] * c[i];
        s = (c[k] + wave_sum(s) * iv) * tk;
        for (int i = k + 1 + lane; i < r; i += 64) c[i] -= s * (a[i] * iv);
        if (lane == 0) c[k] -= s;
      }
    __syncthreads();
    // wave 0 scales column k to its reflector; the next step touches only
    // the later columns, so no barrier before it
    if (wv == 0) {
      if (tk != 0)
        for (int i = k + 1 + lane; i < r; i += 64) a[i] *= iv;
      if (lane == 0) {
        a[k] = alpha;
        sh.tauB[k] = tk;
      }
    }
  }
  __syncthreads();
  // reflectors of Q_B (and R) to Qb (r x r, leading dimension r: in LDS
  // after Am and Vs when there is room, else X), then Am := R^T (lower
  // triangular), Vs := I
  double* Qb = (Am == lds && 3 * (int64_t)r * r <= lds_doubles) ? lds + 2 * (int64_t)r * r : X;
  for (int e = tid; e < r * r; e += nthreads()) Qb[e] = Am[e];
  __syncthreads();
  for (int e = tid; e < r * r; e += nthreads()) {
    const int i = e % r, j = e / r;                  // Am(i, j) = R(j, i)
    Am[e] = j <= i ? Qb[i * r + j] : 0.0;
    Vs[e] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  // one-sided Jacobi on the columns of Am = R^T, round-robin pairs (R = r
  // rounded up to even players; player R - 1 stays, the others rotate; a
  // pair with the player r, when r is odd, is skipped); afterwards
  // Am = R^T Vs has orthogonal columns
  const int R = r + (r & 1);
  const int grp = tid / kJacobiLanes, gl = tid % kJacobiLanes, ngrp = nthreads() / kJacobiLanes;
  // columns below 1e-16 |B|_F carry no singular value the truncation can
  // see and only rounding noise: pairs with such a column are not rotated
  double fro2 = 0;
  for (int e = tid; e < r * r; e += nthreads()) fro2 += Am[e] * Am[e];
  const double tiny = 1e-32 * block_sum(fro2, sh.sv);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0;
    for (int t = 0; t + 1 < R; ++t) {
      for (int pi = grp; pi < R / 2; pi += ngrp) {
        int p, q;
        if (pi == 0) {
          p = t;
          q = R - 1;
        } else {                                     // (t + pi) mod (R - 1), (t - pi) mod (R - 1)
          p = t + pi;
          if (p >= R - 1) p -= R - 1;
          q = t - pi;
          if (q < 0) q += R - 1;
        }
        if (p > q) { const int x = p; p = q; q = x; }
        if (q >= r) continue;                        // the same for the whole group
        double* ap = Am + p * r;
        double* aq = Am + q * r;
        double al = 0, be = 0, ga = 0;
        for (int i = gl; i < r; i += kJacobiLanes) {
          al += ap[i] * ap[i];
          be += aq[i] * aq[i];
          ga += ap[i] * aq[i];
        }
        al = group_sum(al);
        be = group_sum(be);
        ga = group_sum(ga);
        if (ga == 0 || al <= tiny || be <= tiny) continue;
        if (!(ga * ga > 1e-30 * (al * be))) continue;      // |ga| / sqrt(al be) <= 1e-15: converged
        off = 1;                                            // a rotation in this sweep
        const double zeta = (be - al) / (2.0 * ga);
        const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
        double* vp = Vs + p * r;
        double* vq = Vs + q * r;
        for (int i = gl; i < r; i += kJacobiLanes) {
          const double x = ap[i], y = aq[i];
          ap[i] = c * x - sn * y;
          aq[i] = sn * x + c * y;
          const double u = vp[i], w = vq[i];
          vp[i] = c * u - sn * w;
          vq[i] = sn * u + c * w;
        }
      }
      __syncthreads();
    }
    if (gl == 0) sh.offg[grp] = off;
    __syncthreads();
    if (tid == 0) {
      double o = 0;
      for (int g = 0; g < ngrp; ++g) o = std::max(o, sh.offg[g]);
      sh.more = o > 0;
    }
    __syncthreads();
    if (!sh.more) break;
    __syncthreads();
  }
  // singular values: column norms, sorted descending (stable)
  for (int j = tid; j < r; j += nthreads()) {
    double s2 = 0;
    for (int i = 0; i < r; ++i) s2 += Am[j * r + i] * Am[j * r + i];
    sh.nrm[j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = tid; j < r; j += nthreads()) {
    int pos = 0;
    for (int l = 0; l < r; ++l) pos += sh.nrm[l] > sh.nrm[j] || (sh.nrm[l] == sh.nrm[j] && l < j);
    sh.ord[pos] = j;
    sh.S[pos] = sh.nrm[j];
  }
  __syncthreads();
  if (tid == 0) {
    double tot = 0;
    for (int j = 0; j < r; ++j) tot += sh.S[j] * sh.S[j];
    int k = r;
    double tail = 0;
    while (k > 0) {
      const double t2 = tail + sh.S[k - 1] * sh.S[k - 1];
      if (sqrt(t2) <= eps * sqrt(tot)) { tail = t2; --k; } else break;
    }
    sh.keep = k;
  }
  __syncthreads();
  const int k = sh.keep;
  // B = (Q_B Vs) diag(S) (P Am / S)^T: the left singular vectors are Q_B
  // applied to the columns of Vs (reflectors in Qb), the right ones the
  // normalized columns of Am with their rows permuted back by P
  apply_q_waves(Qb, r, r, r, sh.tauB, Vs, r, k, sh.ord);      // the k kept columns only
  // W = Q_U [left(:, 1:k); 0], X = Q_V [right(:, 1:k); 0]
  for (int c = 0; c < k; ++c) {
    const int j = sh.ord[c];
    for (int64_t i = tid; i < m; i += nthreads()) W[(int64_t)c * m + i] = i < r ? Vs[j * r + i] : 0.0;
  }
  __syncthreads();                                  // the reflectors in Qb are read no more
  for (int c = 0; c < k; ++c) {
    const int j = sh.ord[c];
    const double inv = sh.S[c] > 0 ? 1.0 / sh.S[c] : 0.0;
    for (int64_t i = tid; i < n; i += nthreads()) X[(int64_t)c * n + i] = 0.0;
    __syncthreads();
    for (int i = tid; i < r; i += nthreads()) X[(int64_t)c * n + sh.perm[i]] = Am[j * r + i] * inv;
  }
  __syncthreads();
  // W := Q_U W, X := Q_V X: reflectors and result in LDS (apply_q_waves) when they fit
  auto applyq = [&](const double* F, int64_t rows, const double* tau, double* Z) {
    const int ld = (int)(rows | 1);
    if ((int64_t)ld * (r + k) <= lds_doubles && rows <= 4096) {
      copy_mat(F, rows, lds, ld, rows, r);
      copy_mat(Z, rows, lds + (int64_t)ld * r, ld, rows, k);
      apply_q_waves(lds, ld, (int)rows, r, tau, lds + (int64_t)ld * r, ld, k);
      copy_mat(lds + (int64_t)ld * r, ld, Z, rows, rows, k);
    } else {
      apply_q_waves(F, (int)rows, (int)rows, r, tau, Z, (int)rows, k);   // in global memory
    }
  };
  applyq(U, m, sh.tauU, W);
  applyq(V, n, sh.tauV, X);
  for (int c = 0; c < k; ++c) {
    if (sg && tid == 0) sg[c] = sh.S[c];
    if (fold)
      for (int64_t i = tid; i < m; i += nthreads()) W[(int64_t)c * m + i] *= sh.S[c];
  }
  __syncthreads();
  return k;
}

}  // namespace dense
}  // namespace hm
