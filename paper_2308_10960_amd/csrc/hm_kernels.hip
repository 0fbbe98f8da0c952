// HIP kernels (gfx950) of the H-matrix-vector product and their launchers.
//
// One product y += alpha * sum_b E_tau M_b E_sigma^T x (Sec. 2.1, Eq. (1);
// the product only needs the blocks decoded from storage, Sec. 5.4) runs as
// three stream-ordered kernels over the packed store (layout: hm_layout.hpp):
//
//  k_col     far field, phase 1: every wave streams one column tile (the rows
//            of V_b restricted to a column interval, for all low-rank blocks
//            covering it) and writes one partial dot product per column.
//  k_reduce  t_b[l] = s_b[l] * sum of the block's partials in interval order.
//  k_row     near field and far field, phase 2: one workgroup per row panel
//            gathers its sources (x for dense columns, t for U columns) into
//            LDS, streams the panel with 16-byte loads (lane = row), reduces
//            the four waves in LDS and updates its own rows of y once.
//
// Every sum has a fixed order, so results are bitwise reproducible and no
// atomics touch y.  Storage formats (FP64/FP32/FP16/BF16, Table 1) are
// decoded to the accumulation type in registers.

#include <hip/hip_runtime.h>

#include "hm_internal.hpp"

namespace hm {
namespace {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

__device__ __forceinline__ u32x4 ld16(const u32x4* p) { return __builtin_nontemporal_load(p); }

// acc += sum_c v[c] * z[c] over one 16-byte group of storage format DT.
template <typename AccT, int DT>
__device__ __forceinline__ AccT dot_group(u32x4 r, const AccT* __restrict__ z, AccT acc) {
  if constexpr (DT == HM_F64) {
    const f64x2 v = __builtin_bit_cast(f64x2, r);
    acc = fmaT((AccT)v.x, z[0], acc);
    acc = fmaT((AccT)v.y, z[1], acc);
  } else if constexpr (DT == HM_F32) {
    const f32x4 v = __builtin_bit_cast(f32x4, r);
#pragma unroll
    for (int c = 0; c < 4; ++c) acc = fmaT((AccT)v[c], z[c], acc);
  } else if constexpr (DT == HM_F16) {
    const f16x8 v = __builtin_bit_cast(f16x8, r);
#pragma unroll
    for (int c = 0; c < 8; ++c) acc = fmaT((AccT)(float)v[c], z[c], acc);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float lo = __uint_as_float(r[c] << 16);
      const float hi = __uint_as_float(r[c] & 0xffff0000u);
      acc = fmaT((AccT)lo, z[2 * c], acc);
      acc = fmaT((AccT)hi, z[2 * c + 1], acc);
    }
  }
  return acc;
}

// acc[c] += v[c] * xi for the G columns of one 16-byte group.
template <typename AccT, int DT>
__device__ __forceinline__ void axpy_group(u32x4 r, AccT xi, AccT* acc) {
  if constexpr (DT == HM_F64) {
    const f64x2 v = __builtin_bit_cast(f64x2, r);
    acc[0] = fmaT((AccT)v.x, xi, acc[0]);
    acc[1] = fmaT((AccT)v.y, xi, acc[1]);
  } else if constexpr (DT == HM_F32) {
    const f32x4 v = __builtin_bit_cast(f32x4, r);
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = fmaT((AccT)v[c], xi, acc[c]);
  } else if constexpr (DT == HM_F16) {
    const f16x8 v = __builtin_bit_cast(f16x8, r);
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = fmaT((AccT)(float)v[c], xi, acc[c]);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      acc[2 * c] = fmaT((AccT)__uint_as_float(r[c] << 16), xi, acc[2 * c]);
      acc[2 * c + 1] = fmaT((AccT)__uint_as_float(r[c] & 0xffff0000u), xi, acc[2 * c + 1]);
    }
  }
}

// Value of lane i of v (i uniform across the wave).
__device__ __forceinline__ float bcast(float v, int i) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
}
__device__ __forceinline__ double bcast(double v, int i) {
  const unsigned long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffu), i);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), i);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// ---------------------------------------------------------------- k_col

template <typename AccT>
struct ColArgs {
  const uint8_t* store;
  const ColTile* tiles;
  const int32_t* dst;
  const AccT* x;
  AccT* part;
  int64_t n_tiles;
};

template <typename AccT, int DT>
__device__ __forceinline__ void col_tile(const ColArgs<AccT>& a, const ColTile& T, int lane) {
  constexpr int G = group_width(DT);
  const AccT xv = lane < T.nrows ? a.x[T.x0 + lane] : AccT(0);
  AccT acc[G];
#pragma unroll
  for (int c = 0; c < G; ++c) acc[c] = AccT(0);
  const bool act = lane < T.ngroups;
  const int rstride = T.ld * dtype_size(DT) / 16;
  const u32x4* p = reinterpret_cast<const u32x4*>(a.store + T.data_off) + lane;
  int i = 0;
  for (; i + 8 <= T.nrows; i += 8) {
    u32x4 r[8];
    if (act) {
#pragma unroll
      for (int u = 0; u < 8; ++u) r[u] = ld16(p + (size_t)(i + u) * rstride);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const AccT xi = bcast(xv, i + u);
      if (act) axpy_group<AccT, DT>(r[u], xi, acc);
    }
  }
  for (; i < T.nrows; ++i) {
    u32x4 r;
    if (act) r = ld16(p + (size_t)i * rstride);
    const AccT xi = bcast(xv, i);
    if (act) axpy_group<AccT, DT>(r, xi, acc);
  }
  if (act) {
    const int32_t* d = a.dst + T.dst_off + lane * G;
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const int32_t di = d[c];
      if (di >= 0) a.part[di] = acc[c];
    }
  }
}

template <typename AccT>
__global__ __launch_bounds__(256) void k_col(ColArgs<AccT> a) {
  const int lane = threadIdx.x & 63;
  const int64_t ti = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (ti >= a.n_tiles) return;
  const ColTile T = a.tiles[ti];
  switch (T.dtype) {
    case HM_F64:
      if constexpr (sizeof(AccT) == 8) col_tile<AccT, HM_F64>(a, T, lane);
      break;
    case HM_F32: col_tile<AccT, HM_F32>(a, T, lane); break;
    case HM_F16: col_tile<AccT, HM_F16>(a, T, lane); break;
    default: col_tile<AccT, HM_BF16>(a, T, lane); break;
  }
}

// ---------------------------------------------------------------- k_reduce

template <typename AccT>
struct RedArgs {
  const TBlock* tb;
  const int32_t* owner;
  const AccT* sigma;      // nullptr when no block keeps singular values
  const AccT* part;
  AccT* t;
  int64_t n_large, n_large_t, n_t;
};

template <typename AccT>
__global__ __launch_bounds__(256) void k_reduce(RedArgs<AccT> a) {
  __shared__ AccT sh[256];
  const int tid = threadIdx.x;
  if ((int64_t)blockIdx.x < a.n_large) {
    const TBlock B = a.tb[blockIdx.x];
    const int k = B.k;
    if (k <= 256) {
      // thread (phase, l): phases stride the intervals, then a fixed-order
      // sum over phases
      const int P = 256 / k;
      const int l = tid % k, ph = tid / k;
      AccT acc = AccT(0);
      if (ph < P)
        for (int j = ph; j < B.nseg; j += P) acc += a.part[B.pst + (int64_t)j * k + l];
      sh[tid] = acc;
      __syncthreads();
      if (tid < k) {
        AccT s = AccT(0);
        for (int q = 0; q < P; ++q) s += sh[q * k + tid];
        const int64_t o = B.toff + tid;
        a.t[o] = a.sigma ? s * a.sigma[o] : s;
      }
    } else {
      for (int l = tid; l < k; l += 256) {
        AccT s = AccT(0);
        for (int j = 0; j < B.nseg; ++j) s += a.part[B.pst + (int64_t)j * k + l];
        const int64_t o = B.toff + l;
        a.t[o] = a.sigma ? s * a.sigma[o] : s;
      }
    }
    return;
  }
  const int64_t o = a.n_large_t + ((int64_t)blockIdx.x - a.n_large) * 256 + tid;
  if (o >= a.n_t) return;
  const TBlock B = a.tb[a.owner[o - a.n_large_t]];
  const int l = (int)(o - B.toff);
  AccT s = AccT(0);
  for (int j = 0; j < B.nseg; ++j) s += a.part[B.pst + (int64_t)j * B.k + l];
  a.t[o] = a.sigma ? s * a.sigma[o] : s;
}

// ---------------------------------------------------------------- k_row

template <typename AccT>
struct RowArgs {
  const uint8_t* store;
  const RowPanel* rp;
  const RowSection* rs;
  const int32_t* order;
  const int32_t* src;
  const AccT* x;
  const AccT* t;
  AccT* y;
  AccT alpha;
  int32_t n_cols;
};

template <typename AccT, int DT, int U>
__device__ __forceinline__ AccT row_section(const uint8_t* base, int m, int g_lo, int g_hi,
                                            const AccT* z, int lane, int wave, AccT acc) {
  constexpr int G = group_width(DT);
  const u32x4* p = reinterpret_cast<const u32x4*>(base) + lane;
  int g = g_lo + wave;
  for (; g + 4 * (U - 1) < g_hi; g += 4 * U) {
    u32x4 r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = ld16(p + (size_t)(g + 4 * u) * m);
#pragma unroll
    for (int u = 0; u < U; ++u) acc = dot_group<AccT, DT>(r[u], z + (g + 4 * u) * G, acc);
  }
  for (; g < g_hi; g += 4) acc = dot_group<AccT, DT>(ld16(p + (size_t)g * m), z + g * G, acc);
  return acc;
}

template <typename AccT, int CAP, int U>
__global__ __launch_bounds__(256) void k_row(RowArgs<AccT> a) {
  __shared__ AccT zs[CAP];
  __shared__ AccT red[4][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const RowPanel P = a.rp[a.order[blockIdx.x]];
  AccT acc = AccT(0);
  for (int c_lo = 0; c_lo < P.ncols; c_lo += CAP) {
    const int c_hi = min(P.ncols, c_lo + CAP);
    const int32_t* src = a.src + P.src_off;
    for (int c = c_lo + tid; c < c_hi; c += 256) {
      const int s = src[c];
      zs[c - c_lo] = s < a.n_cols ? a.x[s] : a.t[s - a.n_cols];
    }
    __syncthreads();
    if (lane < P.m) {
      for (int q = 0; q < P.nsec; ++q) {
        const RowSection S = a.rs[P.sec0 + q];
        const int G = group_width(S.dtype);
        const int g_lo = max(0, c_lo - S.col0) / G;
        const int g_hi = min(S.ngroups, max(0, c_hi - S.col0) / G);
        if (g_hi <= g_lo) continue;
        const uint8_t* base = a.store + S.data_off;
        const AccT* z = zs + (S.col0 - c_lo);
        switch (S.dtype) {
          case HM_F64:
            if constexpr (sizeof(AccT) == 8)
              acc = row_section<AccT, HM_F64, U>(base, P.m, g_lo, g_hi, z, lane, wave, acc);
            break;
          case HM_F32: acc = row_section<AccT, HM_F32, U>(base, P.m, g_lo, g_hi, z, lane, wave, acc); break;
          case HM_F16: acc = row_section<AccT, HM_F16, U>(base, P.m, g_lo, g_hi, z, lane, wave, acc); break;
          default: acc = row_section<AccT, HM_BF16, U>(base, P.m, g_lo, g_hi, z, lane, wave, acc); break;
        }
      }
    }
    __syncthreads();
  }
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && lane < P.m) {
    const AccT s = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    a.y[P.row0 + lane] += a.alpha * s;
  }
}

// ---------------------------------------------------------------- launch

template <typename AccT>
hipError_t launch_typed(const hm_matrix& A, double alpha, const void* x, void* y, void* work,
                        hipStream_t s, hipEvent_t* ev) {
  const StoreHeader& h = A.hdr;
  const uint8_t* st = A.d_store;
  AccT* part = reinterpret_cast<AccT*>(work);
  AccT* t = reinterpret_cast<AccT*>(reinterpret_cast<uint8_t*>(work) + A.work_t_off);
  if (ev) (void)hipEventRecord(ev[0], s);
  if (h.n_col_tiles > 0) {
    ColArgs<AccT> ca{st, reinterpret_cast<const ColTile*>(st + h.off_col_tiles),
                     reinterpret_cast<const int32_t*>(st + h.off_col_dst),
                     reinterpret_cast<const AccT*>(x), part, h.n_col_tiles};
    hipLaunchKernelGGL(k_col<AccT>, dim3((unsigned)((h.n_col_tiles + 3) / 4)), dim3(256), 0, s, ca);
    if (ev) (void)hipEventRecord(ev[1], s);
    RedArgs<AccT> ra{reinterpret_cast<const TBlock*>(st + h.off_tblocks),
                     reinterpret_cast<const int32_t*>(st + h.off_owner),
                     h.has_sigma ? reinterpret_cast<const AccT*>(st + h.off_sigma) : nullptr,
                     part, t, h.n_large, h.n_large_t, h.n_t};
    const int64_t nred = h.n_large + (h.n_t - h.n_large_t + 255) / 256;
    if (nred > 0) hipLaunchKernelGGL(k_reduce<AccT>, dim3((unsigned)nred), dim3(256), 0, s, ra);
  } else if (ev) {
    (void)hipEventRecord(ev[1], s);
  }
  if (ev) (void)hipEventRecord(ev[2], s);
  RowArgs<AccT> ra{st,
                   reinterpret_cast<const RowPanel*>(st + h.off_row_panels),
                   reinterpret_cast<const RowSection*>(st + h.off_row_sections),
                   reinterpret_cast<const int32_t*>(st + h.off_row_order),
                   reinterpret_cast<const int32_t*>(st + h.off_row_src),
                   reinterpret_cast<const AccT*>(x), t, reinterpret_cast<AccT*>(y), (AccT)alpha,
                   (int32_t)h.n_cols};
  constexpr int CAP = 16384 / sizeof(AccT);
  hipLaunchKernelGGL((k_row<AccT, CAP, 4>), dim3((unsigned)h.n_row_panels), dim3(256), 0, s, ra);
  if (ev) (void)hipEventRecord(ev[3], s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mvm(const hm_matrix& A, double alpha, const void* x, void* y, void* work,
                      hipStream_t s, hipEvent_t* ev) {
  if (!ev && A.prof.on && A.prof.calls < A.prof.max_calls) ev = &A.prof.ev[4 * (size_t)A.prof.calls++];
  return A.acc_dtype == HM_F64 ? launch_typed<double>(A, alpha, x, y, work, s, ev)
                               : launch_typed<float>(A, alpha, x, y, work, s, ev);
}

hipError_t launch_mvm_batch(const hm_matrix& A, int nrhs, double alpha, const void* X, int64_t ldx,
                            void* Y, int64_t ldy, void* work, hipStream_t s) {
  const int vs = A.acc_dtype == HM_F64 ? 8 : 4;
  for (int c = 0; c < nrhs; ++c) {
    hipError_t e = launch_mvm(A, alpha, static_cast<const uint8_t*>(X) + (size_t)c * ldx * vs,
                              static_cast<uint8_t*>(Y) + (size_t)c * ldy * vs, work, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace hm
