// HIP kernels (gfx950) of the H-matrix-vector product and their launchers.
//
// One product y += alpha * sum_b E_tau M_b E_sigma^T x (Sec. 2.1, Eq. (1);
// the product only needs the blocks decoded from storage, Sec. 5.4) runs as
// three stream-ordered kernels over the packed store (layout: hm_layout.hpp):
//
//  k_p1      one grouped launch over two kinds of work item: the dense
//            sections of a row panel (near field, y += alpha D x; one
//            workgroup gathers x into LDS, streams the panel with 16-byte
//            loads, lane = row, and updates its rows of y), and groups of four
//            column tiles (far field, phase 1: a wave streams the rows of V_b
//            restricted to a column interval for all low-rank blocks covering
//            it and writes one partial dot product per column).
//  k_reduce  t_b[l] = s_b[l] * sum of the block's partials in interval order.
//  k_p2      far field, phase 2: the U sections of each row panel, with t
//            gathered into LDS (y += alpha U t).
//
// Every sum has a fixed order, so results are bitwise reproducible and no
// atomics touch y.  Storage formats (FP64/FP32/FP16/BF16, Table 1) are
// decoded to the accumulation type in registers.

#include <algorithm>

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

// ---------------------------------------------------------------- column tiles

template <typename AccT>
struct ColArgs {
  const uint8_t* store;
  const ColTile* tiles;
  const int32_t* dst;
  const AccT* x;
  AccT* part;
  int64_t n_tiles;
};

// One workgroup streams one column tile.  Lane l of every wave owns the G
// columns of group l; the tile's rows go to the four waves in interleaved
// batches of 8 (wave w takes batches w, w + 4, ...), x of 64 rows at a time
// sits in one register per lane and is broadcast by readlane.  The four
// waves' sums are added in a fixed order through LDS (red: 4 x 64 x G).
template <typename AccT, int DT>
__device__ __forceinline__ void col_tile(const ColArgs<AccT>& a, const ColTile& T, AccT* red) {
  constexpr int G = group_width(DT);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool act = lane < T.ngroups;
  AccT acc[G];
#pragma unroll
  for (int c = 0; c < G; ++c) acc[c] = AccT(0);
  const int rstride = T.ld * dtype_size(DT) / 16;
  const u32x4* p = reinterpret_cast<const u32x4*>(a.store + T.data_off) + lane;
  for (int i0 = 0; i0 < T.nrows; i0 += 64) {
    const int nr = min(64, T.nrows - i0);
    const AccT xv = lane < nr ? a.x[T.x0 + i0 + lane] : AccT(0);
    for (int i = 8 * wave; i < nr; i += 32) {
      u32x4 r[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (act && i + u < nr) r[u] = ld16(p + (size_t)(i0 + i + u) * rstride);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i + u < nr) {                           // uniform across the wave
          const AccT xi = bcast(xv, i + u);
          if (act) axpy_group<AccT, DT>(r[u], xi, acc);
        }
    }
  }
#pragma unroll
  for (int c = 0; c < G; ++c) red[(wave * 64 + lane) * G + c] = acc[c];
  __syncthreads();
  if (wave == 0 && act) {
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const int32_t d = a.dst[T.dst_off + lane * G + c];
      if (d >= 0)
        a.part[d] = (red[lane * G + c] + red[(64 + lane) * G + c]) +
                    (red[(128 + lane) * G + c] + red[(192 + lane) * G + c]);
    }
  }
}

// A whole workgroup on tile ti (it synchronizes).  red: 4 * 64 * 8 values
// (four waves x 64 lanes x at most 8 columns per lane).
template <typename AccT>
__device__ __forceinline__ void col_tile_any(const ColArgs<AccT>& a, int64_t ti, AccT* red) {
  const ColTile T = a.tiles[ti];
  switch (T.dtype) {
    case HM_F64:
      if constexpr (sizeof(AccT) == 8) col_tile<AccT, HM_F64>(a, T, red);
      break;
    case HM_F32: col_tile<AccT, HM_F32>(a, T, red); break;
    case HM_F16: col_tile<AccT, HM_F16>(a, T, red); break;
    default: col_tile<AccT, HM_BF16>(a, T, red); break;
  }
}

// ---------------------------------------------------------------- reduction

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
  const TBlock B = a.tb[a.owner[o]];
  const int l = (int)(o - B.toff);
  AccT s = AccT(0);
  for (int j = 0; j < B.nseg; ++j) s += a.part[B.pst + (int64_t)j * B.k + l];
  a.t[o] = a.sigma ? s * a.sigma[o] : s;
}

// ---------------------------------------------------------------- row panels

// Work items.  A plain launch has one workgroup per item; a persistent one
// has a fixed grid whose workgroup b takes items b, b + grid, b + 2 grid, ...
// in the same item order (a persistent grid is a multiple of 8, so every item
// keeps the XCD its index maps to).  The sums of an item do not depend on the
// workgroup that runs it.
//
// Item -> row panel.  order != nullptr: the plan's largest-first list.
// order == nullptr: cluster order cut into 8 contiguous ranges, one per XCD
// (workgroups are dispatched to the 8 XCDs round-robin), so neighbouring
// panels, which share most sources, run under the same L2.  Returns -1 for
// the padding items of that mapping.
__device__ __forceinline__ int panel_of(const int32_t* order, int64_t n_panels, int64_t it) {
  if (order) return order[it];
  const int64_t per = (n_panels + 7) / 8;
  const int64_t p = (it & 7) * per + (it >> 3);
  return p < n_panels ? (int)p : -1;
}

// Items of a row-panel launch under panel_of.
inline int64_t panel_items(bool xcd, int64_t n_panels) {
  return xcd ? 8 * ((n_panels + 7) / 8) : n_panels;
}

// Grid of a launch over n_items: one workgroup per item, or with persist > 0
// at most persist workgroups per CU, rounded down to a multiple of 8.
inline unsigned item_grid(int64_t n_items, int persist, int n_cu) {
  if (persist <= 0) return (unsigned)n_items;
  const int64_t cap = std::max<int64_t>(8, (int64_t)persist * n_cu / 8 * 8);
  return (unsigned)std::min<int64_t>(n_items, cap);
}

template <typename AccT>
struct RowArgs {
  const uint8_t* store;
  const RowPanel* rp;
  const RowSection* rs;
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
  // U groups per wave in flight, all loads issued before the arithmetic
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

// Sections [q_begin, q_end) of row panel P (source slots [s_begin, s_end)):
// sources staged in LDS by chunks of CAP slots, four waves stream the groups,
// a fixed-order LDS reduction, then one update of the panel's rows of y.
// Called by whole workgroups (it synchronizes).
template <typename AccT, int CAP, int U>
__device__ __forceinline__ void row_panel_part(const RowArgs<AccT>& a, const RowPanel& P,
                                               int q_begin, int q_end, int s_begin, int s_end,
                                               AccT* zs, AccT (*red)[64]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  AccT acc = AccT(0);
  const int32_t* src = a.src + P.src_off;
  for (int c_lo = s_begin; c_lo < s_end; c_lo += CAP) {
    const int c_hi = min(s_end, c_lo + CAP);
    for (int c = c_lo + tid; c < c_hi; c += 256) {
      const int s = src[c];
      zs[c - c_lo] = s < a.n_cols ? a.x[s] : a.t[s - a.n_cols];
    }
    __syncthreads();
    if (lane < P.m) {
      for (int q = q_begin; q < q_end; ++q) {
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

// First source slot of the U sections of a panel (= end of its dense slots).
template <typename AccT>
__device__ __forceinline__ int dense_slot_end(const RowArgs<AccT>& a, const RowPanel& P) {
  return P.nsec_dense < P.nsec ? a.rs[P.sec0 + P.nsec_dense].col0 : P.ncols;
}

// Phase 1: the dense parts of the row panels and the column tiles in one
// grouped launch.  Entry >= 0: a row panel; entry < 0: column tile -entry-1.
template <typename AccT, int CAP, int U>
__global__ __launch_bounds__(256) void k_p1(RowArgs<AccT> ra, ColArgs<AccT> ca, const int32_t* order,
                                            int64_t n_items) {
  static_assert(CAP >= 4 * 64 * 8, "staging buffer doubles as the tile reduction buffer");
  __shared__ AccT zs[CAP];
  __shared__ AccT red[4][64];
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    if (it != blockIdx.x) __syncthreads();          // LDS of the previous item
    const int item = order[it];
    if (item >= 0) {
      const RowPanel P = ra.rp[item];
      row_panel_part<AccT, CAP, U>(ra, P, 0, P.nsec_dense, 0, dense_slot_end(ra, P), zs, red);
    } else {
      col_tile_any<AccT>(ca, -(int64_t)item - 1, zs);
    }
  }
}

// Phase 2: the U sections of the row panels (after t is complete).
template <typename AccT, int CAP, int U>
__global__ __launch_bounds__(256) void k_p2(RowArgs<AccT> ra, const int32_t* order, int64_t n_items) {
  __shared__ AccT zs[CAP];
  __shared__ AccT red[4][64];
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    if (it != blockIdx.x) __syncthreads();
    const RowPanel P = ra.rp[order[it]];
    row_panel_part<AccT, CAP, U>(ra, P, P.nsec_dense, P.nsec, dense_slot_end(ra, P), P.ncols, zs, red);
  }
}

// Schedule 0: all column tiles (one per workgroup item), then whole row
// panels (dense and U sections in one pass).
template <typename AccT>
__global__ __launch_bounds__(256) void k_col(ColArgs<AccT> ca) {
  __shared__ AccT cred[4 * 64 * 8];
  for (int64_t it = blockIdx.x; it < ca.n_tiles; it += gridDim.x) {
    if (it != blockIdx.x) __syncthreads();
    col_tile_any<AccT>(ca, it, cred);
  }
}

template <typename AccT, int CAP, int U>
__global__ __launch_bounds__(256) void k_row(RowArgs<AccT> ra, const int32_t* order, int64_t n_panels,
                                             int64_t n_items) {
  __shared__ AccT zs[CAP];
  __shared__ AccT red[4][64];
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int pi = panel_of(order, n_panels, it);
    if (pi < 0) continue;                           // uniform: whole workgroup
    __syncthreads();                                // LDS of the previous item
    const RowPanel P = ra.rp[pi];
    row_panel_part<AccT, CAP, U>(ra, P, 0, P.nsec, 0, P.ncols, zs, red);
  }
}

// Streaming-read probe: reads n16 16-byte words with the same loads the
// kernels use; out[0] is written only if a thread's xor of what it read
// equals one fixed value, which keeps the loads live.
__global__ __launch_bounds__(256) void k_stream_read(const u32x4* __restrict__ p, int64_t n16,
                                                     unsigned* __restrict__ out) {
  u32x4 acc = (u32x4)(0u);
  const int64_t stride = (int64_t)gridDim.x * 256 * 8;
  for (int64_t i = ((int64_t)blockIdx.x * 256 * 8) + threadIdx.x; i < n16; i += stride) {
    u32x4 r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i + 256 * u < n16) r[u] = ld16(p + i + 256 * u);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i + 256 * u < n16) acc ^= r[u];
  }
  const unsigned v = acc[0] ^ acc[1] ^ acc[2] ^ acc[3];
  if (v == 0x9e3779b9u) out[0] = v;
}

// ================================================================ batch (MFMA)
//
// Several right-hand sides with FP32 accumulation on v_mfma_f32_32x32x1_2b_f32.
// In that instruction lane l supplies A_b[l%32][0] and B_b[0][l%32] of block
// b = l/32, and result D_b[i][j] sits in lane j + 32*((i/4)%2), register
// 16*b + 4*(i/8) + i%4.  With the row panels' lane = row layout a lane's
// panel value is exactly its A operand (block 0 = rows 0-31, block 1 = rows
// 32-63) and the B operand is one value of the source row z[k][0..31] per
// lane; the column tiles use the same instruction with rows and columns
// exchanged (A = four columns of V per lane).  Right-hand sides go 32 at a
// time; every result column depends only on its own right-hand side, so a
// column's result is the same whatever else is in the batch.

typedef float f32x32 __attribute__((ext_vector_type(32)));

__device__ __forceinline__ f32x32 mfma32(float a, float b, f32x32 c) {
  return __builtin_amdgcn_mfma_f32_32x32x1f32(a, b, c, 0, 0, 0);
}

// Row (0..63) of the 64-row A operand held by result register v of lane l.
__device__ __forceinline__ int mfma_row(int lane, int v) {
  return 32 * (v >> 4) + 8 * ((v & 15) >> 2) + 4 * (lane >> 5) + (v & 3);
}

// X (column-major, leading dimension ldx) -> Xr (n x RS row-major, zero-padded).
__global__ __launch_bounds__(256) void k_xpose(const float* __restrict__ X, int64_t ldx, int n,
                                               int nrhs, int RS, float* __restrict__ Xr) {
  __shared__ float tile[32][65];
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 32, t = threadIdx.x;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = t & 63, j = (t >> 6) + 4 * u;
    const int gi = i0 + i, gj = j0 + j;
    tile[j][i] = (gi < n && gj < nrhs) ? X[(size_t)gj * ldx + gi] : 0.f;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int j = t & 31, i = (t >> 5) + 8 * u;
    const int gi = i0 + i;
    if (gi < n) Xr[(size_t)gi * RS + j0 + j] = tile[j][i];
  }
}

// Two consecutive stored values (8 bytes of FP32, 4 bytes of FP16/BF16) as floats.
template <int DT>
__device__ __forceinline__ void load2(const uint8_t* p, float (&v)[2]) {
  if constexpr (DT == HM_F32) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const f32x2 r = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(p));
    v[0] = r[0]; v[1] = r[1];
  } else {
    const unsigned r = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p));
    if constexpr (DT == HM_F16) {
      typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
      const f16x2 h = __builtin_bit_cast(f16x2, r);
      v[0] = (float)h[0]; v[1] = (float)h[1];
    } else {
      v[0] = __uint_as_float(r << 16); v[1] = __uint_as_float(r & 0xffff0000u);
    }
  }
}

struct ColBArgs {
  const uint8_t* store;
  const ColTile* tiles;
  const int32_t* dst;
  const float* xr;
  float* part;
  int64_t n_tiles;
  int RS, RH;
};

// One wave: 128 columns [c0, c0 + 128) of a column tile (lane l owns columns
// c0 + 2l and c0 + 2l + 1) for 32 right-hand sides (group rh of RS).
// wd: this wave's 128-entry LDS table of destination indices.
template <int DT>
__device__ __forceinline__ void colb_part(const ColBArgs& a, const ColTile& T, int c0, int rh,
                                          int lane, int32_t* wd) {
  constexpr int SZ = dtype_size(DT);
  const int ncols = T.ngroups * group_width(DT);
  const int cb = c0 + 2 * lane;
  const bool act = cb < ncols;
  // each lane fetches the destinations of its own two columns once
  int32_t d0 = -1, d1 = -1;
  if (act) { d0 = a.dst[T.dst_off + cb]; d1 = a.dst[T.dst_off + cb + 1]; }
  wd[2 * lane] = d0;
  wd[2 * lane + 1] = d1;
  __builtin_amdgcn_wave_barrier();
  f32x32 acc[2];
  acc[0] = (f32x32)(0.f);
  acc[1] = (f32x32)(0.f);
  const uint8_t* base = a.store + T.data_off + (size_t)cb * SZ;
  const size_t rstride = (size_t)T.ld * SZ;
  const float* xb = a.xr + (size_t)T.x0 * a.RS + rh * 32 + (lane & 31);
  int i = 0;
  for (; i + 8 <= T.nrows; i += 8) {
    float v[8][2];
    float b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      v[u][0] = v[u][1] = 0.f;
      if (act) load2<DT>(base + (i + u) * rstride, v[u]);
      b[u] = xb[(size_t)(i + u) * a.RS];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      acc[0] = mfma32(v[u][0], b[u], acc[0]);
      acc[1] = mfma32(v[u][1], b[u], acc[1]);
    }
  }
  for (; i < T.nrows; ++i) {
    float v[2] = {0.f, 0.f};
    if (act) load2<DT>(base + i * rstride, v);
    const float b = xb[(size_t)i * a.RS];
    acc[0] = mfma32(v[0], b, acc[0]);
    acc[1] = mfma32(v[1], b, acc[1]);
  }
  const int j = rh * 32 + (lane & 31);
#pragma unroll
  for (int v = 0; v < 32; ++v) {
    const int R = mfma_row(lane, v);
    const int32_t e0 = wd[2 * R], e1 = wd[2 * R + 1];   // -1: padding or no column
    if (e0 >= 0) a.part[(size_t)e0 * a.RS + j] = acc[0][v];
    if (e1 >= 0) a.part[(size_t)e1 * a.RS + j] = acc[1][v];
  }
}

// Wave w -> (tile, 128-column part, right-hand-side group).
__global__ __launch_bounds__(256) void k_col_b(ColBArgs a) {
  __shared__ int32_t sdst[4][128];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t w = (int64_t)blockIdx.x * 4 + wave;
  const int rh = (int)(w % a.RH);
  const int64_t rest = w / a.RH;
  const int part = (int)(rest & 3);
  const int64_t ti = rest >> 2;
  if (ti >= a.n_tiles) return;
  const ColTile T = a.tiles[ti];
  const int c0 = 128 * part;
  if (c0 >= T.ngroups * group_width(T.dtype)) return;
  switch (T.dtype) {
    case HM_F32: colb_part<HM_F32>(a, T, c0, rh, lane, sdst[wave]); break;
    case HM_F16: colb_part<HM_F16>(a, T, c0, rh, lane, sdst[wave]); break;
    case HM_BF16: colb_part<HM_BF16>(a, T, c0, rh, lane, sdst[wave]); break;
    default: break;
  }
}

struct RedBArgs {
  const TBlock* tb;
  const int32_t* owner;
  const float* sigma;
  const float* part;
  float* t;
  int64_t n_t;
  int RS;
};

// t[o][j] = s_o * sum over the block's intervals (ascending) of its partials.
__global__ __launch_bounds__(256) void k_reduce_b(RedBArgs a) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t o = e / a.RS;
  const int j = (int)(e % a.RS);
  if (o >= a.n_t) return;
  const TBlock B = a.tb[a.owner[o]];
  const int l = (int)(o - B.toff);
  float s = 0.f;
  const float* pp = a.part + ((size_t)B.pst + l) * a.RS + j;
  const size_t step = (size_t)B.k * a.RS;
#pragma unroll 4
  for (int g = 0; g < B.nseg; ++g) s += pp[g * step];
  a.t[o * a.RS + j] = a.sigma ? s * a.sigma[o] : s;
}

struct RowBArgs {
  const uint8_t* store;
  const RowPanel* rp;
  const RowSection* rs;
  const int32_t* order;      // nullptr: XCD-contiguous cluster order
  int64_t n_panels;
  const int32_t* src;
  const float* xr;
  const float* t;
  float* Y;
  int64_t ldy;
  float alpha;
  int32_t n_cols, nrhs;
};

template <int DT>
__device__ __forceinline__ void decode_group(u32x4 r, float* v) {
  if constexpr (DT == HM_F32) {
    const f32x4 f = __builtin_bit_cast(f32x4, r);
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = f[c];
  } else if constexpr (DT == HM_F16) {
    const f16x8 h = __builtin_bit_cast(f16x8, r);
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = (float)h[c];
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      v[2 * c] = __uint_as_float(r[c] << 16);
      v[2 * c + 1] = __uint_as_float(r[c] & 0xffff0000u);
    }
  }
}

// Groups g_lo + wave, + 4, ... of one section; U groups per step with the
// next step's loads issued before this step's matrix-core work.
template <int NH, int DT>
__device__ __forceinline__ void rowb_section(const RowBArgs& a, const RowSection& S, int m,
                                             int g_lo, int g_hi, const float* zs, int lane,
                                             int wave, f32x32 (&acc)[NH]) {
  constexpr int G = group_width(DT), RS = 32 * NH, U = 4;
  const u32x4* p = reinterpret_cast<const u32x4*>(a.store + S.data_off) + lane;
  const bool act = lane < m;
  u32x4 nxt[U];
  int g = g_lo + wave;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int gg = g + 4 * u;
    nxt[u] = (act && gg < g_hi) ? ld16(p + (size_t)gg * m) : (u32x4)(0u);
  }
  for (; g < g_hi; g += 4 * U) {
    u32x4 cur[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cur[u] = nxt[u];
      const int gg = g + 4 * (u + U);
      nxt[u] = (act && gg < g_hi) ? ld16(p + (size_t)gg * m) : (u32x4)(0u);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int gg = g + 4 * u;
      if (gg >= g_hi) break;                    // uniform across the wave
      float v[G];
      decode_group<DT>(cur[u], v);
      const float* zrow = zs + (size_t)gg * G * RS + (lane & 31);
#pragma unroll
      for (int c = 0; c < G; ++c)
#pragma unroll
        for (int h = 0; h < NH; ++h) acc[h] = mfma32(v[c], zrow[c * RS + 32 * h], acc[h]);
    }
  }
}

template <int NH>
__global__ __launch_bounds__(256) void k_row_b(RowBArgs a) {
  extern __shared__ float lds[];
  // CAPB = 256 source columns per LDS chunk; TPC threads per column, CPP columns per pass
  constexpr int RS = 32 * NH, CAPB = 256, TPC = RS / 4, CPP = 256 / TPC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pi = panel_of(a.order, a.n_panels, blockIdx.x);
  if (pi < 0) return;                               // uniform: whole workgroup
  const RowPanel P = a.rp[pi];
  f32x32 acc[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) acc[h] = (f32x32)(0.f);
  const int32_t* src = a.src + P.src_off;
  for (int c_lo = 0; c_lo < P.ncols; c_lo += CAPB) {
    const int c_hi = min(P.ncols, c_lo + CAPB);
    // stage source rows: TPC threads per column, 16 bytes each; all loads of
    // a thread are issued before its LDS writes
    {
      constexpr int PASSES = CAPB / CPP;
      f32x4 val[PASSES];
      const int q = tid % TPC, cq = tid / TPC;
#pragma unroll
      for (int ps = 0; ps < PASSES; ++ps) {
        const int c = c_lo + ps * CPP + cq;
        val[ps] = (f32x4)(0.f);
        if (c < c_hi) {
          const int s = src[c];
          const float* row = s < a.n_cols ? a.xr + (size_t)s * RS : a.t + (size_t)(s - a.n_cols) * RS;
          val[ps] = *reinterpret_cast<const f32x4*>(row + 4 * q);
        }
      }
#pragma unroll
      for (int ps = 0; ps < PASSES; ++ps) {
        const int c = c_lo + ps * CPP + cq;
        if (c < c_hi) *reinterpret_cast<f32x4*>(lds + (size_t)(c - c_lo) * RS + 4 * q) = val[ps];
      }
    }
    __syncthreads();
    for (int qs = 0; qs < P.nsec; ++qs) {
      const RowSection S = a.rs[P.sec0 + qs];
      const int G = group_width(S.dtype);
      const int g_lo = max(0, c_lo - S.col0) / G;
      const int g_hi = min(S.ngroups, max(0, c_hi - S.col0) / G);
      if (g_hi <= g_lo) continue;
      const float* z = lds + (ptrdiff_t)(S.col0 - c_lo) * RS;
      switch (S.dtype) {
        case HM_F32: rowb_section<NH, HM_F32>(a, S, P.m, g_lo, g_hi, z, lane, wave, acc); break;
        case HM_F16: rowb_section<NH, HM_F16>(a, S, P.m, g_lo, g_hi, z, lane, wave, acc); break;
        case HM_BF16: rowb_section<NH, HM_BF16>(a, S, P.m, g_lo, g_hi, z, lane, wave, acc); break;
        default: break;
      }
    }
    __syncthreads();
  }
  // fixed-order reduction of the four waves through LDS, then one update of Y
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int v = 0; v < 32; ++v)
      lds[(size_t)(wave * 64 + mfma_row(lane, v)) * RS + h * 32 + (lane & 31)] = acc[h][v];
  __syncthreads();
  for (int e = tid; e < 64 * RS; e += 256) {
    const int R = e & 63, j = e >> 6;
    if (R < P.m && j < a.nrhs) {
      const float s = (lds[(size_t)R * RS + j] + lds[(size_t)(64 + R) * RS + j]) +
                      (lds[(size_t)(128 + R) * RS + j] + lds[(size_t)(192 + R) * RS + j]);
      float* yp = a.Y + (size_t)j * a.ldy + P.row0 + R;
      *yp += a.alpha * s;
    }
  }
}

// ---------------------------------------------------------------- launch

template <typename AccT, int U>
hipError_t launch_typed_u(const hm_matrix& A, double alpha, const void* x, void* y, void* work,
                          hipStream_t s, hipEvent_t* ev) {
  const StoreHeader& h = A.hdr;
  const uint8_t* st = A.d_store;
  AccT* part = reinterpret_cast<AccT*>(work);
  AccT* t = reinterpret_cast<AccT*>(reinterpret_cast<uint8_t*>(work) + A.work_t_off);
  constexpr int CAP = 16384 / sizeof(AccT);
  RowArgs<AccT> ra{st,
                   reinterpret_cast<const RowPanel*>(st + h.off_row_panels),
                   reinterpret_cast<const RowSection*>(st + h.off_row_sections),
                   reinterpret_cast<const int32_t*>(st + h.off_row_src),
                   reinterpret_cast<const AccT*>(x), t, reinterpret_cast<AccT*>(y), (AccT)alpha,
                   (int32_t)h.n_cols};
  ColArgs<AccT> ca{st, reinterpret_cast<const ColTile*>(st + h.off_col_tiles),
                   reinterpret_cast<const int32_t*>(st + h.off_col_dst),
                   reinterpret_cast<const AccT*>(x), part, h.n_col_tiles};
  const bool grouped = A.launch.schedule == 1;
  const int ps = A.launch.persist, ncu = A.n_cu;
  if (ev) (void)hipEventRecord(ev[0], s);
  if (grouped) {
    if (h.n_p1 > 0)
      hipLaunchKernelGGL((k_p1<AccT, CAP, U>), dim3(item_grid(h.n_p1, ps, ncu)), dim3(256), 0, s, ra,
                         ca, reinterpret_cast<const int32_t*>(st + h.off_p1_order), h.n_p1);
  } else if (h.n_col_tiles > 0) {
    hipLaunchKernelGGL(k_col<AccT>, dim3(item_grid(h.n_col_tiles, ps, ncu)), dim3(256), 0, s, ca);
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  if (h.n_col_tiles > 0) {
    RedArgs<AccT> rd{reinterpret_cast<const TBlock*>(st + h.off_tblocks),
                     reinterpret_cast<const int32_t*>(st + h.off_owner),
                     h.has_sigma ? reinterpret_cast<const AccT*>(st + h.off_sigma) : nullptr,
                     part, t, h.n_large, h.n_large_t, h.n_t};
    const int64_t nred = h.n_large + (h.n_t - h.n_large_t + 255) / 256;
    if (nred > 0) hipLaunchKernelGGL(k_reduce<AccT>, dim3((unsigned)nred), dim3(256), 0, s, rd);
  }
  if (ev) (void)hipEventRecord(ev[2], s);
  if (grouped) {
    if (h.n_p2 > 0)
      hipLaunchKernelGGL((k_p2<AccT, CAP, U>), dim3(item_grid(h.n_p2, ps, ncu)), dim3(256), 0, s, ra,
                         reinterpret_cast<const int32_t*>(st + h.off_p2_order), h.n_p2);
  } else if (h.n_row_panels > 0) {
    const bool xcd = A.launch.order == 1;
    const int64_t items = panel_items(xcd, h.n_row_panels);
    hipLaunchKernelGGL((k_row<AccT, CAP, U>), dim3(item_grid(items, ps, ncu)), dim3(256), 0, s, ra,
                       xcd ? nullptr : reinterpret_cast<const int32_t*>(st + h.off_row_order),
                       h.n_row_panels, items);
  }
  if (ev) (void)hipEventRecord(ev[3], s);
  return hipGetLastError();
}

template <typename AccT>
hipError_t launch_typed(const hm_matrix& A, double alpha, const void* x, void* y, void* work,
                        hipStream_t s, hipEvent_t* ev) {
  return A.launch.row_unroll >= 8 ? launch_typed_u<AccT, 8>(A, alpha, x, y, work, s, ev)
                                  : launch_typed_u<AccT, 4>(A, alpha, x, y, work, s, ev);
}

}  // namespace

hipError_t launch_mvm(const hm_matrix& A, double alpha, const void* x, void* y, void* work,
                      hipStream_t s, hipEvent_t* ev, bool profile) {
  if (profile && !ev && A.prof.on && A.prof.calls < A.prof.max_calls)
    ev = &A.prof.ev[4 * (size_t)A.prof.calls++];
  return A.acc_dtype == HM_F64 ? launch_typed<double>(A, alpha, x, y, work, s, ev)
                               : launch_typed<float>(A, alpha, x, y, work, s, ev);
}

hipError_t launch_stream_read(const void* buf, size_t bytes, void* out, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  const int64_t per_block = 256 * 8;
  const int64_t blocks = std::min<int64_t>((n16 + per_block - 1) / per_block, 256 * 16);
  hipLaunchKernelGGL(k_stream_read, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s,
                     static_cast<const u32x4*>(buf), n16, static_cast<unsigned*>(out));
  return hipGetLastError();
}

hipError_t launch_mvm_batch(const hm_matrix& A, int nrhs, double alpha, const void* X, int64_t ldx,
                            void* Y, int64_t ldy, void* work, hipStream_t s, bool profile) {
  const StoreHeader& h = A.hdr;
  if (A.acc_dtype == HM_F64) {
    for (int c = 0; c < nrhs; ++c) {
      hipError_t e = launch_mvm(A, alpha, static_cast<const uint8_t*>(X) + (size_t)c * ldx * 8,
                                static_cast<uint8_t*>(Y) + (size_t)c * ldy * 8, work, s, nullptr, profile);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  hipEvent_t* ev = nullptr;
  if (profile && A.prof.on && A.prof.calls < A.prof.max_calls) ev = &A.prof.ev[4 * (size_t)A.prof.calls++];
  const uint8_t* st = A.d_store;
  uint8_t* w = static_cast<uint8_t*>(work);
  for (int r0 = 0; r0 < nrhs; r0 += 64) {
    const int nr = min(64, nrhs - r0);
    const int RS = nr <= 32 ? 32 : 64, RH = RS / 32;
    float* part = reinterpret_cast<float*>(w);
    float* t = reinterpret_cast<float*>(w + (size_t)RS * A.work_part_bytes);
    float* xr = reinterpret_cast<float*>(w + (size_t)RS * (A.work_part_bytes + A.work_t_bytes));
    const float* Xc = static_cast<const float*>(X) + (size_t)r0 * ldx;
    float* Yc = static_cast<float*>(Y) + (size_t)r0 * ldy;
    if (ev && r0 == 0) (void)hipEventRecord(ev[0], s);
    hipLaunchKernelGGL(k_xpose, dim3((unsigned)((h.n_cols + 63) / 64), (unsigned)RH), dim3(256), 0, s,
                       Xc, ldx, (int)h.n_cols, nr, RS, xr);
    if (h.n_col_tiles > 0) {
      ColBArgs ca{st, reinterpret_cast<const ColTile*>(st + h.off_col_tiles),
                  reinterpret_cast<const int32_t*>(st + h.off_col_dst), xr, part, h.n_col_tiles, RS, RH};
      const int64_t waves = h.n_col_tiles * 4 * RH;
      hipLaunchKernelGGL(k_col_b, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, ca);
      if (ev && r0 == 0) (void)hipEventRecord(ev[1], s);
      RedBArgs rb{reinterpret_cast<const TBlock*>(st + h.off_tblocks),
                  reinterpret_cast<const int32_t*>(st + h.off_owner),
                  h.has_sigma ? reinterpret_cast<const float*>(st + h.off_sigma) : nullptr, part, t,
                  h.n_t, RS};
      const int64_t nthr = h.n_t * RS;
      if (nthr > 0) hipLaunchKernelGGL(k_reduce_b, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, rb);
    } else if (ev && r0 == 0) {
      (void)hipEventRecord(ev[1], s);
    }
    if (ev && r0 == 0) (void)hipEventRecord(ev[2], s);
    const bool xcd = A.launch.order == 1;
    RowBArgs ra{st,
                reinterpret_cast<const RowPanel*>(st + h.off_row_panels),
                reinterpret_cast<const RowSection*>(st + h.off_row_sections),
                xcd ? nullptr : reinterpret_cast<const int32_t*>(st + h.off_row_order), h.n_row_panels,
                reinterpret_cast<const int32_t*>(st + h.off_row_src),
                xr, t, Yc, ldy, (float)alpha, (int32_t)h.n_cols, nr};
    // 256 rows of RS floats: the 256-column source chunk, reused for the
    // 4 waves x 64 rows reduction
    const size_t lds = (size_t)RS * 256 * sizeof(float);
    const unsigned grid = (unsigned)panel_items(xcd, h.n_row_panels);
    if (RH == 1)
      hipLaunchKernelGGL(k_row_b<1>, dim3(grid), dim3(256), lds, s, ra);
    else
      hipLaunchKernelGGL(k_row_b<2>, dim3(grid), dim3(256), lds, s, ra);
  }
  if (ev) (void)hipEventRecord(ev[3], s);
  return hipGetLastError();
}

}  // namespace hm
