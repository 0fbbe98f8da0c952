// HIP kernels (gfx950) of the product with several right-hand sides and
// FP32 accumulation, on the matrix cores, and their launcher (hm_mvm_batch).
//
// The same packed store as the single-right-hand-side path (hm_layout.hpp):
//  k_xpose    X (column-major) -> row-major source rows of 32 or 64 values;
//  k_col_b    far field, phase 1: column tiles as MFMA tiles, partial
//             products per column chunk;
//  k_reduce_b t_b = s_b * (sum of the partials in chunk order) per column;
//  k_row_b    near field and far field, phase 2: row panels as the A operand
//             of v_mfma_f32_32x32x1_2b_f32, sources staged in LDS, a
//             fixed-order four-wave reduction, one update of Y per row.
// Every sum has a fixed order, so results are bitwise reproducible and do not
// depend on the other right-hand sides of the batch.

#include <algorithm>

#include <hip/hip_runtime.h>

#include "hm_internal.hpp"
#include "hm_device.hpp"

namespace hm {
namespace {

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

}  // namespace

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
