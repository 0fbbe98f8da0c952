// HIP kernels (gfx950) of the product with several right-hand sides and
// FP32 accumulation, on the matrix cores, and their launcher (hm_mvm_batch).
//
// The same packed store as the single-right-hand-side path (hm_layout.hpp):
//  k_xpose    X (column-major) -> row-major source rows of 32 or 64 values;
//  k_col_b    far field, phase 1: column tiles as MFMA tiles, partial
//             products per column chunk;
//  k_reduce_b t_b = s_b * (sum of the partials in chunk order) per column;
//  k_row_b    near field and far field, phase 2: row panels in 16-row
//             blocks as the A operand of v_mfma_f32_16x16x4_f32 (sets of 4
//             columns transposed across the 16-lane groups by
//             v_permlane32_swap / v_permlane16_swap), source rows as the B
//             operand straight from memory, a fixed-order four-wave
//             reduction, one update of Y per row.
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
// Several right-hand sides with FP32 accumulation on the matrix cores:
// v_mfma_f32_32x32x2_f32 (FP32 column tiles) and v_mfma_f32_16x16x4_f32
// (16-bit and multi-format column tiles; row panels).  Operand
// and result layouts are stated beside the wrappers below.  Right-hand
// sides go 32 at a time; every result column depends only on its own
// right-hand side, so a column's result is the same whatever else is in the
// batch.

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

typedef float f32x16 __attribute__((ext_vector_type(16)));

// D (32 x 32) += A (32 x 2) B (2 x 32) on v_mfma_f32_32x32x2_f32: lane l
// gives A[l % 32][l / 32] and B[l / 32][l % 32]; D[i][j] is in lane
// j + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4.
__device__ __forceinline__ f32x16 mfma32x2(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Row (0..31) of D held by register v of lane l in mfma32x2.
__device__ __forceinline__ int mfma32x2_row(int lane, int v) {
  return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
}

struct ColBArgs {
  const uint8_t* store;
  const ColTile* tiles;
  const int32_t* dst;
  const float* xr;
  float* part;            // rows of RS values; t follows at row t_row0
  int32_t t_row0;         // column sums of blocks inside one chunk go to row t_row0 + o
  const float* sigma;     // nullptr when no block keeps singular values
  int64_t n_tiles;
  int RS, RH;
};

// The 8 bytes at p as floats: 2 FP32 values (v[2], v[3] = 0) or 4 FP16 or
// BF16 values.
__device__ __forceinline__ void load_slot(const uint8_t* p, int dt, float (&v)[4]) {
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  const u32x2 r = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
  if (dt == HM_F32) {
    v[0] = __uint_as_float(r[0]);
    v[1] = __uint_as_float(r[1]);
    v[2] = v[3] = 0.f;
  } else if (dt == HM_F16) {
    typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
    const f16x4 h = __builtin_bit_cast(f16x4, r);
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = (float)h[c];
  } else {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      v[2 * c] = __uint_as_float(r[c] << 16);
      v[2 * c + 1] = __uint_as_float(r[c] & 0xffff0000u);
    }
  }
}

// One wave (a workgroup of its own): slots [32 quarter, 32 quarter + 32) of
// a column tile for 32 right-hand sides (group rh of RS).  Slot s is bytes
// [8 s, 8 s + 8) of every tile row: half of group s / 2, i.e. 2 FP32 or 4
// FP16/BF16 columns.  Lane l owns slot 32 quarter + l % 32 of row i + l / 32:
// one v_mfma_f32_32x32x2_f32 per column q < CPL of the slot takes two rows
// at a time (A: the lane's value of column q; B: the x rows i and i + 1 of
// the 32 right-hand sides, one load for both).  DT >= 0: every slot has
// format DT (CPL = its columns per slot); DT < 0: the tile holds runs of
// several formats, CPL = 4 and an FP32 slot leaves columns 2 and 3 empty.
// Rows go in batches of S steps (2S rows); the next batch's loads are in
// flight while this batch's MFMAs run.  wd, ws: the wave's LDS tables of
// destination rows (in part, whose rows from t_row0 on are t) and factors
// (s_b[l] for a column that writes t directly, else 1).
template <int DT, int S>
__device__ __forceinline__ void colb32_part(const ColBArgs& a, const ColTile& T, int quarter, int rh,
                                          int lane, int32_t* wd, float* ws) {
  constexpr int CPL = DT == HM_F32 ? 2 : 4;
  const int l32 = lane & 31, hi = lane >> 5;
  const int sl = 32 * quarter + l32;
  const bool act = sl < 2 * T.ngroups;
  int dt, cps, col;                                  // format, columns, first tile column of the slot
  if constexpr (DT >= 0) {
    dt = DT;
    cps = CPL;
    col = sl * CPL;
  } else {
    const TileGroup tg = tile_group(T, act ? sl / 2 : 0);
    dt = tg.dtype;
    cps = group_width(dt) / 2;
    col = tg.col + (sl % 2) * cps;
  }
  f32x16 acc[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q] = (f32x16)(0.f);
  const size_t rstride = (size_t)T.ngroups * 16;
  // row 0 of the lane's slot (slot 0 for a lane past the tile's slots)
  const uint8_t* base = a.store + T.data_off + (size_t)(act ? sl : 0) * 8;
  const float* xb = a.xr + (size_t)T.x0 * a.RS + rh * 32 + l32;
  const int nr = T.nrows;
  // step k covers rows 2k, 2k + 1; lanes of a missing row give zeros
  const int nsteps = (nr + 1) / 2;
  // Loads without branches (for one-format tiles): a row past the tile
  // reads its last row and a lane past its slots reads slot 0.  At use, the
  // x value of a row past the tile is replaced by zero, so its products add
  // nothing; a lane past the slots fills only result rows that are never
  // written.  (Masking at use, not at load, keeps the loads in flight.)
  // Two buffers of S steps take turns: while one batch's MFMAs run, the
  // next batch's loads are in flight into the other; the loop body has no
  // branch, so the accumulators stay in their registers.
  float a0[S][4], b0[S], a1[S][4], b1[S];
  auto issue = [&](int k0, float (&an)[S][4], float (&bn)[S]) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const int rc = min(2 * (k0 + u) + hi, nr - 1);
      load_slot(base + (size_t)rc * rstride, dt, an[u]);
      bn[u] = xb[(size_t)rc * a.RS];
    }
  };
  auto compute = [&](int k0, const float (&an)[S][4], const float (&bn)[S]) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const float b = 2 * (k0 + u) + hi < nr ? bn[u] : 0.f;
#pragma unroll
      for (int q = 0; q < CPL; ++q) acc[q] = mfma32x2(an[u][q], b, acc[q]);
    }
  };
  // the first loads of the tile and the destinations of the lane's columns
  // go out together; the factors and the LDS tables follow the main loop
  issue(0, a0, b0);
  int32_t e[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) e[q] = (lane < 32 && act && q < cps) ? a.dst[T.dst_off + col + q] : kDstPad;
  for (int k = 0; k < nsteps; k += 2 * S) {
    issue(k + S, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    compute(k, a0, b0);
    issue(k + 2 * S, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    compute(k + S, a1, b1);
  }
  if (lane < 32) {
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      // row of part (partials, then t) the column's sum goes to, and its factor
      const bool direct = e[q] <= -2;
      wd[CPL * lane + q] = direct ? a.t_row0 + dst_t_index(e[q]) : e[q];
      ws[CPL * lane + q] = (direct && a.sigma) ? a.sigma[dst_t_index(e[q])] : 1.f;
    }
  }
  __builtin_amdgcn_wave_barrier();
  const int j = rh * 32 + l32;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int slot = mfma32x2_row(lane, v);         // the slot (D row) of this result
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int32_t e = wd[CPL * slot + q];          // -1: padding or no column
      if (e >= 0) a.part[(size_t)e * a.RS + j] = acc[q][v] * ws[CPL * slot + q];
    }
  }
}

// One wave (a workgroup of its own): groups [32 half, 32 half + 32) of an
// FP32 column tile for 32 right-hand sides (group rh of RS).  Lane l owns
// group 32 half + l % 32 of row 2k + l / 32 in step k: one 16-byte load
// brings its 4 columns, and one v_mfma_f32_32x32x2_f32 per column q takes
// two rows at a time (A: the lane's value of column q; B: the x rows 2k and
// 2k + 1 of the 32 right-hand sides, one load for both); D_q row i is
// column 4 i + q of the half.  Against colb32_part each load is twice as
// wide, so a wave keeps twice the bytes in flight.  Rows go in batches of S
// steps, the next batch's loads in flight while this batch's MFMAs run.  wd,
// ws: the wave's LDS tables of destination rows and factors (128 columns).
template <int S>
__device__ __forceinline__ void colb32g_part(const ColBArgs& a, const ColTile& T, int half, int rh, int lane,
                                            int32_t* wd, float* ws) {
  const int l32 = lane & 31, hi = lane >> 5;
  const int g = 32 * half + l32;
  const bool act = g < T.ngroups;
  f32x16 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = (f32x16)(0.f);
  // row 0 of the lane's group (group 0 for a lane past the tile's groups)
  const u32x4* base = reinterpret_cast<const u32x4*>(a.store + T.data_off) + (act ? g : 0);
  const float* xb = a.xr + (size_t)T.x0 * a.RS + rh * 32 + l32;
  const int nr = T.nrows;
  const int nsteps = (nr + 1) / 2;
  // loads without branches, masked at use, in two buffers that take turns,
  // as in colb32_part
  f32x4 a0[S], a1[S];
  float b0[S], b1[S];
  auto issue = [&](int k0, f32x4 (&an)[S], float (&bn)[S]) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const int rc = min(2 * (k0 + u) + hi, nr - 1);
      an[u] = __builtin_bit_cast(f32x4, ld16(base + (size_t)rc * T.ngroups));
      bn[u] = xb[(size_t)rc * a.RS];
    }
  };
  auto compute = [&](int k0, const f32x4 (&an)[S], const float (&bn)[S]) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const float b = 2 * (k0 + u) + hi < nr ? bn[u] : 0.f;
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = mfma32x2(an[u][q], b, acc[q]);
    }
  };
  issue(0, a0, b0);
  int32_t e[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) e[q] = (lane < 32 && act) ? a.dst[T.dst_off + 4 * g + q] : kDstPad;
  for (int k = 0; k < nsteps; k += 2 * S) {
    issue(k + S, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    compute(k, a0, b0);
    issue(k + 2 * S, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    compute(k + S, a1, b1);
  }
  if (lane < 32) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool direct = e[q] <= -2;
      wd[4 * lane + q] = direct ? a.t_row0 + dst_t_index(e[q]) : e[q];
      ws[4 * lane + q] = (direct && a.sigma) ? a.sigma[dst_t_index(e[q])] : 1.f;
    }
  }
  __builtin_amdgcn_wave_barrier();
  const int j = rh * 32 + l32;
  // one column q at a time (the scheduler barrier keeps the LDS reads of
  // the tables from being hoisted for all 64 results at once)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = mfma32x2_row(lane, v);           // the group (D row) of this result
      const int32_t d = wd[4 * i + q];               // -1: padding or no column
      if (d >= 0) a.part[(size_t)d * a.RS + j] = acc[q][v] * ws[4 * i + q];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// D (16 x 16) += A (16 x 4) B (4 x 16) on v_mfma_f32_16x16x4_f32: lane l
// gives A[l % 16][l / 16] and B[l / 16][l % 16]; D[i][j] is in lane
// j + 16 (i / 4), register i % 4.
__device__ __forceinline__ f32x4 mfma16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// One wave (a workgroup of its own): slots [16 s16, 16 s16 + 16) of a column
// tile for 32 right-hand sides (group rh of RS).  Slot s is bytes [8 s, 8 s
// + 8) of every tile row: half of group s / 2, i.e. 2 FP32 or 4 FP16/BF16
// columns.  Lane l owns slot 16 s16 + l % 16 of row 4 k + l / 16 in step k:
// one v_mfma_f32_16x16x4_f32 per column q < CPL of the slot and per half of
// the 32 right-hand sides takes four rows at a time (A: the lane's value of
// column q; B: one value of the x rows 4k..4k+3 per lane, one load per
// half).  DT >= 0: every slot has format DT (CPL = its columns per slot);
// DT < 0: the tile holds runs of several formats, CPL = 4 and an FP32 slot
// leaves columns 2 and 3 empty.  Rows go in batches of S steps; the next
// batch's loads are in flight while this batch's MFMAs run.  wd, ws: the
// wave's LDS tables of destination rows (in part, whose rows from t_row0 on
// are t) and factors (s_b[l] for a column that writes t directly, else 1).
template <int DT, int S>
__device__ __forceinline__ void colb16_part(const ColBArgs& a, const ColTile& T, int s16, int rh,
                                          int lane, int32_t* wd, float* ws) {
  constexpr int CPL = DT == HM_F32 ? 2 : 4;
  const int l16 = lane & 15, kq = lane >> 4;
  const int sl = 16 * s16 + l16;
  const bool act = sl < 2 * T.ngroups;
  int dt, cps, col;                                  // format, columns, first tile column of the slot
  if constexpr (DT >= 0) {
    dt = DT;
    cps = CPL;
    col = sl * CPL;
  } else {
    const TileGroup tg = tile_group(T, act ? sl / 2 : 0);
    dt = tg.dtype;
    cps = group_width(dt) / 2;
    col = tg.col + (sl % 2) * cps;
  }
  f32x4 acc[CPL][2];
#pragma unroll
  for (int q = 0; q < CPL; ++q) acc[q][0] = acc[q][1] = (f32x4)(0.f);
  const size_t rstride = (size_t)T.ngroups * 16;
  // row 0 of the lane's slot (slot 0 for a lane past the tile's slots)
  const uint8_t* base = a.store + T.data_off + (size_t)(act ? sl : 0) * 8;
  const float* xb = a.xr + (size_t)T.x0 * a.RS + rh * 32 + l16;
  const int nr = T.nrows;
  // step k covers rows 4k .. 4k + 3; lanes of a missing row give zeros
  const int nsteps = (nr + 3) / 4;
  // loads without branches, masked at use, in two buffers that take turns,
  // as in colb32_part
  float a0[S][4], b0[S][2], a1[S][4], b1[S][2];
  auto issue = [&](int k0, float (&an)[S][4], float (&bn)[S][2]) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const int rc = min(4 * (k0 + u) + kq, nr - 1);
      load_slot(base + (size_t)rc * rstride, dt, an[u]);
      bn[u][0] = xb[(size_t)rc * a.RS];
      bn[u][1] = xb[(size_t)rc * a.RS + 16];
    }
  };
  auto compute = [&](int k0, const float (&an)[S][4], const float (&bn)[S][2]) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const bool ok = 4 * (k0 + u) + kq < nr;
#pragma unroll
      for (int q = 0; q < CPL; ++q)
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[q][h] = mfma16x4(an[u][q], ok ? bn[u][h] : 0.f, acc[q][h]);
    }
  };
  // the first loads of the tile and the destinations of the lane's columns
  // go out together; the factors and the LDS tables follow the main loop
  issue(0, a0, b0);
  int32_t e[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) e[q] = (lane < 16 && act && q < cps) ? a.dst[T.dst_off + col + q] : kDstPad;
  for (int k = 0; k < nsteps; k += 2 * S) {
    issue(k + S, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    compute(k, a0, b0);
    issue(k + 2 * S, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    compute(k + S, a1, b1);
  }
  if (lane < 16) {
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      // row of part (partials, then t) the column's sum goes to, and its factor
      const bool direct = e[q] <= -2;
      wd[CPL * lane + q] = direct ? a.t_row0 + dst_t_index(e[q]) : e[q];
      ws[CPL * lane + q] = (direct && a.sigma) ? a.sigma[dst_t_index(e[q])] : 1.f;
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int slot = 4 * kq + v;                    // the slot (D row) of acc[.][.][v]
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int32_t e2 = wd[CPL * slot + q];        // -1: padding or no column
      if (e2 >= 0) {
        float* out = a.part + (size_t)e2 * a.RS + rh * 32 + l16;
        const float f = ws[CPL * slot + q];
        out[0] = acc[q][0][v] * f;
        out[16] = acc[q][1][v] * f;
      }
    }
  }
}

// Column kernels: steps per batch of row loads (measured best).
constexpr int kColBSteps = 4;

// Workgroup (one wave) w -> (tile t0 + w / (4 RH), quarter of its slots,
// right-hand-side group) over the one-format FP32 tiles [t0, t1): 32 slots
// per wave, so each x row loaded serves the most columns.
template <int S>
__global__ __launch_bounds__(64) void k_col_b32(ColBArgs a, int64_t t0, int64_t t1) {
  __shared__ int32_t sdst[64];
  __shared__ float ssig[64];
  const int lane = threadIdx.x;
  const int64_t w = blockIdx.x;
  const int rh = (int)(w % a.RH);
  const int64_t rest = w / a.RH;
  const int quarter = (int)(rest & 3);
  const int64_t ti = t0 + (rest >> 2);
  if (ti >= t1) return;
  const ColTile T = a.tiles[ti];
  if (32 * quarter >= 2 * T.ngroups) return;         // uniform: nothing in this quarter
  colb32_part<HM_F32, S>(a, T, quarter, rh, lane, sdst, ssig);
}

// Workgroup (one wave) w -> (tile t0 + w / (2 RH), half of its groups,
// right-hand-side group) over the one-format FP32 tiles [t0, t1): 32
// 16-byte groups per wave (launch parameter colb = 1).
template <int S>
__global__ __launch_bounds__(64) void k_col_b32g(ColBArgs a, int64_t t0, int64_t t1) {
  __shared__ int32_t sdst[128];
  __shared__ float ssig[128];
  const int lane = threadIdx.x;
  const int64_t w = blockIdx.x;
  const int rh = (int)(w % a.RH);
  const int64_t rest = w / a.RH;
  const int half = (int)(rest & 1);
  const int64_t ti = t0 + (rest >> 1);
  if (ti >= t1) return;
  const ColTile T = a.tiles[ti];
  if (32 * half >= T.ngroups) return;                // uniform: nothing in this half
  colb32g_part<S>(a, T, half, rh, lane, sdst, ssig);
}

// Workgroup (one wave) w -> (tile t0 + w / (8 RH), sixteenth of its slots,
// right-hand-side group) over the tiles [t0, t1) of one class: one format
// DT, or DT < 0 for tiles with runs of several formats.  16 slots per wave
// halve the MFMA work lost on the partly filled last part of a narrow tile.
template <int DT>
__global__ __launch_bounds__(64) void k_col_b16(ColBArgs a, int64_t t0, int64_t t1) {
  __shared__ int32_t sdst[64];
  __shared__ float ssig[64];
  const int lane = threadIdx.x;
  const int64_t w = blockIdx.x;
  const int rh = (int)(w % a.RH);
  const int64_t rest = w / a.RH;
  const int s16 = (int)(rest & 7);
  const int64_t ti = t0 + (rest >> 3);
  if (ti >= t1) return;
  const ColTile T = a.tiles[ti];
  if (16 * s16 >= 2 * T.ngroups) return;             // uniform: nothing in this part
  colb16_part<DT, kColBSteps>(a, T, s16, rh, lane, sdst, ssig);
}

struct RedBArgs {
  const TBlock* tb;
  const int32_t* owner;
  const float* sigma;
  const float* part;
  float* t;
  int64_t n_red_t;        // t entries [0, n_red_t) come from partials
  int RS;
};

// t[o][j] = s_o * sum over the block's intervals (ascending) of its partials,
// for the blocks over several column chunks (t entries [0, n_red_t)); one
// thread per t entry o and four right-hand sides j (16-byte accesses).
template <int RS>
__global__ __launch_bounds__(256) void k_reduce_b(RedBArgs a) {
  constexpr int Q = RS / 4;                          // threads per t entry
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t o = e / Q;                           // division by a power of two
  const int j = 4 * (int)(e % Q);
  if (o >= a.n_red_t) return;
  const TBlock B = a.tb[a.owner[o]];
  const int l = (int)(o - B.toff);
  f32x4 s = (f32x4)(0.f);
  const f32x4* pp = reinterpret_cast<const f32x4*>(a.part + ((size_t)B.pst + l) * RS + j);
  const size_t step = (size_t)B.k * Q;               // f32x4 units between intervals
#pragma unroll 4
  for (int g = 0; g < B.nseg; ++g) {
    const f32x4 v = pp[g * step];
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] += v[c];
  }
  if (a.sigma) {
    const float sg = a.sigma[o];
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] *= sg;
  }
  *reinterpret_cast<f32x4*>(a.t + o * RS + j) = s;
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

// Decode one 16-byte group of storage format dt (FP32: 4 values; FP16 or
// BF16: 8) into v: DT >= 0 fixes the format at compile time, DT < 0 takes
// dt at run time.
template <int DT>
__device__ __forceinline__ void decode_group(int dt, u32x4 r, float (&v)[8]) {
  if constexpr (DT < 0) {
    if (dt == HM_F32) decode_group<HM_F32>(dt, r, v);
    else if (dt == HM_F16) decode_group<HM_F16>(dt, r, v);
    else decode_group<HM_BF16>(dt, r, v);
  } else if constexpr (DT == HM_F32) {
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

// 4 x 4 transpose across the four 16-lane groups: afterwards register q of
// lane 16 c + i holds what register c of lane 16 q + i held (two
// v_permlane32_swap, then two v_permlane16_swap).
__device__ __forceinline__ void xpose16x4(float& v0, float& v1, float& v2, float& v3) {
  const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v0), __float_as_uint(v2), false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v1), __float_as_uint(v3), false, false);
  const auto c = __builtin_amdgcn_permlane16_swap(a[0], b[0], false, false);
  const auto d = __builtin_amdgcn_permlane16_swap(a[1], b[1], false, false);
  v0 = __uint_as_float(c[0]);
  v1 = __uint_as_float(c[1]);
  v2 = __uint_as_float(d[0]);
  v3 = __uint_as_float(d[1]);
}

// One section of a row panel of at most 16 NB rows, storage format DT (or,
// for DT < 0, the section's own), for the groups g = wave, wave + 4, ...:
// per group a 16-byte load of the panel (lane = row, G columns).  Columns
// go in sets of 4: the transpose above turns the set's values of rows
// 16 q .. 16 q + 15 into the A operand of v_mfma_f32_16x16x4_f32 for row
// block q (lane 16 k + i: row 16 q + i, column k of the set).  The B
// operand of half h of the right-hand sides holds, in lane 16 k + j, value
// NV j + h of the source row of column k, so one load of NV = RS / 16
// consecutive values per lane brings all halves.  Groups go in steps of U;
// the loads of the next step are in flight while this step's MFMAs run,
// and the source slots of the step after that are read (scalar loads)
// meanwhile.
// With the format fixed (DT >= 0) the loads have no branches: a group past
// the section reads its last group, whose sources are replaced by zero at use
// (its MFMAs add nothing), and a lane past the panel's rows reads row 0,
// which fills only result rows that are never written; so the loop body is
// one basic block and the accumulators stay in their registers.  With the
// format taken at run time (sections of several formats, often of few
// groups) the steps stop at the section's last group instead.
template <int NH, int U, int NB, int DT>
__device__ __forceinline__ void rowb_section(const RowBArgs& a, const RowSection& S, int m,
                                             const int32_t* src, int lane, int wave,
                                             f32x4 (&acc)[NB][2 * NH]) {
  constexpr int RS = 32 * NH, NV = 2 * NH;
  constexpr bool kPad = DT >= 0;
  const int dt = DT >= 0 ? DT : S.dtype;
  const int G = DT >= 0 ? (DT == HM_F32 ? 4 : 8) : group_width(dt);
  typedef float fv __attribute__((ext_vector_type(NV)));
  const bool act = lane < m;
  const u32x4* p = reinterpret_cast<const u32x4*>(a.store + S.data_off) + (act ? lane : 0);
  const int32_t* sc = src + S.col0;                // source slot of every column of the section
  const int ng = S.ngroups, k = lane >> 4, j = lane & 15;
  auto load_slots = [&](int g0, int (&sn)[U][8]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int gg = g0 + 4 * u;
      if constexpr (kPad) gg = min(gg, ng - 1);
      else if (gg >= ng) break;                    // uniform across the wave
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c < G) sn[u][c] = sc[gg * G + c];
    }
  };
  auto srow = [&](int sl) {
    return sl < a.n_cols ? a.xr + (size_t)sl * RS : a.t + (size_t)(sl - a.n_cols) * RS;
  };
  auto issue = [&](int g0, const int (&sn)[U][8], u32x4 (&an)[U], fv (&bn)[U][2]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int gg = g0 + 4 * u;
      if constexpr (kPad) {
        an[u] = ld16(p + (size_t)min(gg, ng - 1) * m);
      } else {
        if (gg >= ng) break;                        // uniform across the wave
        an[u] = act ? ld16(p + (size_t)gg * m) : (u32x4)(0u);
      }
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        if (4 * s < G) {
          const float* r0 = srow(sn[u][4 * s]);
          const float* r1 = srow(sn[u][4 * s + 1]);
          const float* r2 = srow(sn[u][4 * s + 2]);
          const float* r3 = srow(sn[u][4 * s + 3]);
          const float* row = (k & 2) ? ((k & 1) ? r3 : r2) : ((k & 1) ? r1 : r0);
          bn[u][s] = *reinterpret_cast<const fv*>(row + NV * j);
        }
      }
    }
  };
  auto compute = [&](int g0, const u32x4 (&an)[U], const fv (&bn)[U][2]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (!kPad)
        if (g0 + 4 * u >= ng) break;                // uniform across the wave
      float v[8];
      decode_group<DT>(dt, an[u], v);
      // a group past the section (padded steps): its sources are replaced by zero
      const bool gok = !kPad || g0 + 4 * u < ng;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        if (4 * s < G) {
          xpose16x4(v[4 * s], v[4 * s + 1], v[4 * s + 2], v[4 * s + 3]);
          const fv b = gok ? bn[u][s] : (fv)(0.f);
#pragma unroll
          for (int q = 0; q < NB; ++q)
#pragma unroll
            for (int h = 0; h < NV; ++h) acc[q][h] = mfma16x4(v[4 * s + q], b[h], acc[q][h]);
        }
      }
    }
  };
  u32x4 a0[U], a1[U];
  fv b0[U][2], b1[U][2];                           // B operands of up to 2 sets of 4 columns
  int s0[U][8], s1[U][8];                          // source slots, one step ahead of their loads
  load_slots(wave, s0);
  issue(wave, s0, a0, b0);
  load_slots(wave + 4 * U, s1);
  if constexpr (kPad) {
    // two buffers take turns: while one step's MFMAs run, the next step's
    // loads are in flight into the other
    for (int g = wave; g < ng; g += 8 * U) {
      issue(g + 4 * U, s1, a1, b1);
      load_slots(g + 8 * U, s0);
      __builtin_amdgcn_sched_barrier(0);
      compute(g, a0, b0);
      issue(g + 8 * U, s0, a0, b0);
      load_slots(g + 12 * U, s1);
      __builtin_amdgcn_sched_barrier(0);
      compute(g + 4 * U, a1, b1);
    }
  } else {
    for (int g = wave; g < ng; g += 4 * U) {
      u32x4 ac[U];
      fv bc[U][2];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        ac[u] = a0[u];
        bc[u][0] = b0[u][0];
        bc[u][1] = b0[u][1];
      }
      issue(g + 4 * U, s1, a0, b0);
      load_slots(g + 8 * U, s1);
      compute(g, ac, bc);
    }
  }
}

// Groups per pipeline step in k_row_b: 2 for sections of run-time formats
// (measured fastest; deeper steps cost occupancy), kRowBStepF32 for the
// FP32-only kernel.
constexpr int kRowBStep = 2;
constexpr int kRowBStepF32 = 3;

// A row panel of at most 16 NB rows: the four waves take interleaved groups
// of every section, then their sums are added in a fixed order through LDS
// ((w0 + w2) + (w1 + w3)) and each row of Y is updated once.  red: 2 x 64
// rows of RS + 1 values (the padding keeps the row-wise reads of the update
// free of bank conflicts).
template <int NH, int NB, int DT>
__device__ __forceinline__ void rowb_panel(const RowBArgs& a, const RowPanel& P, float* red,
                                           int tid, int lane, int wave) {
  constexpr int RS = 32 * NH, NV = 2 * NH, RP = RS + 1;
  f32x4 acc[NB][NV];
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int h = 0; h < NV; ++h) acc[q][h] = (f32x4)(0.f);
  const int32_t* src = a.src + P.src_off;
  for (int qs = 0; qs < P.nsec; ++qs) {
    const RowSection S = a.rs[P.sec0 + qs];
    if (DT >= 0 || S.dtype != HM_F64)
      rowb_section<NH, DT >= 0 ? kRowBStepF32 : kRowBStep, NB, DT>(a, S, P.m, src, lane, wave, acc);
  }
  // acc[q][h] register v of lane 16 k + j: row 16 q + 4 k + v, right-hand side NV j + h.
  // Waves 2 and 3 store, waves 0 and 1 add (w0 + w2, w1 + w3), wave 1
  // stores, wave 0 adds and stores the panel's sums; then every thread
  // updates rows of Y (row-contiguous).
  const int k = lane >> 4, j = lane & 15;
  auto put = [&](int slot) {
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int h = 0; h < NV; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(slot * 64 + 16 * q + 4 * k + v) * RP + NV * j + h] = acc[q][h][v];
  };
  auto add = [&](int slot) {
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int h = 0; h < NV; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[q][h][v] += red[(slot * 64 + 16 * q + 4 * k + v) * RP + NV * j + h];
  };
  if (wave >= 2) put(wave - 2);
  __syncthreads();
  if (wave < 2) add(wave);
  __syncthreads();
  if (wave == 1) put(1);
  __syncthreads();
  if (wave == 0) {
    add(1);
    put(0);
  }
  __syncthreads();
  for (int e = tid; e < 16 * NB * RS; e += 256) {
    const int R = e % (16 * NB), c = e / (16 * NB);
    if (R < P.m && c < a.nrhs) {
      float* yp = a.Y + (size_t)c * a.ldy + P.row0 + R;
      *yp += a.alpha * red[R * RP + c];
    }
  }
}

// One workgroup per row panel, specialised on its number of 16-row blocks,
// and on the storage format when the store holds FP32 sections only (DT =
// HM_F32; else DT = -1, the format of each section).
template <int NH, int DT>
__global__ __launch_bounds__(256) void k_row_b(RowBArgs a) {
  constexpr int RS = 32 * NH;
  __shared__ float red[2 * 64 * (RS + 1)];
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  const int pi = panel_of(a.order, a.n_panels, blockIdx.x);
  if (pi < 0) return;                               // uniform: whole workgroup
  const RowPanel P = a.rp[pi];
  switch ((P.m + 15) >> 4) {                        // uniform: whole workgroup
    case 1: rowb_panel<NH, 1, DT>(a, P, red, tid, lane, wave); break;
    case 2: rowb_panel<NH, 2, DT>(a, P, red, tid, lane, wave); break;
    case 3: rowb_panel<NH, 3, DT>(a, P, red, tid, lane, wave); break;
    default: rowb_panel<NH, 4, DT>(a, P, red, tid, lane, wave); break;
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
      const float* sigma = h.has_sigma ? reinterpret_cast<const float*>(st + h.off_sigma) : nullptr;
      ColBArgs ca{st, reinterpret_cast<const ColTile*>(st + h.off_col_tiles),
                  reinterpret_cast<const int32_t*>(st + h.off_col_dst), xr, part,
                  (int32_t)(A.work_part_bytes / (int64_t)sizeof(float)), sigma, h.n_col_tiles, RS, RH};
      // one launch per tile class
      const int64_t* ce = h.tile_class_end;
      auto grid = [&](int64_t t0, int64_t t1, int parts) { return dim3((unsigned)((t1 - t0) * parts * RH)); };
      if (ce[1] > ce[0]) {
        switch (A.launch.colb) {
          case 1: hipLaunchKernelGGL(k_col_b32g<kColBSteps>, grid(ce[0], ce[1], 2), dim3(64), 0, s, ca, ce[0], ce[1]); break;
          case 2: hipLaunchKernelGGL(k_col_b32<2 * kColBSteps>, grid(ce[0], ce[1], 4), dim3(64), 0, s, ca, ce[0], ce[1]); break;
          case 3: hipLaunchKernelGGL(k_col_b32g<2 * kColBSteps>, grid(ce[0], ce[1], 2), dim3(64), 0, s, ca, ce[0], ce[1]); break;
          default: hipLaunchKernelGGL(k_col_b32<kColBSteps>, grid(ce[0], ce[1], 4), dim3(64), 0, s, ca, ce[0], ce[1]); break;
        }
      }
      if (ce[2] > ce[1])
        hipLaunchKernelGGL(k_col_b16<HM_F16>, grid(ce[1], ce[2], 8), dim3(64), 0, s, ca, ce[1], ce[2]);
      if (ce[3] > ce[2])
        hipLaunchKernelGGL(k_col_b16<HM_BF16>, grid(ce[2], ce[3], 8), dim3(64), 0, s, ca, ce[2], ce[3]);
      // (FP64 and DFL tiles, classes 0 and 4..8, do not occur with FP32 accumulation)
      constexpr int M = kNumDtypes;
      if (ce[M] > ce[M - 1])
        hipLaunchKernelGGL(k_col_b16<-1>, grid(ce[M - 1], ce[M], 8), dim3(64), 0, s, ca, ce[M - 1], ce[M]);
      if (ev && r0 == 0) (void)hipEventRecord(ev[1], s);
      RedBArgs rb{reinterpret_cast<const TBlock*>(st + h.off_tblocks),
                  reinterpret_cast<const int32_t*>(st + h.off_owner), sigma, part, t, h.n_red_t, RS};
      const int64_t nthr = h.n_red_t * (RS / 4);
      if (nthr > 0) {
        if (RS == 32)
          hipLaunchKernelGGL(k_reduce_b<32>, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, rb);
        else
          hipLaunchKernelGGL(k_reduce_b<64>, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, rb);
      }
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
    const unsigned grid = (unsigned)panel_items(xcd, h.n_row_panels);
    // FP32 sections only: the format-specialised row kernel
    bool f32_only = A.bytes_by_dtype[HM_F32] > 0;
    for (int d = 0; d < kNumDtypes; ++d) f32_only &= d == HM_F32 || A.bytes_by_dtype[d] == 0;
    if (RH == 1) {
      if (f32_only) hipLaunchKernelGGL((k_row_b<1, HM_F32>), dim3(grid), dim3(256), 0, s, ra);
      else hipLaunchKernelGGL((k_row_b<1, -1>), dim3(grid), dim3(256), 0, s, ra);
    } else {
      if (f32_only) hipLaunchKernelGGL((k_row_b<2, HM_F32>), dim3(grid), dim3(256), 0, s, ra);
      else hipLaunchKernelGGL((k_row_b<2, -1>), dim3(grid), dim3(256), 0, s, ra);
    }
  }
  if (ev) (void)hipEventRecord(ev[3], s);
  return hipGetLastError();
}

}  // namespace hm
