// HIP kernels (gfx950) of the H-matrix-vector product with one right-hand
// side, and their launchers (hm_mvm).
//
// One product y += alpha * sum_b E_tau M_b E_sigma^T x (Sec. 2.1, Eq. (1);
// the product only needs the blocks decoded from storage, Sec. 5.4) runs as
// three stream-ordered kernels over the packed store (layout: hm_layout.hpp).
// Schedule 0:
//  k_col     far field, phase 1: one workgroup per column tile streams the
//            rows of V_b restricted to a column chunk, for all low-rank
//            blocks covering it (lane = group of columns, x of the chunk
//            staged in LDS and read as a broadcast), and writes one partial
//            dot product per column (for a block inside one chunk that sum,
//            times s_b[l], is t_b[l]);
//  k_reduce  t_b[l] = s_b[l] * sum of the block's partials in chunk order,
//            for the blocks over several chunks;
//  k_row     near field and far field, phase 2: one workgroup per row panel
//            gathers its sources (x and t) into LDS, streams the panel's
//            dense and U sections with 16-byte loads (lane = row), and
//            updates its rows of y once.
// Schedule 1 (grouped): k_p1 runs the dense sections of the row panels and
// the column tiles in one launch, then k_reduce, then k_p2 the U sections.
// Either schedule may run as persistent grids that loop over the items.
//
// Every sum has a fixed order, so results are bitwise reproducible and no
// atomics touch y.  Storage formats (FP64/FP32/FP16/BF16, Table 1; the
// byte-aligned DFL, AFLP and BFL formats, Sec. 3.2) are decoded to the
// accumulation type in registers.

#include <algorithm>
#include <mutex>

#include <hip/hip_runtime.h>

#include "hm_internal.hpp"
#include "hm_device.hpp"

namespace hm {
namespace {

// FP64 encoding of value c of a DFL group element (exact).  DFL32 / 40 / 48: r[c] is the
// high word of its FP64 encoding, and the element's low-byte plane entry lo
// holds bits 31..24 in byte c (DFL40) or bits 31..16 in 16-bit half c
// (DFL48).  DFL16 / 24: 16-bit half c of r holds bits 63..48, and byte c of
// lo bits 47..40 (DFL24); the low word is zero.
template <int DT>
__device__ __forceinline__ unsigned long long dfl_bits(u32x4 r, u32x2 lo, int c) {
  unsigned hi, low = 0;
  if constexpr (DT == kDtDfl16 || DT == kDtDfl24) {
    hi = ((r[c >> 1] >> (16 * (c & 1))) & 0xffffu) << 16;
    if constexpr (DT == kDtDfl24) hi |= ((lo[c >> 2] >> (8 * (c & 3))) & 0xffu) << 8;
  } else {
    hi = r[c];
    if constexpr (DT == kDtDfl40) low = ((lo[0] >> (8 * c)) & 0xffu) << 24;
    if constexpr (DT == kDtDfl48) low = ((lo[c >> 1] >> (16 * (c & 1))) & 0xffffu) << 16;
  }
  return ((unsigned long long)hi << 32) | low;
}

template <int DT>
__device__ __forceinline__ double dfl_value(u32x4 r, u32x2 lo, int c) {
  return __longlong_as_double((long long)dfl_bits<DT>(r, lo, c));
}

// sign(P) (d - 1) of an AFLP element (the scale 2^k is applied outside):
// the code P, left-aligned like a DFL encoding of the same bytes, gives d's
// FP64 bits as ((P & ~sign) >> sh) + bits(1.0), sh = 11 - e; d - 1 is
// exact.  The zero code gives d = 1.
template <int DT>
__device__ __forceinline__ double aflp_value(u32x4 r, u32x2 lo, int c, unsigned sh) {
  const unsigned long long P = dfl_bits<storage_dt(DT)>(r, lo, c);
  const unsigned long long d = ((P & 0x7fffffffffffffffull) >> sh) + 0x3ff0000000000000ull;
  const double w = __longlong_as_double((long long)d) - 1.0;
  // P's sign into w's high word (one bit-field insert)
  const unsigned hi = ((unsigned)(P >> 32) & 0x80000000u) | ((unsigned)__double2hiint(w) & 0x7fffffffu);
  return __hiloint2double((int)hi, __double2loint(w));
}

// A BFL element (exact): the code P, left-aligned like a DFL encoding of
// the same bytes, holds FP32's sign, exponent E and leading mantissa bits.
// With the magnitude moved down 3 bits it is the normal FP64 number
// 2^(E - 1023) (1.f) (E >= 1), and 0 for the zero code; times 2^896 (exact)
// it is the value, with no test for zero.
template <int DT>
__device__ __forceinline__ double bfl_value(u32x4 r, u32x2 lo, int c) {
  const unsigned long long P = dfl_bits<storage_dt(DT)>(r, lo, c);
  const unsigned long long q = ((P & 0x7fffffffffffffffull) >> 3) | (P & 0x8000000000000000ull);
  return __longlong_as_double((long long)q) * 0x1p896;
}

// The low-byte plane entry idx of a DFL40 / DFL48 / DFL24 region at p
// (zero for the other formats, which have none).
template <int DT>
__device__ __forceinline__ u32x2 ld_lo(const uint8_t* p, int64_t idx) {
  if constexpr (storage_dt(DT) == kDtDfl40) {
    return u32x2{__builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p) + idx), 0u};
  } else if constexpr (storage_dt(DT) == kDtDfl48 || storage_dt(DT) == kDtDfl24) {
    return __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p) + idx);
  } else {
    return (u32x2)(0u);
  }
}

// acc += sum_c v[c] * z[c] over one 16-byte group of storage format DT
// (lo: its low-byte plane entry, 40 / 48 / 24-bit formats only; AFLP: sh
// the columns' shifts, 16-byte aligned, z already scaled by the columns' 2^k).
template <typename AccT, int DT>
__device__ __forceinline__ AccT dot_group(u32x4 r, u32x2 lo, const AccT* __restrict__ z,
                                          const uint32_t* __restrict__ sh, AccT acc) {
  if constexpr (is_aflp(DT)) {
    constexpr int G = group_width(DT);
    unsigned s[G];
#pragma unroll
    for (int q = 0; q < G / 4; ++q) {
      const u32x4 w = *reinterpret_cast<const u32x4*>(sh + 4 * q);
#pragma unroll
      for (int c = 0; c < 4; ++c) s[4 * q + c] = w[c];
    }
#pragma unroll
    for (int c = 0; c < G; ++c) acc = fmaT((AccT)aflp_value<DT>(r, lo, c, s[c]), z[c], acc);
  } else if constexpr (is_bfl(DT)) {
#pragma unroll
    for (int c = 0; c < group_width(DT); ++c) acc = fmaT((AccT)bfl_value<DT>(r, lo, c), z[c], acc);
  } else if constexpr (is_dfl(DT)) {
#pragma unroll
    for (int c = 0; c < group_width(DT); ++c) acc = fmaT((AccT)dfl_value<DT>(r, lo, c), z[c], acc);
  } else if constexpr (DT == HM_F64) {
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

// acc[c] += v[c] * xi for the G columns of one 16-byte group (AFLP: sh the
// columns' shifts; the sums are scaled by the columns' 2^k afterwards).
template <typename AccT, int DT>
__device__ __forceinline__ void axpy_group(u32x4 r, u32x2 lo, AccT xi, AccT* acc, const unsigned* sh) {
  if constexpr (is_aflp(DT)) {
#pragma unroll
    for (int c = 0; c < group_width(DT); ++c) acc[c] = fmaT((AccT)aflp_value<DT>(r, lo, c, sh[c]), xi, acc[c]);
  } else if constexpr (is_bfl(DT)) {
#pragma unroll
    for (int c = 0; c < group_width(DT); ++c) acc[c] = fmaT((AccT)bfl_value<DT>(r, lo, c), xi, acc[c]);
  } else if constexpr (is_dfl(DT)) {
#pragma unroll
    for (int c = 0; c < group_width(DT); ++c) acc[c] = fmaT((AccT)dfl_value<DT>(r, lo, c), xi, acc[c]);
  } else if constexpr (DT == HM_F64) {
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

// ---------------------------------------------------------------- column tiles

// Orders the LDS accesses of the calling wave's lanes: what a lane wrote
// before is visible to every lane of the wave after (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename AccT>
struct ColArgs {
  const uint8_t* store;
  const ColTile* tiles;
  const int32_t* dst;
  const AccT* x;
  AccT* part;
  AccT* t;                // column sums of blocks inside one chunk go here
  const AccT* sigma;      // nullptr when no block keeps singular values
  const int32_t* aflp;    // aflp_param per tile column (beside dst); nullptr: no AFLP data
  int64_t n_tiles;
};

// One workgroup streams one column tile.  A narrow tile shares each wave
// between RS = 64 / GP rows, GP the smallest power of two >= the tile's
// groups: lane l owns the columns of group g = l % GP in the rows of
// sub-row q = l / GP, so that one 16-byte load per lane covers RS tile
// rows.  The tile's rows go to the four waves in interleaved batches
// of 8 RS (wave w takes rows RS (32 j + 8 w) + [0, 8 RS) for j = 0, 1, ...,
// row RS (32 j + 8 w + u) + q in step u), and the loads of a wave's next
// batch are in flight while it computes the current one.  x of the tile's
// rows is staged in LDS once (xs).  The RS sub-rows' sums are added by a
// butterfly across the lanes, the four waves' sums in a fixed order through
// LDS (red: 4 x 64 x 8), and wave 0 writes each column's sum to its
// destination (a partial, or t).  DT >= 0: every group of the tile has
// format DT; DT < 0: the tile holds runs of several formats and each lane
// decodes its own (T.dtype, T.end); DFL / AFLP / BFL: such a tile may hold
// runs of those formats.  An AFLP lane keeps its columns' shifts in registers and
// scales its sums by the columns' 2^k before they are written.
// WAVE: the calling wave streams the tile alone (all batches of 8 RS rows),
// with xs its own kSegRows values of LDS, and its lanes of sub-row 0 write
// the sums after the butterfly (no workgroup barrier; red unused).
template <typename AccT, int DT, bool DFL = false, bool AFLP = false, bool BFL = false, bool WAVE = false>
__device__ __forceinline__ void col_tile(const ColArgs<AccT>& a, const ColTile& T, AccT* red, AccT* xs) {
  constexpr int NW = WAVE ? 1 : 4;                  // waves sharing the tile
  const int lane = threadIdx.x & 63, wave = WAVE ? 0 : threadIdx.x >> 6;
  const int ng = T.ngroups;
  const int GP = ng <= 1 ? 1 : ng <= 2 ? 2 : ng <= 4 ? 4 : ng <= 8 ? 8 : ng <= 16 ? 16 : ng <= 32 ? 32 : 64;
  const int RS = 64 / GP;                           // rows per wave-wide step (sub-rows)
  const int g = lane & (GP - 1), q = lane / GP;     // group and sub-row of this lane
  const bool act = g < T.ngroups;
  const TileGroup tg = tile_group(T, act ? g : 0);
  const int dt = DT >= 0 ? DT : tg.dtype;
  constexpr bool kAflp = DT >= 0 ? is_aflp(DT) : AFLP;
  constexpr int GW = DT >= 0 ? group_width(DT) : 8;   // columns per lane (at most)
  unsigned sh[GW];
#pragma unroll
  for (int c = 0; c < GW; ++c) sh[c] = 0;
  if constexpr (kAflp) {
    if (act && is_aflp(dt)) {
      const int G = group_width(dt);
#pragma unroll
      for (int c = 0; c < GW; ++c)
        if (c < G) sh[c] = aflp_shift(a.aflp[T.dst_off + tg.col + c]);
    }
  }
  AccT acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = AccT(0);
  const int rstride = T.ngroups;                    // 16-byte groups per tile row
  const int nrows = T.nrows;
  const u32x4* p = reinterpret_cast<const u32x4*>(a.store + T.data_off) + g;
  // low-byte plane: entries of lo_bytes(DT) bytes in a one-format tile; of
  // Lt bytes in a several-format one (read by the lanes whose format has one)
  const uint8_t* lop = a.store + T.data_off + (int64_t)16 * nrows * rstride;
  constexpr bool LOW = DFL || AFLP || BFL;         // several-format tiles: runs with low bytes
  const int Lt = DT < 0 && LOW ? tile_lo_bytes(T) : 0;
  const bool hlo = DT < 0 && LOW && lo_bytes(dt) > 0;
  const int nb = nrows > 8 * RS * wave ? (nrows - 8 * RS * wave + 8 * NW * RS - 1) / (8 * NW * RS) : 0;   // this wave's batches
  u32x4 rn[8];
  u32x2 ln[8];
  auto issue = [&](int j) {
    const int r0 = RS * (8 * NW * j + 8 * wave) + q;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (act && r0 + RS * u < nrows) {
        const int64_t row = r0 + RS * u;
        rn[u] = ld16(p + (size_t)row * rstride);
        if constexpr (DT >= 0) {
          ln[u] = ld_lo<DT>(lop, row * rstride + g);
        } else if constexpr (LOW) {
          if (hlo) {
            const int64_t e = row * rstride + g;
            ln[u] = Lt == 8 ? ld_lo<kDtDfl48>(lop, e) : ld_lo<kDtDfl40>(lop, e);
          }
        }
      }
  };
  if (nb > 0) issue(0);
  if constexpr (WAVE) {
    for (int i = lane; i < nrows; i += 64) xs[i] = a.x[T.x0 + i];
    wave_sync();
  } else {
    for (int i = threadIdx.x; i < nrows; i += 256) xs[i] = a.x[T.x0 + i];
    __syncthreads();
  }
  for (int j = 0; j < nb; ++j) {
    u32x4 rc[8];
    u32x2 lc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      rc[u] = rn[u];
      lc[u] = ln[u];
    }
    if (j + 1 < nb) issue(j + 1);
    const int r0 = RS * (8 * NW * j + 8 * wave) + q;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (r0 + RS * u < nrows) {                    // uniform across a sub-row
        const AccT xi = xs[r0 + RS * u];
        if (act) {
          if constexpr (DT >= 0) {
            axpy_group<AccT, DT>(rc[u], lc[u], xi, acc, sh);
          } else if (dt == HM_F32) {
            axpy_group<AccT, HM_F32>(rc[u], lc[u], xi, acc, sh);
          } else if (dt == HM_F16) {
            axpy_group<AccT, HM_F16>(rc[u], lc[u], xi, acc, sh);
          } else if (dt == HM_BF16) {
            axpy_group<AccT, HM_BF16>(rc[u], lc[u], xi, acc, sh);
          } else if constexpr (sizeof(AccT) == 8) {
            // FP64-accumulation formats
            if (DFL && dt == kDtDfl32) axpy_group<AccT, kDtDfl32>(rc[u], lc[u], xi, acc, sh);
            else if (DFL && dt == kDtDfl16) axpy_group<AccT, kDtDfl16>(rc[u], lc[u], xi, acc, sh);
            else if (DFL && dt == kDtDfl24) axpy_group<AccT, kDtDfl24>(rc[u], lc[u], xi, acc, sh);
            else if (DFL && dt == kDtDfl40) axpy_group<AccT, kDtDfl40>(rc[u], lc[u], xi, acc, sh);
            else if (DFL && dt == kDtDfl48) axpy_group<AccT, kDtDfl48>(rc[u], lc[u], xi, acc, sh);
            else if (AFLP && dt == kDtAflp32) axpy_group<AccT, kDtAflp32>(rc[u], lc[u], xi, acc, sh);
            else if (AFLP && dt == kDtAflp16) axpy_group<AccT, kDtAflp16>(rc[u], lc[u], xi, acc, sh);
            else if (AFLP && dt == kDtAflp24) axpy_group<AccT, kDtAflp24>(rc[u], lc[u], xi, acc, sh);
            else if (AFLP && dt == kDtAflp40) axpy_group<AccT, kDtAflp40>(rc[u], lc[u], xi, acc, sh);
            else if (AFLP && dt == kDtAflp48) axpy_group<AccT, kDtAflp48>(rc[u], lc[u], xi, acc, sh);
            else if (BFL && dt == kDtBfl40) axpy_group<AccT, kDtBfl40>(rc[u], lc[u], xi, acc, sh);
            else if (BFL && dt == kDtBfl48) axpy_group<AccT, kDtBfl48>(rc[u], lc[u], xi, acc, sh);
            else if (BFL && dt == kDtBfl24) axpy_group<AccT, kDtBfl24>(rc[u], lc[u], xi, acc, sh);
            else axpy_group<AccT, HM_F64>(rc[u], lc[u], xi, acc, sh);
          }
        }
      }
  }
  // sum over the sub-rows: a butterfly over the lanes of one group (fixed order)
  for (int o = GP; o < 64; o <<= 1) {
#pragma unroll
    for (int c = 0; c < GW; ++c) acc[c] += __shfl_xor(acc[c], o, 64);
  }
  if constexpr (!WAVE) {
#pragma unroll
    for (int c = 0; c < GW; ++c) red[(wave * 64 + lane) * GW + c] = acc[c];   // red stride GW per lane
    __syncthreads();
  }
  if (wave == 0 && q == 0 && act) {
    const int G = group_width(dt);
    // all destinations and factors first, then the stores
    int32_t d[GW];
    AccT f[GW];
#pragma unroll
    for (int c = 0; c < GW; ++c) d[c] = c < G ? a.dst[T.dst_off + tg.col + c] : kDstPad;
#pragma unroll
    for (int c = 0; c < GW; ++c) f[c] = (d[c] <= -2 && a.sigma) ? a.sigma[dst_t_index(d[c])] : AccT(1);
    int ks[GW];                                     // AFLP: the columns' scale exponents
#pragma unroll
    for (int c = 0; c < GW; ++c) ks[c] = 0;
    if constexpr (kAflp) {
      if (is_aflp(dt)) {
#pragma unroll
        for (int c = 0; c < GW; ++c)
          if (c < G) ks[c] = aflp_scale_exp(a.aflp[T.dst_off + tg.col + c]);
      }
    }
#pragma unroll
    for (int c = 0; c < GW; ++c) {
      AccT sum = acc[c];
      if constexpr (!WAVE)
        sum = (red[g * GW + c] + red[(64 + g) * GW + c]) + (red[(128 + g) * GW + c] + red[(192 + g) * GW + c]);
      if constexpr (kAflp) sum = ldexp(sum, ks[c]);     // exact: a power of two
      if (d[c] >= 0)
        a.part[d[c]] = sum;
      else if (d[c] != kDstPad)
        a.t[dst_t_index(d[c])] = a.sigma ? sum * f[c] : sum;
    }
  }
}

// Tile kinds one instantiation decodes (a bit set; launches go per tile
// class, so that the FP64 / IEEE paths carry no code of the DFL formats).
constexpr int kColIeee = 1;     // one-format tiles of FP64, FP32, FP16, BF16
constexpr int kColMulti = 2;    // several-format tiles
constexpr int kColDfl = 4;      // one-format DFL tiles, and DFL runs in several-format tiles
constexpr int kColAflp = 8;     // AFLP runs in several-format tiles
constexpr int kColBfl = 16;     // BFL runs in several-format tiles

// A whole workgroup on tile ti (it synchronizes).  red: 4 * 64 * 8 values
// (four waves x 64 lanes x at most 8 columns per lane); xs: kSegRows
// values (x of the tile's rows).
// DT >= 0: every tile has that one format.
// WAVE: the calling wave alone (col_tile).
template <typename AccT, int KIND, int DT = -1, bool WAVE = false>
__device__ __forceinline__ void col_tile_any(const ColArgs<AccT>& a, int64_t ti, AccT* red, AccT* xs) {
  const ColTile T = a.tiles[ti];
  if constexpr (DT >= 0) {
    col_tile<AccT, DT, false, false, false, WAVE>(a, T, red, xs);
    return;
  }
  constexpr bool dfl = (KIND & kColDfl) && sizeof(AccT) == 8;
  constexpr bool aflp = (KIND & kColAflp) && sizeof(AccT) == 8;
  constexpr bool bfl = (KIND & kColBfl) && sizeof(AccT) == 8;
  if constexpr ((KIND & kColMulti) != 0) {
    if (T.end[0] < T.ngroups) {                     // several formats in the tile
      col_tile<AccT, -1, dfl, aflp, bfl, WAVE>(a, T, red, xs);
      return;
    }
  }
  if constexpr (bfl) {
    switch (T.dtype[0]) {
      case kDtBfl24: col_tile<AccT, kDtBfl24, false, false, false, WAVE>(a, T, red, xs); return;
      case kDtBfl40: col_tile<AccT, kDtBfl40, false, false, false, WAVE>(a, T, red, xs); return;
      case kDtBfl48: col_tile<AccT, kDtBfl48, false, false, false, WAVE>(a, T, red, xs); return;
      default: break;
    }
  }
  if constexpr (aflp) {
    switch (T.dtype[0]) {
      case kDtAflp32: col_tile<AccT, kDtAflp32, false, false, false, WAVE>(a, T, red, xs); return;
      case kDtAflp40: col_tile<AccT, kDtAflp40, false, false, false, WAVE>(a, T, red, xs); return;
      case kDtAflp48: col_tile<AccT, kDtAflp48, false, false, false, WAVE>(a, T, red, xs); return;
      case kDtAflp16: col_tile<AccT, kDtAflp16, false, false, false, WAVE>(a, T, red, xs); return;
      case kDtAflp24: col_tile<AccT, kDtAflp24, false, false, false, WAVE>(a, T, red, xs); return;
      default: break;
    }
  }
  if constexpr (dfl) {
    switch (T.dtype[0]) {
      case kDtDfl32: col_tile<AccT, kDtDfl32, false, false, false, WAVE>(a, T, red, xs); return;
      case kDtDfl40: col_tile<AccT, kDtDfl40, false, false, false, WAVE>(a, T, red, xs); return;
      case kDtDfl48: col_tile<AccT, kDtDfl48, false, false, false, WAVE>(a, T, red, xs); return;
      case kDtDfl16: col_tile<AccT, kDtDfl16, false, false, false, WAVE>(a, T, red, xs); return;
      case kDtDfl24: col_tile<AccT, kDtDfl24, false, false, false, WAVE>(a, T, red, xs); return;
      default: break;
    }
  }
  if constexpr ((KIND & kColIeee) != 0) {
    switch (T.dtype[0]) {
      case HM_F64:
        if constexpr (sizeof(AccT) == 8) col_tile<AccT, HM_F64, false, false, false, WAVE>(a, T, red, xs);
        break;
      case HM_F32: col_tile<AccT, HM_F32, false, false, false, WAVE>(a, T, red, xs); break;
      case HM_F16: col_tile<AccT, HM_F16, false, false, false, WAVE>(a, T, red, xs); break;
      default: col_tile<AccT, HM_BF16, false, false, false, WAVE>(a, T, red, xs); break;
    }
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
  int64_t n_large, n_large_t, n_red_t;
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
  if (o >= a.n_red_t) return;
  const TBlock B = a.tb[a.owner[o]];
  const int l = (int)(o - B.toff);
  AccT s = AccT(0);
  for (int j = 0; j < B.nseg; ++j) s += a.part[B.pst + (int64_t)j * B.k + l];
  a.t[o] = a.sigma ? s * a.sigma[o] : s;
}

// ---------------------------------------------------------------- row panels

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
  const int32_t* aflp;    // aflp_param per source slot (beside src); nullptr: no AFLP data
};

// Formats a row-panel instantiation decodes besides FP64 / FP32 / FP16 /
// BF16 (a bit set; FP64 accumulation only).
constexpr int kXfDfl = 1, kXfAflp = 2, kXfBfl = 4;

// Groups [g_lo, g_hi) of a section at base (its low-byte plane, if any, at
// lo_base), groups g_lo + wave, + 4, ... for this wave.
template <typename AccT, int DT, int U>
__device__ __forceinline__ AccT row_section(const uint8_t* base, const uint8_t* lo_base, int m, int g_lo,
                                            int g_hi, const AccT* z, const uint32_t* shz, int lane, int wave,
                                            AccT acc) {
  constexpr int G = group_width(DT);
  const u32x4* p = reinterpret_cast<const u32x4*>(base) + lane;
  int g = g_lo + wave;
  // U groups per wave in flight, all loads issued before the arithmetic
  for (; g + 4 * (U - 1) < g_hi; g += 4 * U) {
    u32x4 r[U];
    u32x2 l[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      r[u] = ld16(p + (size_t)(g + 4 * u) * m);
      l[u] = ld_lo<DT>(lo_base, (int64_t)(g + 4 * u) * m + lane);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      acc = dot_group<AccT, DT>(r[u], l[u], z + (g + 4 * u) * G, shz + (g + 4 * u) * G, acc);
  }
  for (; g < g_hi; g += 4)
    acc = dot_group<AccT, DT>(ld16(p + (size_t)g * m), ld_lo<DT>(lo_base, (int64_t)g * m + lane), z + g * G,
                              shz + g * G, acc);
  return acc;
}

// Sections [q_begin, q_end) of row panel P (source slots [s_begin, s_end)):
// sources staged in LDS by chunks of CAP slots, four waves stream the groups,
// a fixed-order LDS reduction, then one update of the panel's rows of y.
// Called by whole workgroups (it synchronizes).
// XF: the store holds DFL / AFLP sections (decoded only by such
// instantiations).  AFLP: a slot's source is staged times its column's 2^k
// (exact) and its shift beside it (shs, CAP words).
template <typename AccT, int CAP, int U, int XF>
__device__ __forceinline__ void row_panel_part(const RowArgs<AccT>& a, const RowPanel& P,
                                               int q_begin, int q_end, int s_begin, int s_end,
                                               AccT* zs, AccT (*red)[64], uint32_t* shs) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  AccT acc = AccT(0);
  const int32_t* src = a.src + P.src_off;
  for (int c_lo = s_begin; c_lo < s_end; c_lo += CAP) {
    const int c_hi = min(s_end, c_lo + CAP);
    for (int c = c_lo + tid; c < c_hi; c += 256) {
      const int s = src[c];
      AccT z = s < a.n_cols ? a.x[s] : a.t[s - a.n_cols];
      if constexpr ((XF & kXfAflp) != 0) {
        const int32_t q = a.aflp[P.src_off + c];
        z = ldexp(z, aflp_scale_exp(q));
        shs[c - c_lo] = (uint32_t)aflp_shift(q);
      }
      zs[c - c_lo] = z;
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
        const uint8_t* lob = base + (int64_t)16 * S.ngroups * P.m;   // low-byte plane (40 / 48 / 24 bits)
        const AccT* z = zs + (S.col0 - c_lo);
        const uint32_t* sz = shs + (S.col0 - c_lo);
#define HM_ROW_SECTION(D) acc = row_section<AccT, D, U>(base, lob, P.m, g_lo, g_hi, z, sz, lane, wave, acc)
        switch (S.dtype) {
          case HM_F32: HM_ROW_SECTION(HM_F32); break;
          case HM_F16: HM_ROW_SECTION(HM_F16); break;
          case HM_BF16: HM_ROW_SECTION(HM_BF16); break;
          default:                                  // FP64-accumulation formats
            if constexpr (sizeof(AccT) == 8 && XF == 0) {
              HM_ROW_SECTION(HM_F64);
            } else if constexpr (sizeof(AccT) == 8) {
              switch (S.dtype) {
                case HM_F64: HM_ROW_SECTION(HM_F64); break;
                case kDtDfl32: if constexpr ((XF & kXfDfl) != 0) HM_ROW_SECTION(kDtDfl32); break;
                case kDtDfl40: if constexpr ((XF & kXfDfl) != 0) HM_ROW_SECTION(kDtDfl40); break;
                case kDtDfl16: if constexpr ((XF & kXfDfl) != 0) HM_ROW_SECTION(kDtDfl16); break;
                case kDtDfl24: if constexpr ((XF & kXfDfl) != 0) HM_ROW_SECTION(kDtDfl24); break;
                case kDtDfl48: if constexpr ((XF & kXfDfl) != 0) HM_ROW_SECTION(kDtDfl48); break;
                case kDtAflp32: if constexpr ((XF & kXfAflp) != 0) HM_ROW_SECTION(kDtAflp32); break;
                case kDtAflp40: if constexpr ((XF & kXfAflp) != 0) HM_ROW_SECTION(kDtAflp40); break;
                case kDtAflp16: if constexpr ((XF & kXfAflp) != 0) HM_ROW_SECTION(kDtAflp16); break;
                case kDtAflp24: if constexpr ((XF & kXfAflp) != 0) HM_ROW_SECTION(kDtAflp24); break;
                case kDtAflp48: if constexpr ((XF & kXfAflp) != 0) HM_ROW_SECTION(kDtAflp48); break;
                case kDtBfl40: if constexpr ((XF & kXfBfl) != 0) HM_ROW_SECTION(kDtBfl40); break;
                case kDtBfl48: if constexpr ((XF & kXfBfl) != 0) HM_ROW_SECTION(kDtBfl48); break;
                default: if constexpr ((XF & kXfBfl) != 0) HM_ROW_SECTION(kDtBfl24); break;
              }
            }
            break;
        }
#undef HM_ROW_SECTION
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
template <typename AccT, int CAP, int U, int XF>
__global__ __launch_bounds__(256) void k_p1(RowArgs<AccT> ra, ColArgs<AccT> ca, const int32_t* order,
                                            int64_t n_items) {
  static_assert(CAP >= 4 * 64 * 8, "staging buffer doubles as the tile reduction buffer");
  __shared__ AccT zs[CAP];
  __shared__ AccT red[4][64];
  __shared__ AccT pxs[kSegRows];
  __shared__ __align__(16) uint32_t shs[(XF & kXfAflp) ? CAP : 4];
  constexpr int KIND = kColIeee | kColMulti | ((XF & kXfDfl) ? kColDfl : 0) | ((XF & kXfAflp) ? kColAflp : 0) |
                       ((XF & kXfBfl) ? kColBfl : 0);
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    if (it != blockIdx.x) __syncthreads();          // LDS of the previous item
    const int item = order[it];
    if (item >= 0) {
      const RowPanel P = ra.rp[item];
      row_panel_part<AccT, CAP, U, XF>(ra, P, 0, P.nsec_dense, 0, dense_slot_end(ra, P), zs, red, shs);
    } else {
      col_tile_any<AccT, KIND>(ca, -(int64_t)item - 1, zs, pxs);
    }
  }
}

// Phase 2: the U sections of the row panels (after t is complete).
template <typename AccT, int CAP, int U, int XF>
__global__ __launch_bounds__(256) void k_p2(RowArgs<AccT> ra, const int32_t* order, int64_t n_items) {
  __shared__ AccT zs[CAP];
  __shared__ AccT red[4][64];
  __shared__ __align__(16) uint32_t shs[(XF & kXfAflp) ? CAP : 4];
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    if (it != blockIdx.x) __syncthreads();
    const RowPanel P = ra.rp[order[it]];
    row_panel_part<AccT, CAP, U, XF>(ra, P, P.nsec_dense, P.nsec, dense_slot_end(ra, P), P.ncols, zs, red,
                                     shs);
  }
}

// Schedule 0: all column tiles (one per workgroup item), then whole row
// panels (dense and U sections in one pass).
// Tiles [t0, t1) of the classes KIND decodes (DT >= 0: the one-format
// class DT).  Four workgroups per CU, three where the registers need it
// (several-format tiles; the DFL formats with low-byte loads).
constexpr int col_wgs(int kind, int dt) {
  return (kind == kColIeee || dt == kDtDfl32 || dt == kDtDfl16) ? 4 : 3;
}
template <typename AccT, int KIND, int DT = -1>
__global__ __launch_bounds__(256, col_wgs(KIND, DT))
void k_col(ColArgs<AccT> ca, int64_t t0, int64_t t1) {
  __shared__ AccT cred[4 * 64 * 8];
  __shared__ AccT cxs[kSegRows];
  for (int64_t it = t0 + blockIdx.x; it < t1; it += gridDim.x) {
    if (it != t0 + blockIdx.x) __syncthreads();
    col_tile_any<AccT, KIND, DT>(ca, it, cred, cxs);
  }
}

// The same tiles, one per wave: wave w of workgroup b takes tiles
// t0 + 4 b + w, t0 + 4 (b + gridDim.x) + w, ...  For classes of small tiles,
// whose rows one wave covers in a batch or two, where a workgroup per tile
// would leave waves idle.
template <typename AccT, int KIND, int DT = -1>
__global__ __launch_bounds__(256, col_wgs(KIND, DT))
void k_col_w(ColArgs<AccT> ca, int64_t t0, int64_t t1) {
  __shared__ AccT cxs[4][kSegRows];
  const int wave = wave_id();
  for (int64_t it = t0 + 4 * (int64_t)blockIdx.x + wave; it < t1; it += 4 * (int64_t)gridDim.x) {
    wave_sync();                                    // xs of the wave's previous tile read
    col_tile_any<AccT, KIND, DT, true>(ca, it, nullptr, cxs[wave]);
  }
}

// Two neighbouring launch classes in one launch, a wave per tile: tiles
// [t0, tm) of class (KA, DA), [tm, t1) of class (KB, DB).  One ramp and
// tail instead of two where a store spreads its columns over many formats.
template <typename AccT, int KA, int DA, int KB, int DB>
__global__ __launch_bounds__(256, col_wgs(KA, DA) < col_wgs(KB, DB) ? col_wgs(KA, DA) : col_wgs(KB, DB))
void k_col_w2(ColArgs<AccT> ca, int64_t t0, int64_t tm, int64_t t1) {
  __shared__ AccT cxs[4][kSegRows];
  const int wave = wave_id();
  for (int64_t it = t0 + 4 * (int64_t)blockIdx.x + wave; it < t1; it += 4 * (int64_t)gridDim.x) {
    wave_sync();                                    // xs of the wave's previous tile read
    if (it < tm) col_tile_any<AccT, KA, DA, true>(ca, it, nullptr, cxs[wave]);
    else col_tile_any<AccT, KB, DB, true>(ca, it, nullptr, cxs[wave]);
  }
}

// U = 4: five workgroups per CU (fewer loads in flight per wave, more
// panels in flight per CU); U = 8: as many as the registers allow.
template <typename AccT, int CAP, int U, int XF>
__global__ __launch_bounds__(256, U == 4 ? 5 : 1) void k_row(RowArgs<AccT> ra, const int32_t* order, int64_t n_panels,
                                             int64_t n_items) {
  __shared__ AccT zs[CAP];
  __shared__ AccT red[4][64];
  __shared__ __align__(16) uint32_t shs[(XF & kXfAflp) ? CAP : 4];
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int pi = panel_of(order, n_panels, it);
    if (pi < 0) continue;                           // uniform: whole workgroup
    __syncthreads();                                // LDS of the previous item
    const RowPanel P = ra.rp[pi];
    row_panel_part<AccT, CAP, U, XF>(ra, P, 0, P.nsec, 0, P.ncols, zs, red, shs);
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

// ---------------------------------------------------------------- launch

template <typename AccT, int U, int XF>
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
                   (int32_t)h.n_cols,
                   h.has_aflp ? reinterpret_cast<const int32_t*>(st + h.off_row_aflp) : nullptr};
  const AccT* sigma = h.has_sigma ? reinterpret_cast<const AccT*>(st + h.off_sigma) : nullptr;
  ColArgs<AccT> ca{st, reinterpret_cast<const ColTile*>(st + h.off_col_tiles),
                   reinterpret_cast<const int32_t*>(st + h.off_col_dst),
                   reinterpret_cast<const AccT*>(x), part, t, sigma,
                   h.has_aflp ? reinterpret_cast<const int32_t*>(st + h.off_col_aflp) : nullptr,
                   h.n_col_tiles};
  const bool grouped = A.launch.schedule == 1;
  const int ps = A.launch.persist, ncu = A.n_cu;
  if (ev) (void)hipEventRecord(ev[0], s);
  if (grouped) {
    if (h.n_p1 > 0)
      hipLaunchKernelGGL((k_p1<AccT, CAP, U, XF>), dim3(item_grid(h.n_p1, ps, ncu)), dim3(256), 0, s, ra,
                         ca, reinterpret_cast<const int32_t*>(st + h.off_p1_order), h.n_p1);
  } else {
    // classes: one-format IEEE tiles [0, ce[3]), one-format DFL tiles
    // [ce[3], ce[8]), one-format AFLP tiles [ce[8], ce[13]), one-format BFL
    // tiles [ce[13], ce[16]), several-format tiles [ce[16], ce[17])
    // (a wave per tile for the classes col_wave marks, or as colw says)
    const int64_t* ce = h.tile_class_end;
    auto wave_mode = [&](int bit) {
      return A.launch.colw == 2 || (A.launch.colw == 1 && ((A.col_wave >> bit) & 1u));
    };
    auto run = [&](auto kern, auto kern_w, int bit, int64_t t0, int64_t t1) {
      const int64_t n = t1 - t0;
      if (n <= 0) return;
      if (wave_mode(bit))
        hipLaunchKernelGGL(kern_w, dim3(item_grid((n + 3) / 4, ps, ncu)), dim3(256), 0, s, ca, t0, t1);
      else
        hipLaunchKernelGGL(kern, dim3(item_grid(n, ps, ncu)), dim3(256), 0, s, ca, t0, t1);
    };
    // two neighbouring classes that both run a wave per tile and both have
    // tiles share one launch (k_col_w2): classes bitA [a0, a1), bitB [a1, b1)
    auto pair = [&](auto kern2, int bitA, int64_t a0, int64_t a1, int bitB, int64_t b1) {
      if (a1 <= a0 || b1 <= a1 || !wave_mode(bitA) || !wave_mode(bitB)) return false;
      hipLaunchKernelGGL(kern2, dim3(item_grid((b1 - a0 + 3) / 4, ps, ncu)), dim3(256), 0, s, ca, a0, a1, b1);
      return true;
    };
    auto cls = [&](auto kern, auto kern_w, int c) { run(kern, kern_w, c, ce[c - 1], ce[c]); };   // one launch per class
    if constexpr ((XF & kXfDfl) != 0 && sizeof(AccT) == 8) {
      // DFL stores pair the IEEE class with DFL32 and DFL40 with DFL48 (a
      // pair of DFL16 and DFL24 was slower: DFL16 would lose a workgroup per CU)
      if (!pair(k_col_w2<AccT, kColIeee, -1, kColDfl, kDtDfl32>, 0, 0, ce[HM_BF16], kDtDfl32, ce[kDtDfl32])) {
        run(k_col<AccT, kColIeee>, k_col_w<AccT, kColIeee>, 0, 0, ce[HM_BF16]);
        cls(k_col<AccT, kColDfl, kDtDfl32>, k_col_w<AccT, kColDfl, kDtDfl32>, kDtDfl32);
      }
      if (!pair(k_col_w2<AccT, kColDfl, kDtDfl40, kColDfl, kDtDfl48>, kDtDfl40, ce[kDtDfl40 - 1], ce[kDtDfl40],
                kDtDfl48, ce[kDtDfl48])) {
        cls(k_col<AccT, kColDfl, kDtDfl40>, k_col_w<AccT, kColDfl, kDtDfl40>, kDtDfl40);
        cls(k_col<AccT, kColDfl, kDtDfl48>, k_col_w<AccT, kColDfl, kDtDfl48>, kDtDfl48);
      }
      cls(k_col<AccT, kColDfl, kDtDfl16>, k_col_w<AccT, kColDfl, kDtDfl16>, kDtDfl16);
      cls(k_col<AccT, kColDfl, kDtDfl24>, k_col_w<AccT, kColDfl, kDtDfl24>, kDtDfl24);
    } else {
      run(k_col<AccT, kColIeee>, k_col_w<AccT, kColIeee>, 0, 0, ce[HM_BF16]);
    }
    if constexpr ((XF & kXfAflp) != 0 && sizeof(AccT) == 8) {
      cls(k_col<AccT, kColAflp, kDtAflp16>, k_col_w<AccT, kColAflp, kDtAflp16>, kDtAflp16);
      cls(k_col<AccT, kColAflp, kDtAflp24>, k_col_w<AccT, kColAflp, kDtAflp24>, kDtAflp24);
      cls(k_col<AccT, kColAflp, kDtAflp32>, k_col_w<AccT, kColAflp, kDtAflp32>, kDtAflp32);
      cls(k_col<AccT, kColAflp, kDtAflp40>, k_col_w<AccT, kColAflp, kDtAflp40>, kDtAflp40);
      cls(k_col<AccT, kColAflp, kDtAflp48>, k_col_w<AccT, kColAflp, kDtAflp48>, kDtAflp48);
    }
    if constexpr ((XF & kXfBfl) != 0 && sizeof(AccT) == 8) {
      cls(k_col<AccT, kColBfl, kDtBfl24>, k_col_w<AccT, kColBfl, kDtBfl24>, kDtBfl24);
      cls(k_col<AccT, kColBfl, kDtBfl40>, k_col_w<AccT, kColBfl, kDtBfl40>, kDtBfl40);
      cls(k_col<AccT, kColBfl, kDtBfl48>, k_col_w<AccT, kColBfl, kDtBfl48>, kDtBfl48);
    }
    constexpr int KM = kColMulti | ((XF & kXfDfl) ? kColDfl : 0) | ((XF & kXfAflp) ? kColAflp : 0) |
                       ((XF & kXfBfl) ? kColBfl : 0);
    run(k_col<AccT, KM>, k_col_w<AccT, KM>, kNumDtypes, ce[kNumDtypes - 1], h.n_col_tiles);
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  if (h.n_col_tiles > 0) {
    RedArgs<AccT> rd{reinterpret_cast<const TBlock*>(st + h.off_tblocks),
                     reinterpret_cast<const int32_t*>(st + h.off_owner), sigma, part, t, h.n_large,
                     h.n_large_t, h.n_red_t};
    const int64_t nred = h.n_large + (h.n_red_t - h.n_large_t + 255) / 256;
    if (nred > 0) hipLaunchKernelGGL(k_reduce<AccT>, dim3((unsigned)nred), dim3(256), 0, s, rd);
  }
  if (ev) (void)hipEventRecord(ev[2], s);
  if (grouped) {
    if (h.n_p2 > 0)
      hipLaunchKernelGGL((k_p2<AccT, CAP, U, XF>), dim3(item_grid(h.n_p2, ps, ncu)), dim3(256), 0, s, ra,
                         reinterpret_cast<const int32_t*>(st + h.off_p2_order), h.n_p2);
  } else if (h.n_row_panels > 0) {
    const bool xcd = A.launch.order == 1;
    const int64_t items = panel_items(xcd, h.n_row_panels);
    hipLaunchKernelGGL((k_row<AccT, CAP, U, XF>), dim3(item_grid(items, ps, ncu)), dim3(256), 0, s, ra,
                       xcd ? nullptr : reinterpret_cast<const int32_t*>(st + h.off_row_order),
                       h.n_row_panels, items);
  }
  if (ev) (void)hipEventRecord(ev[3], s);
  return hipGetLastError();
}

// DFL / AFLP / BFL instantiations (FP64 accumulation only) run when the
// store holds such bytes; a store with several of these families runs
// instantiations that decode all of them present.
template <typename AccT>
hipError_t launch_typed(const hm_matrix& A, double alpha, const void* x, void* y, void* work,
                        hipStream_t s, hipEvent_t* ev) {
  const bool u8 = A.launch.row_unroll >= 8;
  if constexpr (sizeof(AccT) == 8) {
    bool dfl = false, aflp = false, bfl = false;
    for (int d = 0; d < kNumDtypes; ++d) {
      dfl = dfl || (is_dfl(d) && A.bytes_by_dtype[d] > 0);
      aflp = aflp || (is_aflp(d) && A.bytes_by_dtype[d] > 0);
      bfl = bfl || (is_bfl(d) && A.bytes_by_dtype[d] > 0);
    }
    constexpr int kAll = kXfDfl | kXfAflp | kXfBfl;
    if (bfl && (dfl || aflp))
      return u8 ? launch_typed_u<AccT, 8, kAll>(A, alpha, x, y, work, s, ev)
                : launch_typed_u<AccT, 4, kAll>(A, alpha, x, y, work, s, ev);
    if (bfl)
      return u8 ? launch_typed_u<AccT, 8, kXfBfl>(A, alpha, x, y, work, s, ev)
                : launch_typed_u<AccT, 4, kXfBfl>(A, alpha, x, y, work, s, ev);
    if (aflp && dfl)
      return u8 ? launch_typed_u<AccT, 8, kXfDfl | kXfAflp>(A, alpha, x, y, work, s, ev)
                : launch_typed_u<AccT, 4, kXfDfl | kXfAflp>(A, alpha, x, y, work, s, ev);
    if (aflp)
      return u8 ? launch_typed_u<AccT, 8, kXfAflp>(A, alpha, x, y, work, s, ev)
                : launch_typed_u<AccT, 4, kXfAflp>(A, alpha, x, y, work, s, ev);
    if (dfl)
      return u8 ? launch_typed_u<AccT, 8, kXfDfl>(A, alpha, x, y, work, s, ev)
                : launch_typed_u<AccT, 4, kXfDfl>(A, alpha, x, y, work, s, ev);
  }
  return u8 ? launch_typed_u<AccT, 8, 0>(A, alpha, x, y, work, s, ev)
            : launch_typed_u<AccT, 4, 0>(A, alpha, x, y, work, s, ev);
}

}  // namespace

hipError_t launch_mvm(const hm_matrix& A, double alpha, const void* x, void* y, void* work,
                      hipStream_t s, hipEvent_t* ev, bool profile) {
  if (profile && !ev && A.prof.on && A.prof.calls < A.prof.max_calls)
    ev = &A.prof.ev[4 * (size_t)A.prof.calls++];
  return A.acc_dtype == HM_F64 ? launch_typed<double>(A, alpha, x, y, work, s, ev)
                               : launch_typed<float>(A, alpha, x, y, work, s, ev);
}

// Fixed workspace of hm_mvm_noalloc, for callers that cannot allocate device
// memory: one copy of this array on every GPU the library runs on, held
// until the process ends.  In host code the name `scratch` denotes a
// host-side stand-in, not device memory, so it is never passed to a kernel
// or a copy: host code uses the device address that hipGetSymbolAddress
// returns, looked up once per device with that device current and kept
// here.  The product writes every partial sum and t entry it reads within
// the same call, so the array needs no clearing between calls.
static __device__ __align__(256) uint8_t scratch[HM_NOALLOC_SCRATCH_BYTES];

hipError_t scratch_address(int device, void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
}

hipError_t launch_stream_read(const void* buf, size_t bytes, void* out, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  const int64_t per_block = 256 * 8;
  const int64_t blocks = std::min<int64_t>((n16 + per_block - 1) / per_block, 256 * 16);
  hipLaunchKernelGGL(k_stream_read, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s,
                     static_cast<const u32x4*>(buf), n16, static_cast<unsigned*>(out));
  return hipGetLastError();
}

}  // namespace hm
