// Host side of libhm: block-table validation, the block scheduler (panel
// and work-list construction), the store layout, packing with RNE format
// conversion, and the C-ABI entry points that enqueue the HIP kernels.
//
// Paper references (Kriemann, "Hierarchical Lowrank Arithmetic with Binary
// Compression"): leaf partition of I x J (Sec. 2.1, Definition "Block
// Tree"); dense and low-rank leaves (Definition "H-Matrix", Eq. (1)); U and
// V stored separately (Sec. 3); column groups per format with singular
// values (Sec. 3.3); formats of Table 1; conversion after assembly
// (Sec. 5.3).

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/hm.h"
#include "hm_internal.hpp"

namespace hm {

thread_local std::string g_err;

hm_status fail(hm_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

hm_status ok() {
  g_err.clear();
  return HM_OK;
}

static inline int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// ------------------------------------------------------------------ rounding
// Round-to-nearest-even from FP64 straight to the storage format (one
// rounding), on the IEEE-754 bit patterns.  Formats per Table 1.

static uint16_t round_bits(double d, int man_bits, int bias, int exp_max_field) {
  uint64_t b;
  std::memcpy(&b, &d, 8);
  const int total = 1 + (exp_max_field == 31 ? 5 : 8) + man_bits;
  const uint16_t sign = (uint16_t)((b >> 63) << (total - 1));
  const int e = (int)((b >> 52) & 0x7ff);
  const uint64_t man = b & ((1ull << 52) - 1);
  const uint16_t inf = (uint16_t)(exp_max_field << man_bits);
  if (e == 0x7ff) return sign | inf | (man ? (uint16_t)(1u << (man_bits - 1)) : 0);
  if (e == 0) return sign;                       // FP64 subnormal: far below any target
  const int E = e - 1023;
  const int emin = 1 - bias;
  const uint64_t sig = man | (1ull << 52);
  int shift, field;
  if (E >= emin) { shift = 52 - man_bits; field = E + bias; }
  else { shift = 52 - man_bits + (emin - E); field = 0; }
  if (shift > 63) return sign;
  uint64_t kept = sig >> shift;
  const uint64_t rem = sig & ((1ull << shift) - 1);
  const uint64_t half = 1ull << (shift - 1);
  if (rem > half || (rem == half && (kept & 1))) ++kept;
  if (field == 0) return sign | (uint16_t)kept;  // subnormal (a carry gives the min normal)
  if (kept == (1ull << (man_bits + 1))) { kept >>= 1; ++field; }
  if (field >= exp_max_field) return sign | inf;
  return sign | (uint16_t)(field << man_bits) | (uint16_t)(kept & ((1ull << man_bits) - 1));
}

uint16_t f64_to_f16(double d) { return round_bits(d, 10, 15, 31); }
uint16_t f64_to_bf16(double d) { return round_bits(d, 7, 127, 255); }

// DFL (Sec. 3.2): the leading nbytes bytes of the FP64 encoding, rounded to
// nearest even on the bit pattern (a carry out of the mantissa moves into
// the exponent, as the rounding of the value requires).  Returns the
// rounded encoding with the dropped bits zero.
static uint64_t dfl_bits(double v, int nbytes) {
  uint64_t b;
  std::memcpy(&b, &v, 8);
  const int drop = 64 - 8 * nbytes;
  if (((b >> 52) & 0x7ff) == 0x7ff)                // Inf stays Inf; NaN stays a (quiet) NaN
    return (b & ~((1ull << drop) - 1)) | ((b & ((1ull << 52) - 1)) ? (1ull << 51) : 0);
  uint64_t kept = b >> drop;
  const uint64_t rem = b & ((1ull << drop) - 1), half = 1ull << (drop - 1);
  if (rem > half || (rem == half && (kept & 1))) ++kept;
  return kept << drop;
}

// AFLP (Sec. 3.2) parameter of one data block of nbytes-byte values (the
// n values v[i * inc], i < n; see aflp_param): k with 2^k at or below the
// smallest nonzero magnitude, and the fewest exponent bits e whose field
// holds the binary exponent of every rounded d = |v| 2^-k + 1.  Fails for
// values that are not finite or a range that needs more than 10 bits.
static uint64_t rne_mantissa(uint64_t bits, int m) {   // positive normal FP64, m explicit bits
  const int drop = 52 - m;
  uint64_t kept = bits >> drop;
  const uint64_t rem = bits & ((1ull << drop) - 1), half = 1ull << (drop - 1);
  if (rem > half || (rem == half && (kept & 1))) ++kept;   // a carry moves into the exponent
  return kept << drop;
}
static bool aflp_block_param(const double* v, int64_t rows, int64_t cols, int64_t ld, int nbytes, int32_t* out) {
  double mn = HUGE_VAL, mx = 0;
  for (int64_t j = 0; j < cols; ++j)
    for (int64_t i = 0; i < rows; ++i) {
      const double a = std::fabs(v[j * ld + i]);
      if (!std::isfinite(a)) return false;
      if (a > 0) { mn = std::min(mn, a); mx = std::max(mx, a); }
    }
  if (mx == 0) { *out = aflp_param(0, 0); return true; }
  int k;
  (void)std::frexp(mn, &k);
  k -= 1;                                          // 2^k <= mn < 2^(k+1)
  const double dmax = std::ldexp(mx, -k) + 1.0;
  if (!std::isfinite(dmax)) return false;
  uint64_t b;
  std::memcpy(&b, &dmax, 8);
  const int top = (int)(b >> 52) - 1023;           // binary exponent of the largest d (>= 1)
  int e = 0;
  while ((1 << e) <= top) ++e;
  for (;; ++e) {
    const int m = 8 * nbytes - 1 - e;
    if (e > 10 || m < 1) return false;
    if ((int)(rne_mantissa(b, m) >> 52) - 1023 < (1 << e)) break;
  }
  *out = aflp_param(k, e);
  return true;
}

// The left-aligned 64-bit AFLP code of v (sign, e exponent bits, m mantissa
// bits of the rounded d; the low 64 - 8 nbytes bits zero).
static uint64_t aflp_code(double v, int32_t prm, int nbytes) {
  if (v == 0) return 0;
  const int k = aflp_scale_exp(prm), sh = aflp_shift(prm), e = 11 - sh, m = 8 * nbytes - 1 - e;
  const double d = std::ldexp(std::fabs(v), -k) + 1.0;
  uint64_t b;
  std::memcpy(&b, &d, 8);
  const uint64_t mag = (rne_mantissa(b, m) - 0x3ff0000000000000ull) << sh;
  return (std::signbit(v) ? 1ull << 63 : 0) | mag;
}

// The left-aligned 64-bit BFL code of v in nbytes bytes (see kBflRebias);
// false for a value that is not finite or rounds to 2^128 or beyond.
static bool bfl_code(double v, int nbytes, uint64_t* out) {
  if (!std::isfinite(v)) return false;
  uint64_t b;
  std::memcpy(&b, &v, 8);
  const uint64_t sign = b & (1ull << 63), mag = b & ~(1ull << 63);
  *out = 0;
  if (mag == 0) return true;
  const uint64_t r = rne_mantissa(mag, 8 * nbytes - 9);
  const int e8 = (int)(r >> 52) - 896;             // FP32's biased exponent
  if (e8 >= 255) return false;
  if (e8 >= 1) *out = sign | ((r - kBflRebias) << 3);
  return true;                                     // below 2^-126: zero
}

// A left-aligned 64-bit code r of a DFL, AFLP or BFL value: its leading 4 bytes
// (32 / 40 / 48-bit formats: the high word) or 2 bytes (16 / 24-bit
// formats) at hi; for the 40 / 48 / 24-bit formats bits 31..24 / 31..16 /
// 47..40 at lo.
static inline void put_code(uint8_t* hi, uint8_t* lo, int dt, uint64_t r) {
  dt = storage_dt(dt);
  if (dtype_size(dt) == 4) {
    const uint32_t w = (uint32_t)(r >> 32);
    std::memcpy(hi, &w, 4);
  } else {
    const uint16_t w = (uint16_t)(r >> 48);
    std::memcpy(hi, &w, 2);
  }
  if (dt == kDtDfl40) { const uint8_t q = (uint8_t)(r >> 24); std::memcpy(lo, &q, 1); }
  if (dt == kDtDfl48) { const uint16_t q = (uint16_t)(r >> 16); std::memcpy(lo, &q, 2); }
  if (dt == kDtDfl24) { const uint8_t q = (uint8_t)(r >> 40); std::memcpy(lo, &q, 1); }
}

// The BFL code of a value the pre-pass has checked (see bfl_code).
static inline uint64_t bfl_or_zero(double v, int nbytes) {
  uint64_t c;
  return bfl_code(v, nbytes, &c) ? c : 0;
}

static inline void put_dfl(uint8_t* hi, uint8_t* lo, int dt, double v) {
  put_code(hi, lo, dt, dfl_bits(v, value_bytes(dt)));
}

static inline void put(uint8_t* dst, int dt, double v) {
  switch (dt) {
    case HM_F64: std::memcpy(dst, &v, 8); break;
    case HM_F32: { float f = (float)v; std::memcpy(dst, &f, 4); break; }
    case HM_F16: { uint16_t h = f64_to_f16(v); std::memcpy(dst, &h, 2); break; }
    case HM_BF16: { uint16_t h = f64_to_bf16(v); std::memcpy(dst, &h, 2); break; }
    default: put_dfl(dst, nullptr, HM_DFL32, v); break;   // callers of put: no low-byte plane
  }
}

// ------------------------------------------------------------------ plan

static hm_status validate_block(const hm_block_desc& b, int64_t i, int64_t n_rows, int64_t n_cols,
                                int acc) {
  if (b.row_begin < 0 || b.row_end > n_rows || b.row_begin >= b.row_end || b.col_begin < 0 ||
      b.col_end > n_cols || b.col_begin >= b.col_end)
    return fail(HM_ESHAPE, "block %lld: range [%lld,%lld)x[%lld,%lld) outside or empty",
                (long long)i, (long long)b.row_begin, (long long)b.row_end,
                (long long)b.col_begin, (long long)b.col_end);
  if (b.row_end - b.row_begin > INT32_MAX / 2 || b.col_end - b.col_begin > INT32_MAX / 2)
    return fail(HM_ESHAPE, "block %lld too large", (long long)i);
  auto dt_ok = [&](int dt) {
    if (dt < HM_F64 || dt >= kNumDtypes) return false;
    if (acc == HM_F32 && (dt == HM_F64 || is_dfl(dt) || is_aflp(dt) || is_bfl(dt))) return false;
    return true;
  };
  if (b.kind == HM_DENSE) {
    if (b.rank != 0) return fail(HM_ESHAPE, "block %lld: dense block with rank %d", (long long)i, b.rank);
    if (b.ngroups != 1) return fail(HM_ESHAPE, "block %lld: dense block needs ngroups = 1", (long long)i);
    if (!dt_ok(b.group_dtype[0]))
      return fail(HM_EDTYPE, "block %lld: storage dtype %d not allowed", (long long)i, b.group_dtype[0]);
    if (b.has_sigma) return fail(HM_ESHAPE, "block %lld: dense block with has_sigma", (long long)i);
    return HM_OK;
  }
  if (b.kind != HM_LOWRANK) return fail(HM_EINVAL, "block %lld: unknown kind %d", (long long)i, b.kind);
  if (b.rank < 0) return fail(HM_ESHAPE, "block %lld: negative rank", (long long)i);
  const int64_t m = b.row_end - b.row_begin, n = b.col_end - b.col_begin;
  if (b.rank > std::min(m, n)) return fail(HM_ESHAPE, "block %lld: rank %d exceeds min(m,n)", (long long)i, b.rank);
  if (b.ngroups < 0 || b.ngroups > 4 || (b.rank > 0 && b.ngroups < 1))
    return fail(HM_ESHAPE, "block %lld: ngroups %d", (long long)i, b.ngroups);
  int64_t sum = 0;
  for (int g = 0; g < b.ngroups; ++g) {
    if (b.group_cols[g] < 0) return fail(HM_ESHAPE, "block %lld: negative group size", (long long)i);
    if (!dt_ok(b.group_dtype[g]))
      return fail(HM_EDTYPE, "block %lld: storage dtype %d not allowed", (long long)i, b.group_dtype[g]);
    sum += b.group_cols[g];
  }
  if (sum != b.rank) return fail(HM_ESHAPE, "block %lld: group sizes sum to %lld, rank %d",
                                 (long long)i, (long long)sum, b.rank);
  if (b.has_sigma != 0 && b.has_sigma != 1) return fail(HM_EINVAL, "block %lld: has_sigma", (long long)i);
  return HM_OK;
}

// Elementary intervals from sorted unique breakpoints, split to <= cap.
static void split_intervals(const std::vector<int64_t>& bp, int cap, std::vector<int64_t>& out,
                            std::vector<int32_t>& parent) {
  out.clear();
  parent.clear();
  for (size_t q = 0; q + 1 < bp.size(); ++q) {
    int64_t a = bp[q], len = bp[q + 1] - bp[q];
    int64_t pieces = (len + cap - 1) / cap;
    for (int64_t p = 0; p < pieces; ++p) {
      out.push_back(a + len * p / pieces);
      parent.push_back((int32_t)q);
    }
  }
  out.push_back(bp.back());
}

// Byte offset of element (row i, column sc of run S) of column panel Cp.
// The panel's groups (run by run) are stored tile by tile (tiles of 64
// groups, the last one narrower); inside a tile, row i holds the tile's
// groups contiguously, so a tile row is one contiguous block.
// Cuts a column panel's group sequence (its runs, in order) into tiles of
// at most kTileGroups groups and at most 4 runs (the tile descriptor's
// limit); with one_format, every run starts a tile of its own.  A tile's low-byte plane has one entry of tile_lo[t] bytes (the
// largest lo_bytes of its runs; 0: none) per row and group; groups of a
// format without one leave theirs unused.  Fills tile_g0 / tile_off /
// tile_lo.
static void cut_tiles(ColPanelHost& Cp, int32_t tile_groups, bool one_format) {
  Cp.tile_g0.assign(1, 0);
  Cp.tile_off.assign(1, 0);
  Cp.tile_lo.clear();
  int32_t open = 0, runs = 0, L = 0;                // the open tile: groups, runs, entry bytes
  auto close = [&]() {
    Cp.tile_g0.push_back(Cp.tile_g0.back() + open);
    Cp.tile_off.push_back(Cp.tile_off.back() + (int64_t)open * Cp.nrows * (16 + L));
    Cp.tile_lo.push_back(L);
    open = runs = L = 0;
  };
  for (auto& S : Cp.secs) {
    const int32_t n = S.ld / group_width(S.dtype);
    if (one_format && open > 0) close();
    for (int32_t g = 0; g < n;) {
      if (runs == 4) close();
      const int32_t take = std::min(tile_groups - open, n - g);
      open += take;
      g += take;
      ++runs;
      L = std::max(L, lo_bytes(S.dtype));
      if (open == tile_groups) close();
    }
  }
  if (open > 0) close();
}

// Tile of group g of column panel Cp.
static int64_t tile_of(const ColPanelHost& Cp, int64_t g) {
  return std::upper_bound(Cp.tile_g0.begin(), Cp.tile_g0.end(), (int32_t)g) - Cp.tile_g0.begin() - 1;
}

static int64_t col_elem_offset(const ColPanelHost& Cp, const ColSectionHost& S, int64_t i, int64_t sc) {
  const int G = group_width(S.dtype), sz = dtype_size(S.dtype);
  const int64_t g = S.g0 + sc / G, t = tile_of(Cp, g), gl = g - Cp.tile_g0[t];
  const int64_t ngt = Cp.tile_g0[t + 1] - Cp.tile_g0[t];
  return Cp.data_off + Cp.tile_off[t] + (i * ngt + gl) * 16 + (sc % G) * sz;
}

// Byte offset of the low-byte part of that element (formats with lo_bytes > 0).
static int64_t col_lo_offset(const ColPanelHost& Cp, const ColSectionHost& S, int64_t i, int64_t sc) {
  const int G = group_width(S.dtype), L = lo_bytes(S.dtype);
  const int64_t g = S.g0 + sc / G, t = tile_of(Cp, g), gl = g - Cp.tile_g0[t];
  const int64_t ngt = Cp.tile_g0[t + 1] - Cp.tile_g0[t];
  return Cp.data_off + Cp.tile_off[t] + 16 * ngt * (int64_t)Cp.nrows + (i * ngt + gl) * Cp.tile_lo[t] +
         (sc % G) * (L / G);
}

static int rank_class(const hm_plan* P);

hm_status build_plan(int64_t n_rows, int64_t n_cols, const hm_block_desc* blocks, int64_t nb,
                     const hm_plan_opts* o, hm_plan** out) {
  if (!out) return fail(HM_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_rows <= 0 || n_cols <= 0 || n_rows > INT32_MAX / 4 || n_cols > INT32_MAX / 4)
    return fail(HM_EINVAL, "bad matrix size %lld x %lld", (long long)n_rows, (long long)n_cols);
  if (nb <= 0 || !blocks) return fail(HM_EINVAL, "empty block table");
  hm_plan_opts opts{HM_F64, HM_F64, 1, 0, nullptr, 0, 0, 0};
  if (o) opts = *o;
  if (opts.acc_dtype != HM_F64 && opts.acc_dtype != HM_F32)
    return fail(HM_EDTYPE, "acc_dtype must be HM_F64 or HM_F32");
  if (opts.vec_dtype != opts.acc_dtype) return fail(HM_EDTYPE, "vec_dtype must equal acc_dtype");
  if (opts.max_nrhs < 1 || opts.max_nrhs > 4096) return fail(HM_EINVAL, "max_nrhs out of range");
  const int acc = opts.acc_dtype;

  auto P = std::make_unique<hm_plan>();
  P->n_rows = n_rows;
  P->n_cols = n_cols;
  P->opts = opts;
  P->tune_path = opts.tune_cache ? opts.tune_cache : "";
  P->opts.tune_cache = nullptr;
  P->blocks.assign(blocks, blocks + nb);
  for (int64_t i = 0; i < nb; ++i) {
    hm_status st = validate_block(P->blocks[i], i, n_rows, n_cols, acc);
    if (st) return st;
  }
  // launch parameters and tile shape of this kind of matrix from the tune
  // cache, then the tile shape the caller gives
  P->rank_class = rank_class(P.get());
  if (opts.tune && !P->tune_path.empty()) read_tune_cache(P.get());
  if (opts.chunk_rows < 0 || opts.tile_groups < 0) return fail(HM_EINVAL, "negative tile shape");
  P->chunk_rows = opts.chunk_rows ? opts.chunk_rows : P->launch.chunk ? P->launch.chunk : kSegRows;
  P->tile_groups = opts.tile_groups ? opts.tile_groups : P->launch.tile ? P->launch.tile : kTileGroups;
  if (P->chunk_rows < kMaxTileRows || P->chunk_rows > kSegRows)
    return fail(HM_EINVAL, "chunk_rows %d outside [%d, %d]", P->chunk_rows, kMaxTileRows, kSegRows);
  if (P->tile_groups < 8 || P->tile_groups > kTileGroups)
    return fail(HM_EINVAL, "tile_groups %d outside [8, %d]", P->tile_groups, kTileGroups);
  P->launch.chunk = P->chunk_rows;
  P->launch.tile = P->tile_groups;
  if (opts.tile_mix < 0 || opts.tile_mix > 2) return fail(HM_EINVAL, "tile_mix %d outside [0, 2]", opts.tile_mix);
  if (opts.tile_mix) P->launch.tmix = opts.tile_mix - 1;

  // ---- elementary row intervals and the tiling proof
  std::vector<int64_t> rbp;
  rbp.reserve(2 * nb + 2);
  for (auto& b : P->blocks) { rbp.push_back(b.row_begin); rbp.push_back(b.row_end); }
  std::sort(rbp.begin(), rbp.end());
  rbp.erase(std::unique(rbp.begin(), rbp.end()), rbp.end());
  if (rbp.front() != 0 || rbp.back() != n_rows)
    return fail(HM_EPARTITION, "rows [0,%lld) are not covered", (long long)n_rows);
  const int64_t nri = (int64_t)rbp.size() - 1;
  std::vector<int64_t> cnt(nri + 1, 0);
  std::vector<int32_t> bi0(nb), bi1(nb);
  for (int64_t i = 0; i < nb; ++i) {
    bi0[i] = (int32_t)(std::lower_bound(rbp.begin(), rbp.end(), P->blocks[i].row_begin) - rbp.begin());
    bi1[i] = (int32_t)(std::lower_bound(rbp.begin(), rbp.end(), P->blocks[i].row_end) - rbp.begin());
    for (int32_t q = bi0[i]; q < bi1[i]; ++q) cnt[q + 1]++;
  }
  for (int64_t q = 0; q < nri; ++q) cnt[q + 1] += cnt[q];
  std::vector<int32_t> cover(cnt[nri]);
  {
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < nb; ++i)
      for (int32_t q = bi0[i]; q < bi1[i]; ++q) cover[fill[q]++] = (int32_t)i;
  }
  for (int64_t q = 0; q < nri; ++q) {
    auto first = cover.begin() + cnt[q], last = cover.begin() + cnt[q + 1];
    std::sort(first, last, [&](int32_t a, int32_t b) {
      return P->blocks[a].col_begin < P->blocks[b].col_begin;
    });
    int64_t c = 0;
    for (auto it = first; it != last; ++it) {
      const auto& b = P->blocks[*it];
      if (b.col_begin != c)
        return fail(HM_EPARTITION, "rows [%lld,%lld): columns %s at %lld (block %d)",
                    (long long)rbp[q], (long long)rbp[q + 1],
                    b.col_begin < c ? "overlap" : "gap", (long long)c, *it);
      c = b.col_end;
    }
    if (c != n_cols)
      return fail(HM_EPARTITION, "rows [%lld,%lld): columns [%lld,%lld) not covered",
                  (long long)rbp[q], (long long)rbp[q + 1], (long long)c, (long long)n_cols);
  }

  // ---- low-rank blocks: column chunks, t and partial offsets
  // The rows of each V_b are cut into chunks: sigma_b itself when it has at
  // most chunk_rows rows, else the largest sub-ranges of sigma_b with at most
  // chunk_rows rows among the block ranges (for a block tree these are the
  // clusters of the cluster tree), recursively.  A range that has no
  // sub-ranges covering it, or a family of ranges that is not nested, falls
  // back to near-equal pieces of at most 64 rows.  Equal ranges always get
  // equal chunks, so every chunk is shared by all blocks over it.
  std::vector<std::pair<int64_t, int64_t>> rng;
  rng.reserve(2 * nb);
  for (auto& b : P->blocks) {
    rng.push_back({b.row_begin, b.row_end});
    rng.push_back({b.col_begin, b.col_end});
  }
  std::sort(rng.begin(), rng.end(), [](const std::pair<int64_t, int64_t>& x,
                                       const std::pair<int64_t, int64_t>& y) {
    return x.first != y.first ? x.first < y.first : x.second > y.second;
  });
  rng.erase(std::unique(rng.begin(), rng.end()), rng.end());
  std::vector<std::vector<int32_t>> kids(rng.size());
  bool laminar = true;
  {
    std::vector<int32_t> stack;
    for (int32_t r = 0; r < (int32_t)rng.size(); ++r) {
      while (!stack.empty() && !(rng[stack.back()].second >= rng[r].second)) {
        if (rng[stack.back()].second > rng[r].first) laminar = false;   // crossing ranges
        stack.pop_back();
      }
      if (!stack.empty()) kids[stack.back()].push_back(r);
      stack.push_back(r);
    }
  }
  auto find_range = [&](int64_t b0, int64_t e0) -> int32_t {
    auto it = std::lower_bound(rng.begin(), rng.end(), std::make_pair(b0, e0),
                               [](const std::pair<int64_t, int64_t>& x, const std::pair<int64_t, int64_t>& y) {
                                 return x.first != y.first ? x.first < y.first : x.second > y.second;
                               });
    return (it != rng.end() && *it == std::make_pair(b0, e0)) ? (int32_t)(it - rng.begin()) : -1;
  };
  std::map<std::pair<int64_t, int64_t>, int32_t> chunk_id;
  std::vector<std::pair<int64_t, int64_t>> chunks;
  auto add_chunk = [&](int64_t b0, int64_t e0) {
    auto key = std::make_pair(b0, e0);
    auto it = chunk_id.find(key);
    if (it != chunk_id.end()) return it->second;
    const int32_t id = (int32_t)chunks.size();
    chunk_id.emplace(key, id);
    chunks.push_back(key);
    return id;
  };
  std::function<void(int64_t, int64_t, std::vector<int32_t>&)> chunk_range =
      [&](int64_t b0, int64_t e0, std::vector<int32_t>& out) {
        if (e0 - b0 <= P->chunk_rows) { out.push_back(add_chunk(b0, e0)); return; }
        const int32_t r = laminar ? find_range(b0, e0) : -1;
        if (r >= 0 && !kids[r].empty()) {
          int64_t covered = b0;
          for (int32_t c : kids[r]) {
            if (rng[c].first != covered) { covered = -1; break; }
            covered = rng[c].second;
          }
          if (covered == e0) {
            for (int32_t c : kids[r]) chunk_range(rng[c].first, rng[c].second, out);
            return;
          }
        }
        const int64_t pieces = (e0 - b0 + kMaxTileRows - 1) / kMaxTileRows;
        for (int64_t q = 0; q < pieces; ++q)
          out.push_back(add_chunk(b0 + (e0 - b0) * q / pieces, b0 + (e0 - b0) * (q + 1) / pieces));
      };
  P->binfo.assign(nb, BlockInfo{});
  P->chunk_off.assign(nb + 1, 0);
  std::vector<int32_t> lr_large, lr_multi, lr_single;
  {
    std::map<std::pair<int64_t, int64_t>, std::vector<int32_t>> memo;   // sigma -> chunk list
    for (int64_t i = 0; i < nb; ++i) {
      const auto& b = P->blocks[i];
      P->chunk_off[i + 1] = P->chunk_off[i];
      if (b.kind != HM_LOWRANK || b.rank == 0) continue;
      auto key = std::make_pair(b.col_begin, b.col_end);
      auto it = memo.find(key);
      if (it == memo.end()) {
        std::vector<int32_t> out;
        chunk_range(b.col_begin, b.col_end, out);
        it = memo.emplace(key, std::move(out)).first;
      }
      P->chunk_list.insert(P->chunk_list.end(), it->second.begin(), it->second.end());
      P->chunk_off[i + 1] = (int64_t)P->chunk_list.size();
      BlockInfo& bi = P->binfo[i];
      bi.nseg = (int32_t)it->second.size();
      (bi.nseg > kLargeSeg ? lr_large : bi.nseg > 1 ? lr_multi : lr_single).push_back((int32_t)i);
    }
  }
  // t: blocks over many chunks, over a few, inside one; partials only for
  // the first two classes (a block inside one chunk gets t from its tiles)
  int64_t toff = 0, pst = 0;
  for (const auto* cls : {&lr_large, &lr_multi, &lr_single})
    for (int32_t i : *cls) {
      BlockInfo& bi = P->binfo[i];
      bi.toff = toff;
      toff += P->blocks[i].rank;
      if (cls == &lr_single) {
        bi.pst = -1;
      } else {
        bi.pst = pst;
        pst += (int64_t)bi.nseg * P->blocks[i].rank;
      }
    }
  if (toff + n_cols > INT32_MAX || pst > INT32_MAX)
    return fail(HM_ENOMEM, "too many low-rank entries for 32-bit indices");
  P->n_t = toff;
  P->n_partials = pst;
  P->n_large = (int64_t)lr_large.size();
  P->n_large_t = 0;
  for (int32_t i : lr_large) P->n_large_t += P->blocks[i].rank;
  P->n_red_t = P->n_large_t;
  for (int32_t i : lr_multi) P->n_red_t += P->blocks[i].rank;
  P->lr_order.reserve(lr_large.size() + lr_multi.size() + lr_single.size());
  for (const auto* cls : {&lr_large, &lr_multi, &lr_single})
    P->lr_order.insert(P->lr_order.end(), cls->begin(), cls->end());
  P->has_sigma = 0;
  for (auto& b : P->blocks)
    if (b.kind == HM_LOWRANK && b.rank > 0 && b.has_sigma) P->has_sigma = 1;

  // ---- row panels
  std::vector<int32_t> rparent;
  split_intervals(rbp, kMaxPanelRows, P->rint, rparent);
  const int64_t nrp = (int64_t)P->rint.size() - 1;
  P->rps.resize(nrp);
  for (int64_t p = 0; p < nrp; ++p) {
    RowPanelHost& R = P->rps[p];
    R.row0 = P->rint[p];
    R.m = (int32_t)(P->rint[p + 1] - P->rint[p]);
    const int32_t q = rparent[p];
    std::vector<Seg> segs;
    for (int64_t c = cnt[q]; c < cnt[q + 1]; ++c) {
      const int32_t i = cover[c];
      const auto& b = P->blocks[i];
      if (b.kind == HM_DENSE) {
        segs.push_back(Seg{i, 0, (int32_t)(b.col_end - b.col_begin), (int32_t)b.col_begin,
                           b.group_dtype[0], 0, HM_DENSE});
      } else if (b.rank > 0) {
        int32_t c0 = 0;
        for (int g = 0; g < b.ngroups; ++g) {
          if (b.group_cols[g] > 0)
            segs.push_back(Seg{i, c0, b.group_cols[g],
                               (int32_t)(n_cols + P->binfo[i].toff + c0), b.group_dtype[g], 0,
                               HM_LOWRANK});
          c0 += b.group_cols[g];
        }
      }
    }
    // sections: dense blocks first, then U factors, each by dtype; every
    // section starts at a multiple of 8 source slots
    int32_t slot = 0;
    for (int kind = 0; kind < 2; ++kind)
      for (int dt = 0; dt < kNumDtypes; ++dt) {
        int32_t cols = 0;
        for (auto& s : segs)
          if (s.kind == kind && s.dtype == dt) { s.seccol = cols; cols += s.ncols; }
        if (cols == 0) continue;
        const int G = group_width(dt);
        RowSectionHost S;
        S.kind = kind;
        S.dtype = dt;
        S.ngroups = (cols + G - 1) / G;
        S.col0 = slot;
        slot += align_up(S.ngroups * G, 8);
        R.secs.push_back(S);
        if (kind == 0) R.nsec_dense++;
      }
    R.ncols = slot;
    R.segs = std::move(segs);
  }

  // ---- column panels (one per chunk) and their sections
  const int64_t nck = (int64_t)chunks.size();
  std::vector<int64_t> ccnt(nck + 1, 0);
  for (int64_t i = 0; i < nb; ++i)
    for (int64_t q = P->chunk_off[i]; q < P->chunk_off[i + 1]; ++q) ccnt[P->chunk_list[q] + 1]++;
  for (int64_t q = 0; q < nck; ++q) ccnt[q + 1] += ccnt[q];
  std::vector<int32_t> ccover(nck ? ccnt[nck] : 0), cseg(nck ? ccnt[nck] : 0);
  {
    std::vector<int64_t> fill(ccnt.begin(), ccnt.end() - 1);
    for (int64_t i = 0; i < nb; ++i)               // ascending block index: reproducible order
      for (int64_t q = P->chunk_off[i]; q < P->chunk_off[i + 1]; ++q) {
        const int32_t c = P->chunk_list[q];
        ccover[fill[c]] = (int32_t)i;
        cseg[fill[c]++] = (int32_t)(q - P->chunk_off[i]);
      }
  }
  P->cps.resize(nck);
  for (int64_t q = 0; q < nck; ++q) {
    ColPanelHost& Cp = P->cps[q];
    Cp.x0 = chunks[q].first;
    Cp.nrows = (int32_t)(chunks[q].second - chunks[q].first);
    if (Cp.nrows < 1 || Cp.nrows > kSegRows)           // the kernels stage a chunk's x in LDS
      return fail(HM_EINVAL, "internal error: column chunk of %d rows", Cp.nrows);
    for (int64_t c = ccnt[q]; c < ccnt[q + 1]; ++c) {
      const int32_t i = ccover[c];
      const auto& b = P->blocks[i];
      const BlockInfo& bi = P->binfo[i];
      const int32_t seg = cseg[c];
      int32_t c0 = 0;
      const bool direct = bi.nseg == 1;
      for (int g = 0; g < b.ngroups; ++g) {
        if (b.group_cols[g] > 0)
          Cp.segs.push_back(Seg{i, c0, b.group_cols[g],
                                (int32_t)(direct ? bi.toff + c0 : bi.pst + (int64_t)seg * b.rank + c0),
                                b.group_dtype[g], 0, HM_LOWRANK, direct ? 1 : 0});
        c0 += b.group_cols[g];
      }
    }
    for (int dt = 0; dt < kNumDtypes; ++dt) {    // one run per format, formats ascending
      int32_t cols = 0;
      for (auto& s : Cp.segs)
        if (s.dtype == dt) { s.seccol = cols; cols += s.ncols; }
      if (cols == 0) continue;
      const int G = group_width(dt);
      ColSectionHost S;
      S.dtype = dt;
      S.ld = (int32_t)align_up(cols, G);
      S.g0 = Cp.ngroups;
      S.c0 = Cp.ncols;
      Cp.ngroups += S.ld / G;
      Cp.ncols += S.ld;
      Cp.secs.push_back(S);
    }
    cut_tiles(Cp, P->tile_groups, P->launch.tmix == 0);
  }

  return layout_store(P.release(), out);
}

// ------------------------------------------------------------------ tuning

static bool parse_launch(const char* text, LaunchParams& lp) {
  if (!text) return false;
  LaunchParams r = lp;
  std::string t(text);
  size_t i = 0;
  while (i < t.size()) {
    while (i < t.size() && (t[i] == ' ' || t[i] == '\t')) ++i;
    size_t j = i;
    while (j < t.size() && t[j] != ' ' && t[j] != '\t' && t[j] != '\n') ++j;
    if (j == i) break;
    const std::string kv = t.substr(i, j - i);
    const size_t eq = kv.find('=');
    if (eq == std::string::npos) return false;
    const std::string k = kv.substr(0, eq);
    char* end = nullptr;
    const long v = std::strtol(kv.c_str() + eq + 1, &end, 10);
    if (!end || *end) return false;
    if (k == "schedule" && (v == 0 || v == 1)) r.schedule = (int)v;
    else if (k == "unroll" && (v == 4 || v == 8)) r.row_unroll = (int)v;
    else if (k == "order" && (v == 0 || v == 1)) r.order = (int)v;
    else if (k == "persist" && (v == 0 || v == 1 || v == 2 || v == 4 || v == 8)) r.persist = (int)v;
    else if (k == "chunk" && v >= kMaxTileRows && v <= kSegRows) r.chunk = (int)v;
    else if (k == "tile" && v >= 8 && v <= kTileGroups) r.tile = (int)v;
    else if (k == "colb" && v >= 0 && v <= 3) r.colb = (int)v;
    else if (k == "tmix" && (v == 0 || v == 1)) r.tmix = (int)v;
    else if (k == "colw" && v >= 0 && v <= 2) r.colw = (int)v;
    else return false;
    i = j;
  }
  lp = r;
  return true;
}

// Kind of matrix a tuned choice applies to: accumulation type, storage
// formats present, size class, rank class (floor(log2) of the mean rank of
// the low-rank blocks), and "-batch" for plans made for several right-hand
// sides (their products run the multi-right-hand-side kernels).
static std::string tune_key_mask(int acc, int mask, int64_t n_rows, int rank_class, int max_nrhs) {
  int lg = 0;
  while ((int64_t(1) << (lg + 1)) <= n_rows) ++lg;
  char buf[64];
  std::snprintf(buf, sizeof buf, "acc%d-fmt%d-n2^%d-r%d%s", acc, mask, lg, rank_class,
                max_nrhs > 1 ? "-batch" : "");
  return buf;
}
static std::string tune_key(int acc, const size_t* bytes_by_dtype, int64_t n_rows, int rank_class,
                            int max_nrhs) {
  int mask = 0;
  for (int d = 0; d < kNumDtypes; ++d) if (bytes_by_dtype[d]) mask |= 1 << d;
  return tune_key_mask(acc, mask, n_rows, rank_class, max_nrhs);
}

// floor(log2) of the mean rank of the low-rank blocks of nonzero rank (0
// when there are none).
static int rank_class(const hm_plan* P) {
  double sum = 0;
  int64_t cnt = 0;
  for (auto& b : P->blocks)
    if (b.kind == HM_LOWRANK && b.rank > 0) { sum += b.rank; ++cnt; }
  int c = 0;
  if (cnt > 0)
    while (std::ldexp(1.0, c + 1) <= sum / (double)cnt) ++c;
  return c;
}

// The formats a plan's blocks store values in (the formats with stored
// bytes once it is laid out).
static int format_mask(const hm_plan* P) {
  int mask = 0;
  for (auto& b : P->blocks) {
    if (b.kind == HM_DENSE) mask |= 1 << b.group_dtype[0];
    else
      for (int g = 0; g < b.ngroups; ++g)
        if (b.group_cols[g] > 0) mask |= 1 << b.group_dtype[g];
  }
  return mask;
}

void read_tune_cache(hm_plan* P) {
  FILE* f = std::fopen(P->tune_path.c_str(), "r");
  if (!f) return;
  const std::string key =
      tune_key_mask(P->opts.acc_dtype, format_mask(P), P->n_rows, P->rank_class, P->opts.max_nrhs);
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    std::string l(line);
    const size_t sp = l.find(' ');
    if (sp == std::string::npos || l[0] == '#') continue;
    if (l.substr(0, sp) == key) {
      LaunchParams lp = P->launch;
      if (parse_launch(l.c_str() + sp + 1, lp)) P->launch = lp;
    }
  }
  std::fclose(f);
}

hm_status layout_store(hm_plan* Pp, hm_plan** out) {
  std::unique_ptr<hm_plan> P(Pp);
  const int acc_sz = P->opts.acc_dtype == HM_F64 ? 8 : 4;
  StoreHeader& H = P->hdr;
  std::memset(&H, 0, sizeof H);
  H.magic = kStoreMagic;
  H.n_rows = P->n_rows;
  H.n_cols = P->n_cols;
  H.n_row_panels = (int64_t)P->rps.size();
  H.acc_dtype = P->opts.acc_dtype;
  H.has_sigma = P->has_sigma;
  H.n_t = P->n_t;
  H.n_partials = P->n_partials;
  H.n_large = P->n_large;
  H.n_large_t = P->n_large_t;
  H.n_red_t = P->n_red_t;
  H.n_tblocks = (int64_t)P->lr_order.size();
  int64_t nsec = 0, nsrc = 0;
  for (auto& R : P->rps) { nsec += (int64_t)R.secs.size(); nsrc += R.ncols; }
  H.n_row_sections = nsec;
  int64_t ntiles = 0, ndst = 0;
  for (auto& Cp : P->cps) {
    ntiles += (int64_t)Cp.tile_lo.size();
    ndst += Cp.ncols;
  }
  H.n_col_tiles = ntiles;
  {
    // tiles per class (one format, or several: runs of a panel that meet in a tile)
    int64_t cnt[kNumDtypes + 1] = {};
    for (auto& Cp : P->cps)
      for (size_t t = 0; t < Cp.tile_lo.size(); ++t) {
        const int32_t g0 = Cp.tile_g0[t], g1 = Cp.tile_g0[t + 1];
        int runs = 0, fmt = 0;
        for (auto& S : Cp.secs) {
          const int32_t a = S.g0, b = S.g0 + S.ld / group_width(S.dtype);
          if (std::max(a, g0) < std::min(b, g1)) { ++runs; fmt = S.dtype; }
        }
        ++cnt[runs == 1 ? fmt : kNumDtypes];
      }
    int64_t acc_end = 0;
    for (int c = 0; c <= kNumDtypes; ++c) H.tile_class_end[c] = (acc_end += cnt[c]);
  }
  {
    // launch classes of small tiles.  A tile of g groups is read in batches
    // of 8 RS rows (RS = 64 / GP, GP the power of two >= g); a workgroup
    // gives its four waves a batch each in turn, so a tile of b batches
    // keeps 4 ceil(b / 4) wave slots busy for b batches of work.  A class
    // where that wastes more than a quarter runs a wave per tile.
    double work[kNumDtypes + 1] = {}, slots[kNumDtypes + 1] = {};
    for (auto& Cp : P->cps)
      for (size_t t = 0; t < Cp.tile_lo.size(); ++t) {
        const int32_t g0 = Cp.tile_g0[t], g1 = Cp.tile_g0[t + 1];
        int runs = 0, fmt = 0;
        for (auto& S : Cp.secs) {
          const int32_t a = S.g0, b = S.g0 + S.ld / group_width(S.dtype);
          if (std::max(a, g0) < std::min(b, g1)) { ++runs; fmt = S.dtype; }
        }
        const int c = runs != 1 ? kNumDtypes : fmt <= HM_BF16 ? 0 : fmt;
        int gp = 1;
        while (gp < g1 - g0) gp *= 2;
        const int64_t rs = 64 / gp, b = (Cp.nrows + 8 * rs - 1) / (8 * rs);
        work[c] += (double)b;
        slots[c] += 4.0 * (double)((b + 3) / 4);
      }
    P->col_wave = 0;
    for (int c = 0; c <= kNumDtypes; ++c)
      if (slots[c] > 0 && work[c] < 0.75 * slots[c]) P->col_wave |= 1u << c;
  }

  int64_t off = align_up(sizeof(StoreHeader), kAlign);
  auto take = [&](int64_t bytes) { int64_t o = off; off = align_up(off + bytes, kAlign); return o; };
  H.off_row_panels = take(H.n_row_panels * (int64_t)sizeof(RowPanel));
  H.off_row_sections = take(nsec * (int64_t)sizeof(RowSection));
  H.off_row_order = take(H.n_row_panels * 4);
  H.off_row_src = take(nsrc * 4);
  H.off_col_tiles = take(ntiles * (int64_t)sizeof(ColTile));
  H.off_col_dst = take(ndst * 4);
  H.off_tblocks = take(H.n_tblocks * (int64_t)sizeof(TBlock));
  H.off_large = take(H.n_large * 4);
  H.off_owner = take(H.n_t * 4);
  H.off_sigma = take(P->has_sigma ? H.n_t * acc_sz : 0);
  {
    int64_t nd = 0, nu = 0;
    for (auto& R : P->rps) {
      nd += R.nsec_dense > 0;
      nu += (int32_t)R.secs.size() > R.nsec_dense;
    }
    H.n_p1 = nd + ntiles;
    H.n_p2 = nu;
  }
  H.off_p1_order = take(H.n_p1 * 4);
  H.off_p2_order = take(H.n_p2 * 4);
  for (auto& b : P->blocks)
    for (int g = 0; g < b.ngroups; ++g) H.has_aflp |= is_aflp(b.group_dtype[g]);
  H.off_row_aflp = take(H.has_aflp ? nsrc * 4 : 0);
  H.off_col_aflp = take(H.has_aflp ? ndst * 4 : 0);
  const int64_t meta_end = off;

  // data: row sections, then column sections
  int64_t src_off = 0;
  double factor_bytes = 0, pad_bytes = 0;
  for (int d = 0; d < kNumDtypes; ++d) P->bytes_by_dtype[d] = 0;
  for (auto& R : P->rps) {
    R.src_off = src_off;
    src_off += R.ncols;
    for (auto& S : R.secs) {
      const int64_t bytes = (int64_t)S.ngroups * R.m * (16 + lo_bytes(S.dtype));
      S.data_off = take(bytes);
      int64_t real = 0;
      for (auto& s : R.segs)
        if (s.dtype == S.dtype && s.kind == S.kind) real += s.ncols;
      const int64_t real_bytes = real * R.m * value_bytes(S.dtype);
      factor_bytes += (double)real_bytes;
      pad_bytes += (double)(bytes - real_bytes);
      P->bytes_by_dtype[S.dtype] += (size_t)real_bytes;
    }
  }
  for (auto& Cp : P->cps) {
    Cp.data_off = take(Cp.tile_off.back());
    for (auto& S : Cp.secs) {
      const int64_t bytes = (int64_t)S.ld * Cp.nrows * value_bytes(S.dtype);
      int64_t real = 0;
      for (auto& s : Cp.segs)
        if (s.dtype == S.dtype) real += s.ncols;
      const int64_t real_bytes = real * Cp.nrows * value_bytes(S.dtype);
      factor_bytes += (double)real_bytes;
      pad_bytes += (double)(bytes - real_bytes);
      P->bytes_by_dtype[S.dtype] += (size_t)real_bytes;
    }
  }
  P->store_bytes = (size_t)off;
  P->meta_bytes = (size_t)meta_end;
  P->factor_bytes = factor_bytes;

  // work per right-hand side: partials, t, and a slot for the transposed
  // right-hand sides of the batched path, each 256-byte aligned
  P->work_part_bytes = align_up(P->n_partials * acc_sz, kAlign);
  P->work_t_bytes = align_up(P->n_t * acc_sz, kAlign);
  P->work_x_bytes = align_up(P->n_cols * acc_sz, kAlign);
  P->work_part_off = 0;
  P->work_t_off = P->work_part_bytes;
  P->work_bytes_per_rhs = (size_t)(P->work_part_bytes + P->work_t_bytes + P->work_x_bytes);
  // the batched column kernel addresses partials and t as one table of rows
  if (P->work_part_bytes / 4 + P->n_t > INT32_MAX)
    return fail(HM_ENOMEM, "too many partials and t entries for 32-bit indices");

  // accounting
  const int vec_sz = acc_sz;
  double alg = factor_bytes + (double)P->n_cols * vec_sz + 2.0 * (double)P->n_rows * vec_sz;
  if (P->has_sigma) alg += (double)P->n_t * acc_sz;
  double flops = 0;
  int64_t nd = 0, nl = 0;
  for (auto& b : P->blocks) {
    const double m = (double)(b.row_end - b.row_begin), n = (double)(b.col_end - b.col_begin);
    if (b.kind == HM_DENSE) { flops += 2 * m * n; ++nd; }
    else { flops += 2 * (m + n) * b.rank; ++nl; }
  }
  P->alg_bytes = alg;
  P->alg_flops = flops;
  P->n_dense = nd;
  P->n_lowrank = nl;
  P->overhead_bytes = (double)(nsrc + ndst) * (H.has_aflp ? 8 : 4) + pad_bytes +
                      (double)H.n_row_panels * (sizeof(RowPanel) + 4) + nsec * sizeof(RowSection) +
                      ntiles * sizeof(ColTile) + H.n_tblocks * sizeof(TBlock) +
                      (double)H.n_t * 4 + 2.0 * P->n_partials * acc_sz +
                      2.0 * P->n_t * acc_sz;
  *out = P.release();
  return ok();
}

// ------------------------------------------------------------------ packing

static const double* fac(const double* const* arr, int64_t i) { return arr ? arr[i] : nullptr; }

// Column group of column c of block b (its first group for a dense block).
static int group_of(const hm_block_desc& b, int64_t c) {
  int64_t end = 0;
  for (int g = 0; g < b.ngroups; ++g)
    if (c < (end += b.group_cols[g])) return g;
  return 0;
}

// Runs f(i) for i in [0, n) on the process's CPU share.
static void parallel_for(size_t n, const std::function<void(size_t)>& f) {
  unsigned nthr = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (const char* e = std::getenv("OMP_NUM_THREADS")) {    // the process's CPU share, if stated
    const int v = std::atoi(e);
    if (v > 0) nthr = std::min(nthr, (unsigned)v);
  }
  nthr = (unsigned)std::min<size_t>(nthr, std::max<size_t>(1, n));
  std::atomic<size_t> next{0};
  auto worker = [&]() {
    for (size_t i; (i = next.fetch_add(1)) < n;) f(i);
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nthr; ++t) th.emplace_back(worker);
  worker();
  for (auto& t : th) t.join();
}

// Every factor pointer a block needs is present.
static hm_status check_factors(const hm_plan* P, const double* const* a, const double* const* bf,
                               const double* const* s) {
  for (size_t i = 0; i < P->blocks.size(); ++i) {
    const auto& b = P->blocks[i];
    if (!fac(a, (int64_t)i) && (b.kind == HM_DENSE || b.rank > 0))
      return fail(HM_EINVAL, "block %zu: missing first factor", i);
    if (b.kind == HM_LOWRANK && b.rank > 0 && !fac(bf, (int64_t)i))
      return fail(HM_EINVAL, "block %zu: missing second factor", i);
    if (b.kind == HM_LOWRANK && b.rank > 0 && b.has_sigma && !fac(s, (int64_t)i))
      return fail(HM_EINVAL, "block %zu: missing singular values", i);
  }
  return HM_OK;
}

// Every BFL value of block b (its BFL column groups) can be encoded.
static bool bfl_block_ok(const hm_block_desc& b, const double* a, const double* bf) {
  const int64_t m = b.row_end - b.row_begin, nb = b.col_end - b.col_begin;
  auto ok = [](const double* v, int64_t n, int dt) {
    uint64_t c;
    for (int64_t i = 0; i < n; ++i)
      if (!bfl_code(v[i], value_bytes(dt), &c)) return false;
    return true;
  };
  if (b.kind == HM_DENSE) return !is_bfl(b.group_dtype[0]) || ok(a, m * nb, b.group_dtype[0]);
  int64_t c0 = 0;
  for (int g = 0; g < b.ngroups; ++g) {
    const int dt = b.group_dtype[g];
    const int64_t kc = b.group_cols[g];
    if (is_bfl(dt) && kc > 0 && !(ok(a + c0 * m, m * kc, dt) && ok(bf + c0 * nb, nb * kc, dt))) return false;
    c0 += kc;
  }
  return true;
}

hm_status AflpTable::build(const hm_plan* P, const double* const* a, const double* const* bf) {
  base.assign(P->blocks.size(), -1);
  bool any_bfl = false;
  for (auto& b : P->blocks)
    for (int g = 0; g < b.ngroups; ++g) any_bfl |= is_bfl(b.group_dtype[g]);
  if (any_bfl) {                                   // BFL data in range (checked before any packing)
    std::atomic<int64_t> bad{-1};
    parallel_for(P->blocks.size(), [&](size_t i) {
      const auto& b = P->blocks[i];
      if ((b.kind == HM_DENSE || b.rank > 0) && !bfl_block_ok(b, a[i], b.kind == HM_DENSE ? nullptr : bf[i]))
        bad.store((int64_t)i);
    });
    if (bad.load() >= 0)
      return fail(HM_EINVAL, "block %lld: BFL needs finite values within FP32's range", (long long)bad.load());
  }
  int64_t n = 0;
  for (size_t i = 0; i < P->blocks.size(); ++i) {
    const auto& b = P->blocks[i];
    bool any = false;
    for (int g = 0; g < b.ngroups; ++g) any |= is_aflp(b.group_dtype[g]);
    if (!any) continue;
    if (b.kind == HM_LOWRANK && b.rank == 0) continue;
    base[i] = n;
    n += b.kind == HM_DENSE ? 1 : 2 * b.ngroups;
  }
  prm.assign((size_t)n, 0);
  if (n == 0) return HM_OK;                        // no AFLP data
  std::atomic<int64_t> bad{-1};
  parallel_for(P->blocks.size(), [&](size_t i) {
    if (base[i] < 0) return;
    const auto& b = P->blocks[i];
    const int64_t m = b.row_end - b.row_begin, nb = b.col_end - b.col_begin;
    bool good = true;
    if (b.kind == HM_DENSE) {
      good = aflp_block_param(a[i], m, nb, m, value_bytes(b.group_dtype[0]), &prm[base[i]]);
    } else {
      int64_t c0 = 0;
      for (int g = 0; g < b.ngroups && good; ++g) {
        const int dt = b.group_dtype[g];
        const int64_t kc = b.group_cols[g];
        if (is_aflp(dt) && kc > 0)
          good = aflp_block_param(a[i] + c0 * m, m, kc, m, value_bytes(dt), &prm[base[i] + g]) &&
                 aflp_block_param(bf[i] + c0 * nb, nb, kc, nb, value_bytes(dt), &prm[base[i] + b.ngroups + g]);
        c0 += kc;
      }
    }
    if (!good) bad.store((int64_t)i);
  });
  if (bad.load() >= 0)
    return fail(HM_EINVAL, "block %lld: AFLP needs finite values whose range fits its bytes",
                (long long)bad.load());
  return HM_OK;
}

int32_t AflpTable::get(const hm_plan* P, int64_t block, int which, int64_t col) const {
  const auto& b = P->blocks[block];
  if (base[block] < 0) return 0;
  if (b.kind == HM_DENSE) return prm[base[block]];
  return prm[base[block] + which * b.ngroups + group_of(b, col)];
}

// Header and descriptor tables: bytes [0, meta_bytes) of the store.
hm_status pack_meta(const hm_plan* P, const double* const* a, const double* const* bf,
                    const double* const* s, const AflpTable& T, uint8_t* buf) {
  const StoreHeader& H = P->hdr;
  std::memcpy(buf, &H, sizeof H);
  const int acc_sz = P->opts.acc_dtype == HM_F64 ? 8 : 4;
  if (hm_status st = check_factors(P, a, bf, s)) return st;
  // descriptor tables
  auto* rp = reinterpret_cast<RowPanel*>(buf + H.off_row_panels);
  auto* rs = reinterpret_cast<RowSection*>(buf + H.off_row_sections);
  auto* ro = reinterpret_cast<int32_t*>(buf + H.off_row_order);
  auto* rsrc = reinterpret_cast<int32_t*>(buf + H.off_row_src);
  int32_t sec = 0;
  for (size_t p = 0; p < P->rps.size(); ++p) {
    const RowPanelHost& R = P->rps[p];
    RowPanel& d = rp[p];
    d.src_off = R.src_off;
    d.row0 = (int32_t)R.row0;
    d.m = R.m;
    d.ncols = R.ncols;
    d.sec0 = sec;
    d.nsec = (int32_t)R.secs.size();
    d.nsec_dense = R.nsec_dense;
    for (auto& S : R.secs) {
      RowSection& e = rs[sec++];
      e.data_off = S.data_off;
      e.dtype = S.dtype;
      e.ngroups = S.ngroups;
      e.col0 = S.col0;
      e.pad_[0] = e.pad_[1] = e.pad_[2] = 0;
    }
    int32_t* src = rsrc + R.src_off;
    for (int32_t c = 0; c < R.ncols; ++c) src[c] = 0;   // padding slots read x[0] (times 0)
    int32_t* ra = H.has_aflp ? reinterpret_cast<int32_t*>(buf + H.off_row_aflp) + R.src_off : nullptr;
    if (ra) for (int32_t c = 0; c < R.ncols; ++c) ra[c] = 0;
    for (auto& sg : R.segs) {
      const RowSectionHost* S = nullptr;
      for (auto& x : R.secs) if (x.dtype == sg.dtype && x.kind == sg.kind) S = &x;
      for (int32_t c = 0; c < sg.ncols; ++c) src[S->col0 + sg.seccol + c] = sg.src0 + c;
      if (ra && is_aflp(sg.dtype))
        for (int32_t c = 0; c < sg.ncols; ++c) ra[S->col0 + sg.seccol + c] = T.get(P, sg.block, 0, sg.c_first + c);
    }
  }
  // launch order of row panels: largest first (longest-processing-time order)
  {
    std::vector<int32_t> ord(P->rps.size());
    std::iota(ord.begin(), ord.end(), 0);
    auto bytes = [&](int32_t p) {
      int64_t s = 0;
      for (auto& S : P->rps[p].secs) s += (int64_t)S.ngroups * P->rps[p].m * (16 + lo_bytes(S.dtype));
      return s;
    };
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return bytes(x) > bytes(y); });
    std::copy(ord.begin(), ord.end(), ro);
    // phase orders: bytes of the dense part and of the U part of each panel
    auto part_bytes = [&](int32_t p, int kind) {
      int64_t s = 0;
      for (auto& S : P->rps[p].secs)
        if (S.kind == kind) s += (int64_t)S.ngroups * P->rps[p].m * (16 + lo_bytes(S.dtype));
      return s;
    };
    std::vector<int32_t> dense, upart;
    for (int32_t p = 0; p < (int32_t)P->rps.size(); ++p) {
      if (P->rps[p].nsec_dense > 0) dense.push_back(p);
      if ((int32_t)P->rps[p].secs.size() > P->rps[p].nsec_dense) upart.push_back(p);
    }
    std::stable_sort(dense.begin(), dense.end(),
                     [&](int32_t x, int32_t y) { return part_bytes(x, 0) > part_bytes(y, 0); });
    std::stable_sort(upart.begin(), upart.end(),
                     [&](int32_t x, int32_t y) { return part_bytes(x, 1) > part_bytes(y, 1); });
    // interleave dense panels (largest first) with tile groups evenly
    auto* p1 = reinterpret_cast<int32_t*>(buf + H.off_p1_order);
    const int64_t A = (int64_t)dense.size(), B = H.n_p1 - A;
    int64_t ia = 0, ib = 0;
    for (int64_t k = 0; k < H.n_p1; ++k) {
      const bool take_panel = ib >= B || (ia < A && ia * B <= ib * A);
      p1[k] = take_panel ? dense[ia++] : (int32_t)(-(ib++) - 1);
    }
    auto* p2 = reinterpret_cast<int32_t*>(buf + H.off_p2_order);
    std::copy(upart.begin(), upart.end(), p2);
  }
  // column tiles and destinations: per panel, the destination of every
  // column in the panel's column order (run by run), and tiles of 64 groups
  auto* ct = reinterpret_cast<ColTile*>(buf + H.off_col_tiles);
  auto* cdst = reinterpret_cast<int32_t*>(buf + H.off_col_dst);
  int64_t tile = 0, dsto = 0;
  for (auto& Cp : P->cps) {
    int32_t* dst = cdst + dsto;
    for (int32_t c = 0; c < Cp.ncols; ++c) dst[c] = kDstPad;
    int32_t* ca = H.has_aflp ? reinterpret_cast<int32_t*>(buf + H.off_col_aflp) + dsto : nullptr;
    if (ca) for (int32_t c = 0; c < Cp.ncols; ++c) ca[c] = 0;
    for (auto& sg : Cp.segs) {
      const ColSectionHost* S = nullptr;
      for (auto& x : Cp.secs) if (x.dtype == sg.dtype) S = &x;
      for (int32_t c = 0; c < sg.ncols; ++c)
        dst[S->c0 + sg.seccol + c] = sg.direct ? dst_direct(sg.src0 + c) : sg.src0 + c;
      if (ca && is_aflp(sg.dtype))
        for (int32_t c = 0; c < sg.ncols; ++c) ca[S->c0 + sg.seccol + c] = T.get(P, sg.block, 1, sg.c_first + c);
    }
    for (size_t ti = 0; ti < Cp.tile_lo.size(); ++ti) {
      ColTile& T = ct[tile++];
      const int32_t g0 = Cp.tile_g0[ti], ngt = Cp.tile_g0[ti + 1] - g0;
      T.data_off = Cp.data_off + Cp.tile_off[ti];   // tiles one after another
      T.nrows = Cp.nrows;
      T.x0 = (int32_t)Cp.x0;
      T.ngroups = ngt;
      // runs of the tile: the panel's runs cut to groups [g0, g0 + ngt)
      int nr = 0, first_col = -1;
      for (auto& S : Cp.secs) {
        const int32_t G = group_width(S.dtype);
        const int32_t lo = std::max(S.g0, g0), hi = std::min(S.g0 + S.ld / G, g0 + ngt);
        if (hi <= lo) continue;
        if (nr == 4) return fail(HM_EINVAL, "internal error: column tile with more than 4 runs");
        if (first_col < 0) first_col = S.c0 + (lo - S.g0) * G;
        T.dtype[nr] = (uint8_t)S.dtype;
        T.end[nr] = (uint8_t)(hi - g0);
        ++nr;
      }
      for (int r = nr; r < 4; ++r) {               // empty runs at the end
        T.dtype[r] = T.dtype[nr - 1];
        T.end[r] = (uint8_t)ngt;
      }
      T.dst_off = (int32_t)(dsto + first_col);
    }
    dsto += Cp.ncols;
  }
  // tile order, grouped by class (each class runs in a launch of its own):
  // FP64 and DFL tiles (formats of the FP64-accumulation plans) are
  // near-uniform in size and stream best in store order; the other classes
  // vary more and go largest first (longest-processing-time order against
  // the tail)
  std::stable_sort(ct, ct + H.n_col_tiles, [](const ColTile& x, const ColTile& y) {
    const int cx = tile_class(x), cy = tile_class(y);
    if (cx != cy) return cx < cy;
    if (cx == HM_F64 || is_dfl(cx)) return x.data_off < y.data_off;
    return (int64_t)x.nrows * x.ngroups > (int64_t)y.nrows * y.ngroups;
  });
  // reduction tables
  auto* tb = reinterpret_cast<TBlock*>(buf + H.off_tblocks);
  auto* lg = reinterpret_cast<int32_t*>(buf + H.off_large);
  auto* own = reinterpret_cast<int32_t*>(buf + H.off_owner);
  for (size_t q = 0; q < P->lr_order.size(); ++q) {
    const int32_t i = P->lr_order[q];
    const BlockInfo& bi = P->binfo[i];
    TBlock& T = tb[q];
    T.pst = (int32_t)bi.pst;
    T.k = P->blocks[i].rank;
    T.nseg = bi.nseg;
    T.toff = (int32_t)bi.toff;
    if ((int64_t)q < H.n_large) lg[q] = (int32_t)q;
    for (int32_t l = 0; l < T.k; ++l) own[bi.toff + l] = (int32_t)q;
    if (P->has_sigma) {
      const auto& b = P->blocks[i];
      for (int32_t l = 0; l < T.k; ++l) {
        double v = b.has_sigma ? s[i][l] : 1.0;
        put(buf + H.off_sigma + (bi.toff + l) * acc_sz, P->opts.acc_dtype, v);
      }
    }
  }
  return HM_OK;
}

size_t pack_jobs_count(const hm_plan* P) { return P->rps.size() + P->cps.size(); }

// Store bytes [lo, hi) of packing job j (row panels, then column panels):
// its sections, which are contiguous; jobs follow each other without gaps.
void pack_job_range(const hm_plan* P, size_t j, int64_t* lo, int64_t* hi) {
  const size_t nrp = P->rps.size();
  auto span = [&](auto& secs, auto bytes_of) {
    if (secs.empty()) { *lo = *hi = -1; return; }
    *lo = secs.front().data_off;
    *hi = align_up(secs.back().data_off + bytes_of(secs.back()), kAlign);
  };
  if (j < nrp) {
    const RowPanelHost& R = P->rps[j];
    span(R.secs, [&](const RowSectionHost& S) { return (int64_t)S.ngroups * R.m * (16 + lo_bytes(S.dtype)); });
  } else {
    const ColPanelHost& Cp = P->cps[j - nrp];
    if (Cp.ngroups == 0) {
      *lo = *hi = -1;
    } else {
      *lo = Cp.data_off;
      *hi = align_up(Cp.data_off + Cp.tile_off.back(), kAlign);
    }
  }
}

// Factor data of packing jobs [j_begin, j_end), in parallel; store byte o
// goes to out[o - out_off] (out covers the jobs' byte ranges).
void pack_jobs(const hm_plan* P, const double* const* a, const double* const* bf, const AflpTable& T,
               size_t j_begin, size_t j_end, uint8_t* out, int64_t out_off) {
  auto at = [&](int64_t o) { return out + (o - out_off); };
  const size_t nrp = P->rps.size();
  std::atomic<size_t> next{j_begin};
  auto worker = [&]() {
    for (;;) {
      size_t job = next.fetch_add(1);
      if (job >= j_end) return;
      if (job < nrp) {
        const RowPanelHost& R = P->rps[job];
        for (auto& sg : R.segs) {
          const RowSectionHost* S = nullptr;
          for (auto& x : R.secs) if (x.dtype == sg.dtype && x.kind == sg.kind) S = &x;
          const int G = group_width(S->dtype), sz = dtype_size(S->dtype);
          const auto& b = P->blocks[sg.block];
          const int64_t mb = b.row_end - b.row_begin;
          const int64_t r_local = R.row0 - b.row_begin;
          const double* A = a[sg.block];
          uint8_t* base = at(S->data_off);
          const int L = lo_bytes(S->dtype);
          uint8_t* lo_base = base + (int64_t)16 * S->ngroups * R.m;   // low-byte plane (DFL40 / DFL48)
          for (int32_t c = 0; c < sg.ncols; ++c) {
            const int32_t sc = sg.seccol + c;
            const int32_t g = sc / G, cc = sc % G;
            const double* col = A + (int64_t)(sg.c_first + c) * mb + r_local;
            const int32_t prm = is_aflp(S->dtype) ? T.get(P, sg.block, 0, sg.c_first + c) : 0;
            for (int32_t i = 0; i < R.m; ++i) {
              uint8_t* hi = base + (((int64_t)g * R.m + i) * G + cc) * sz;
              uint8_t* lo = lo_base + ((int64_t)g * R.m + i) * L + cc * (L / G);
              if (is_dfl(S->dtype))
                put_dfl(hi, lo, S->dtype, col[i]);
              else if (is_aflp(S->dtype))
                put_code(hi, lo, S->dtype, aflp_code(col[i], prm, value_bytes(S->dtype)));
              else if (is_bfl(S->dtype))
                put_code(hi, lo, S->dtype, bfl_or_zero(col[i], value_bytes(S->dtype)));
              else
                put(hi, S->dtype, col[i]);
            }
          }
        }
      } else {
        const ColPanelHost& Cp = P->cps[job - nrp];
        for (auto& sg : Cp.segs) {
          const ColSectionHost* S = nullptr;
          for (auto& x : Cp.secs) if (x.dtype == sg.dtype) S = &x;
          const auto& b = P->blocks[sg.block];
          const int64_t nbk = b.col_end - b.col_begin;
          const int64_t c_local = Cp.x0 - b.col_begin;
          const double* V = bf[sg.block];
          const bool lo = lo_bytes(S->dtype) > 0;
          for (int32_t c = 0; c < sg.ncols; ++c) {
            const double* col = V + (int64_t)(sg.c_first + c) * nbk + c_local;
            const int32_t prm = is_aflp(S->dtype) ? T.get(P, sg.block, 1, sg.c_first + c) : 0;
            for (int32_t i = 0; i < Cp.nrows; ++i) {
              uint8_t* hi = at(col_elem_offset(Cp, *S, i, sg.seccol + c));
              uint8_t* lp = lo ? at(col_lo_offset(Cp, *S, i, sg.seccol + c)) : nullptr;
              if (is_dfl(S->dtype))
                put_dfl(hi, lp, S->dtype, col[i]);
              else if (is_aflp(S->dtype))
                put_code(hi, lp, S->dtype, aflp_code(col[i], prm, value_bytes(S->dtype)));
              else if (is_bfl(S->dtype))
                put_code(hi, lp, S->dtype, bfl_or_zero(col[i], value_bytes(S->dtype)));
              else
                put(hi, S->dtype, col[i]);
            }
          }
        }
      }
    }
  };
  unsigned nthr = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (const char* e = std::getenv("OMP_NUM_THREADS")) {    // the process's CPU share, if stated
    const int v = std::atoi(e);
    if (v > 0) nthr = std::min(nthr, (unsigned)v);
  }
  nthr = (unsigned)std::min<size_t>(nthr, std::max<size_t>(1, j_end - j_begin));
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nthr; ++t) th.emplace_back(worker);
  worker();
  for (auto& t : th) t.join();
}

hm_status pack_store(const hm_plan* P, const double* const* a, const double* const* bf,
                     const double* const* s, uint8_t* buf) {
  AflpTable T;
  if (hm_status st = check_factors(P, a, bf, s)) return st;
  if (hm_status st = T.build(P, a, bf)) return st;
  if (hm_status st = pack_meta(P, a, bf, s, T, buf)) return st;
  pack_jobs(P, a, bf, T, 0, pack_jobs_count(P), buf, 0);
  return HM_OK;
}

}  // namespace hm

using namespace hm;

// ====================================================================== C-ABI
extern "C" {

hm_status hm_build_plan(int64_t n_rows, int64_t n_cols, const hm_block_desc* blocks,
                        int64_t n_blocks, const hm_plan_opts* opts, hm_plan** out) {
  try {
    return build_plan(n_rows, n_cols, blocks, n_blocks, opts, out);
  } catch (const std::bad_alloc&) {
    return fail(HM_ENOMEM, "host allocation failed while building the plan");
  } catch (...) {
    return fail(HM_EINVAL, "unexpected error while building the plan");
  }
}

hm_status hm_plan_info(const hm_plan* p, hm_plan_info_t* out) {
  if (!p || !out) return fail(HM_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof *out);
  out->store_bytes = p->store_bytes;
  out->work_bytes_per_rhs = p->work_bytes_per_rhs;
  out->alg_bytes = p->alg_bytes;
  out->alg_flops = p->alg_flops;
  out->overhead_bytes = p->overhead_bytes;
  out->n_dense = p->n_dense;
  out->n_lowrank = p->n_lowrank;
  out->n_row_panels = p->hdr.n_row_panels;
  out->n_col_tiles = p->hdr.n_col_tiles;
  out->n_partials = p->n_partials;
  out->n_t = p->n_t;
  for (int d = 0; d < kNumDtypes; ++d) out->bytes_by_dtype[d] = p->bytes_by_dtype[d];
  return ok();
}

void hm_plan_destroy(hm_plan* p) { delete p; }

hm_status hm_plan_locate(const hm_plan* p, int64_t block, int32_t which, int64_t i, int64_t j,
                         size_t* byte_offset, int32_t* dtype, size_t* lo_offset) {
  if (!p || !byte_offset || !dtype) return fail(HM_EINVAL, "NULL argument");
  if (lo_offset) *lo_offset = 0;
  if (block < 0 || block >= (int64_t)p->blocks.size()) return fail(HM_EINVAL, "block out of range");
  const auto& b = p->blocks[block];
  const int64_t m = b.row_end - b.row_begin, n = b.col_end - b.col_begin;
  if (which == 0) {
    const int64_t ncol = b.kind == HM_DENSE ? n : b.rank;
    if (i < 0 || i >= m || j < 0 || j >= ncol) return fail(HM_EINVAL, "entry out of range");
    const int64_t row = b.row_begin + i;
    const int64_t pi = std::upper_bound(p->rint.begin(), p->rint.end(), row) - p->rint.begin() - 1;
    const RowPanelHost& R = p->rps[pi];
    for (auto& sg : R.segs)
      if (sg.block == block && j >= sg.c_first && j < sg.c_first + sg.ncols) {
        for (auto& S : R.secs)
          if (S.dtype == sg.dtype && S.kind == sg.kind) {
            const int G = group_width(S.dtype), L = lo_bytes(S.dtype);
            const int64_t sc = sg.seccol + (j - sg.c_first);
            const int64_t e = (sc / G) * R.m + (row - R.row0);      // group element
            *byte_offset = (size_t)(S.data_off + (e * G + sc % G) * dtype_size(S.dtype));
            if (lo_offset && L)
              *lo_offset = (size_t)(S.data_off + (int64_t)16 * S.ngroups * R.m + e * L + (sc % G) * (L / G));
            *dtype = S.dtype;
            return ok();
          }
      }
    return fail(HM_EINVAL, "entry not stored (zero-rank block?)");
  }
  if (which == 1) {
    if (b.kind != HM_LOWRANK || i < 0 || i >= n || j < 0 || j >= b.rank)
      return fail(HM_EINVAL, "entry out of range");
    const int64_t col = b.col_begin + i;
    const ColPanelHost* found = nullptr;
    for (int64_t q = p->chunk_off[block]; q < p->chunk_off[block + 1]; ++q) {
      const ColPanelHost& Cq = p->cps[p->chunk_list[q]];
      if (col >= Cq.x0 && col < Cq.x0 + Cq.nrows) found = &Cq;
    }
    if (!found) return fail(HM_EINVAL, "entry not stored");
    const ColPanelHost& Cp = *found;
    for (auto& sg : Cp.segs)
      if (sg.block == block && j >= sg.c_first && j < sg.c_first + sg.ncols) {
        for (auto& S : Cp.secs)
          if (S.dtype == sg.dtype) {
            *byte_offset = (size_t)col_elem_offset(Cp, S, col - Cp.x0, sg.seccol + (j - sg.c_first));
            if (lo_offset && lo_bytes(S.dtype))
              *lo_offset = (size_t)col_lo_offset(Cp, S, col - Cp.x0, sg.seccol + (j - sg.c_first));
            *dtype = S.dtype;
            return ok();
          }
      }
    return fail(HM_EINVAL, "entry not stored");
  }
  return fail(HM_EINVAL, "which must be 0 or 1");
}

// Bytes of one upload window: HM_UPLOAD_WINDOW_BYTES if set (>= 4096),
// else 256 MiB.
static size_t upload_window_bytes() {
  if (const char* e = std::getenv("HM_UPLOAD_WINDOW_BYTES")) {
    const long long v = std::atoll(e);
    if (v >= 4096) return (size_t)v;
  }
  return (size_t)256 << 20;
}

// Factor data of the store, packed window by window into two pinned host
// buffers and copied on `hs` while the next window is packed.
static hm_status upload_factor_data(const hm_plan* p, const double* const* a, const double* const* bf,
                                    const AflpTable& aflp, uint8_t* d_store, hipStream_t hs) {
  const size_t njobs = pack_jobs_count(p);
  int64_t max_job = 0;
  for (size_t j = 0; j < njobs; ++j) {
    int64_t lo, hi;
    pack_job_range(p, j, &lo, &hi);
    max_job = std::max(max_job, hi - lo);
  }
  const size_t wbytes = std::max(upload_window_bytes(), (size_t)max_job);
  uint8_t* stage[2] = {nullptr, nullptr};
  hipEvent_t done[2] = {nullptr, nullptr};
  hm_status st = HM_OK;
  for (int b = 0; b < 2 && st == HM_OK; ++b) {
    if (hipHostMalloc((void**)&stage[b], wbytes, hipHostMallocDefault) != hipSuccess) {
      stage[b] = nullptr;
      st = fail(HM_ENOMEM, "pinned staging allocation of %zu bytes failed", wbytes);
    } else if (hipEventCreateWithFlags(&done[b], hipEventDisableTiming) != hipSuccess) {
      done[b] = nullptr;
      st = fail(HM_EDEVICE, "event creation failed");
    }
  }
  int64_t cursor = (int64_t)p->meta_bytes;
  size_t j = 0;
  for (int k = 0; st == HM_OK && j < njobs; ++k) {
    // the window: whole jobs [j, j2) covering store bytes [lo, hi)
    const int64_t lo = cursor;
    int64_t hi = cursor;
    size_t j2 = j;
    for (; j2 < njobs; ++j2) {
      int64_t l, h;
      pack_job_range(p, j2, &l, &h);
      if (l < 0) continue;                         // job without data
      if (l != hi) { st = fail(HM_EINVAL, "internal error: store layout is not contiguous"); break; }
      if (hi > lo && h - lo > (int64_t)wbytes) break;
      hi = h;
    }
    if (st != HM_OK) break;
    const int b = k & 1;
    if (k >= 2 && hipEventSynchronize(done[b]) != hipSuccess) {
      st = fail(HM_EDEVICE, "upload copy failed");
      break;
    }
    std::memset(stage[b], 0, (size_t)(hi - lo));
    pack_jobs(p, a, bf, aflp, j, j2, stage[b], lo);
    if (hi > lo && (hipMemcpyAsync(d_store + lo, stage[b], (size_t)(hi - lo), hipMemcpyHostToDevice, hs) !=
                        hipSuccess ||
                    hipEventRecord(done[b], hs) != hipSuccess)) {
      st = fail(HM_EDEVICE, "upload copy failed: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    cursor = hi;
    j = j2;
  }
  if (hipStreamSynchronize(hs) != hipSuccess && st == HM_OK) st = fail(HM_EDEVICE, "upload copy failed");
  if (st == HM_OK && cursor != (int64_t)p->store_bytes)
    st = fail(HM_EINVAL, "internal error: packed %lld of %zu store bytes", (long long)cursor, p->store_bytes);
  for (int b = 0; b < 2; ++b) {
    if (done[b]) (void)hipEventDestroy(done[b]);
    if (stage[b]) (void)hipHostFree(stage[b]);
  }
  return st;
}

hm_status hm_upload(const hm_plan* p, const double* const* a, const double* const* bf,
                    const double* const* s, void* d_store, size_t store_bytes, void* stream,
                    hm_matrix** out) {
  if (!p || !out || !d_store) return fail(HM_EINVAL, "NULL argument");
  *out = nullptr;
  if (store_bytes < p->store_bytes)
    return fail(HM_ENOMEM, "store has %zu bytes, plan needs %zu", store_bytes, p->store_bytes);
  if (((uintptr_t)d_store) % kAlign) return fail(HM_EINVAL, "store must be 256-byte aligned");
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
    return fail(HM_EDEVICE, "no usable HIP device");
  hipStream_t hs = (hipStream_t)stream;
  // header and tables (validates the factor pointers), then the factor data
  AflpTable aflp;
  {
    std::vector<uint8_t> meta;
    hm_status st;
    try {
      meta.assign(p->meta_bytes, 0);
      st = check_factors(p, a, bf, s);
      if (!st) st = aflp.build(p, a, bf);
      if (!st) st = pack_meta(p, a, bf, s, aflp, meta.data());
    } catch (...) {
      st = fail(HM_ENOMEM, "packing failed");
    }
    if (st) return st;
    hipError_t e = hipMemcpyAsync(d_store, meta.data(), p->meta_bytes, hipMemcpyHostToDevice, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return fail(HM_EDEVICE, "upload copy failed: %s", hipGetErrorString(e));
  }
  hm_status st;
  try {
    st = upload_factor_data(p, a, bf, aflp, (uint8_t*)d_store, hs);
  } catch (...) {
    st = fail(HM_ENOMEM, "packing failed");
  }
  if (st) return st;
  auto* M = new (std::nothrow) hm_matrix();
  if (!M) return fail(HM_ENOMEM, "host allocation failed");
  M->hdr = p->hdr;
  M->d_store = (const uint8_t*)d_store;
  M->store_bytes = p->store_bytes;
  M->work_bytes_per_rhs = p->work_bytes_per_rhs;
  M->work_t_off = p->work_t_off;
  M->work_part_bytes = p->work_part_bytes;
  M->work_t_bytes = p->work_t_bytes;
  M->work_x_bytes = p->work_x_bytes;
  M->acc_dtype = p->opts.acc_dtype;
  M->max_nrhs = p->opts.max_nrhs;
  M->launch = p->launch;
  M->rank_class = p->rank_class;
  M->device = dev;
  M->n_cu = ncu;
  std::memcpy(M->bytes_by_dtype, p->bytes_by_dtype, sizeof M->bytes_by_dtype);
  M->col_wave = p->col_wave;
  *out = M;
  return ok();
}

hm_status hm_pack_host(const hm_plan* p, const double* const* a, const double* const* bf,
                       const double* const* s, void* h_buf, size_t buf_bytes) {
  if (!p || !h_buf) return fail(HM_EINVAL, "NULL argument");
  if (buf_bytes < p->store_bytes)
    return fail(HM_ENOMEM, "buffer has %zu bytes, plan needs %zu", buf_bytes, p->store_bytes);
  std::memset(h_buf, 0, p->store_bytes);
  hm_status st;
  try {
    st = pack_store(p, a, bf, s, (uint8_t*)h_buf);
  } catch (...) {
    st = fail(HM_ENOMEM, "packing failed");
  }
  return st ? st : ok();
}

void hm_matrix_destroy(hm_matrix* A) {
  if (!A) return;
  for (auto e : A->prof.ev) (void)hipEventDestroy(e);
  delete A;
}

hm_status hm_profile_begin(hm_matrix* A, int32_t max_calls) {
  if (!A || max_calls < 1 || max_calls > 1 << 16) return fail(HM_EINVAL, "bad profile arguments");
  const size_t need = 4 * (size_t)max_calls;
  while (A->prof.ev.size() < need) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return fail(HM_EDEVICE, "event creation failed");
    A->prof.ev.push_back(e);
  }
  A->prof.max_calls = max_calls;
  A->prof.calls = 0;
  A->prof.on = true;
  return ok();
}

hm_status hm_profile_end(hm_matrix* A, double* ms, int64_t* calls) {
  if (!A || !ms) return fail(HM_EINVAL, "NULL argument");
  A->prof.on = false;
  ms[0] = ms[1] = ms[2] = 0;
  for (int32_t c = 0; c < A->prof.calls; ++c) {
    hipEvent_t* e = &A->prof.ev[4 * (size_t)c];
    if (hipEventSynchronize(e[3]) != hipSuccess) return fail(HM_EDEVICE, "event wait failed");
    for (int k = 0; k < 3; ++k) {
      float t = 0;
      if (hipEventElapsedTime(&t, e[k], e[k + 1]) != hipSuccess)
        return fail(HM_EDEVICE, "event timing failed");
      ms[k] += t;
    }
  }
  if (calls) *calls = A->prof.calls;
  return ok();
}

static hm_status check_mvm(const hm_matrix* A, const void* d_x, const void* d_y, const void* d_work,
                           size_t work_bytes) {
  if (!A || !d_x || !d_y) return fail(HM_EINVAL, "NULL argument");
  if (d_x == d_y) return fail(HM_EINVAL, "x must not alias y");
  if (work_bytes < A->work_bytes_per_rhs || (A->work_bytes_per_rhs > 0 && !d_work))
    return fail(HM_ENOMEM, "workspace has %zu bytes, needs %zu", work_bytes, A->work_bytes_per_rhs);
  if (d_work && ((uintptr_t)d_work) % kAlign) return fail(HM_EINVAL, "workspace must be 256-byte aligned");
  return ok();
}

static hm_status check_batch(const hm_matrix* A, int32_t nrhs, const void* d_X, int64_t ldx,
                             const void* d_Y, int64_t ldy, const void* d_work, size_t work_bytes) {
  if (!A || !d_X || !d_Y) return fail(HM_EINVAL, "NULL argument");
  if (nrhs < 1 || nrhs > A->max_nrhs) return fail(HM_EINVAL, "nrhs %d outside [1, %d]", nrhs, A->max_nrhs);
  if (ldx < A->hdr.n_cols || ldy < A->hdr.n_rows) return fail(HM_EINVAL, "leading dimension too small");
  const size_t need = (size_t)batch_slots(A->acc_dtype, nrhs) * A->work_bytes_per_rhs;
  if (work_bytes < need || (need > 0 && !d_work))
    return fail(HM_ENOMEM, "workspace has %zu bytes, needs %zu", work_bytes, need);
  if (d_work && ((uintptr_t)d_work) % kAlign) return fail(HM_EINVAL, "workspace must be 256-byte aligned");
  const int vs = A->acc_dtype == HM_F64 ? 8 : 4;
  const uint8_t* X = (const uint8_t*)d_X;
  const uint8_t* Y = (const uint8_t*)d_Y;
  if (X < Y + (size_t)ldy * vs * nrhs && Y < X + (size_t)ldx * vs * nrhs)
    return fail(HM_EINVAL, "X must not overlap Y");
  return ok();
}

hm_status hm_mvm(const hm_matrix* A, double alpha, const void* d_x, void* d_y, void* d_work,
                 size_t work_bytes, void* stream) {
  if (hm_status st = check_mvm(A, d_x, d_y, d_work, work_bytes)) return st;
  hipError_t e = launch_mvm(*A, alpha, d_x, d_y, d_work, (hipStream_t)stream);
  if (e != hipSuccess) return fail(HM_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  return ok();
}

hm_status hm_mvm_noalloc(const hm_matrix* A, double alpha, const void* d_x, void* d_y, void* stream) {
  if (!A || !d_x || !d_y) return fail(HM_EINVAL, "NULL argument");
  if (A->work_bytes_per_rhs > (size_t)HM_NOALLOC_SCRATCH_BYTES)
    return fail(HM_ENOMEM, "the product needs %zu bytes of workspace, above the fixed %zu of hm_mvm_noalloc",
                A->work_bytes_per_rhs, (size_t)HM_NOALLOC_SCRATCH_BYTES);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != A->device)
    return fail(HM_EINVAL, "the current device is not the matrix's device");
  void* work = nullptr;
  hipError_t e = scratch_address(dev, &work);
  if (e != hipSuccess) return fail(HM_EDEVICE, "fixed workspace lookup failed: %s", hipGetErrorString(e));
  if (hm_status st = check_mvm(A, d_x, d_y, work, HM_NOALLOC_SCRATCH_BYTES)) return st;
  e = launch_mvm(*A, alpha, d_x, d_y, work, (hipStream_t)stream);
  if (e != hipSuccess) return fail(HM_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  return ok();
}

hm_status hm_mvm_batch(const hm_matrix* A, int32_t nrhs, double alpha, const void* d_X,
                       int64_t ldx, void* d_Y, int64_t ldy, void* d_work, size_t work_bytes,
                       void* stream) {
  if (hm_status st = check_batch(A, nrhs, d_X, ldx, d_Y, ldy, d_work, work_bytes)) return st;
  hipError_t e = launch_mvm_batch(*A, nrhs, alpha, d_X, ldx, d_Y, ldy, d_work, (hipStream_t)stream);
  if (e != hipSuccess) return fail(HM_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  return ok();
}

// ------------------------------------------------------------------ graphs

struct hm_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t device = 0;
};

void hm_graph_destroy(hm_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

hm_status hm_graph_create(const hm_matrix* A, int32_t nrhs, double alpha, const void* d_X, int64_t ldx,
                          void* d_Y, int64_t ldy, void* d_work, size_t work_bytes, hm_graph** out) {
  if (!out) return fail(HM_EINVAL, "out is NULL");
  *out = nullptr;
  if (nrhs == 1) {
    if (hm_status st = check_mvm(A, d_X, d_Y, d_work, work_bytes)) return st;
  } else if (hm_status st = check_batch(A, nrhs, d_X, ldx, d_Y, ldy, d_work, work_bytes)) {
    return st;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != A->device)
    return fail(HM_EINVAL, "the current device is not the matrix's device");
  auto* G = new (std::nothrow) hm_graph();
  if (!G) return fail(HM_ENOMEM, "host allocation failed");
  G->device = dev;
  // a private stream in capture mode: the launches become graph nodes
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t le = nrhs == 1
        ? launch_mvm(*A, alpha, d_X, d_Y, d_work, cs, nullptr, false)
        : launch_mvm_batch(*A, nrhs, alpha, d_X, ldx, d_Y, ldy, d_work, cs, false);
    e = hipStreamEndCapture(cs, &G->graph);
    if (e == hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
  if (cs) (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    hm_graph_destroy(G);
    return fail(HM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  }
  *out = G;
  return ok();
}

hm_status hm_graph_launch(hm_graph* g, void* stream) {
  if (!g) return fail(HM_EINVAL, "NULL argument");
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(HM_EDEVICE, "graph launch failed: %s", hipGetErrorString(e));
  return ok();
}

hm_status hm_matrix_set_launch(hm_matrix* A, const char* params) {
  if (!A || !params) return fail(HM_EINVAL, "NULL argument");
  LaunchParams lp = A->launch;
  if (!parse_launch(params, lp)) return fail(HM_EINVAL, "bad launch parameters '%s'", params);
  if (lp.chunk != A->launch.chunk || lp.tile != A->launch.tile || lp.tmix != A->launch.tmix)
    return fail(HM_EINVAL, "the tile shape (chunk, tile, tmix) is the plan's; set it when the plan is built");
  A->launch = lp;
  return ok();
}

hm_status hm_matrix_get_launch(const hm_matrix* A, char* buf, size_t len) {
  if (!A || !buf || len == 0) return fail(HM_EINVAL, "NULL argument");
  std::snprintf(buf, len, "schedule=%d unroll=%d order=%d persist=%d chunk=%d tile=%d colb=%d tmix=%d colw=%d",
                A->launch.schedule, A->launch.row_unroll, A->launch.order, A->launch.persist, A->launch.chunk,
                A->launch.tile, A->launch.colb, A->launch.tmix, A->launch.colw);
  return ok();
}

hm_status hm_matrix_tune_key(const hm_matrix* A, char* buf, size_t len) {
  if (!A || !buf || len == 0) return fail(HM_EINVAL, "NULL argument");
  std::snprintf(buf, len, "%s",
                tune_key(A->acc_dtype, A->bytes_by_dtype, A->hdr.n_rows, A->rank_class, A->max_nrhs).c_str());
  return ok();
}

hm_status hm_stream_read(const void* d_buf, size_t bytes, void* d_out, void* stream) {
  if (!d_buf || !d_out || bytes % 16) return fail(HM_EINVAL, "bad stream-read arguments");
  if (((uintptr_t)d_buf) % 16) return fail(HM_EINVAL, "buffer must be 16-byte aligned");
  hipError_t e = launch_stream_read(d_buf, bytes, d_out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(HM_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  return ok();
}

hm_status hm_permute(const int64_t* d_perm, int64_t n, int32_t dtype, int32_t direction, int32_t nvec,
                     const void* d_in, int64_t ld_in, void* d_out, int64_t ld_out, void* stream) {
  if (!d_perm || !d_in || !d_out) return fail(HM_EINVAL, "NULL argument");
  if (n < 1 || nvec < 1 || ld_in < n || ld_out < n)
    return fail(HM_EINVAL, "bad sizes n=%lld nvec=%d ld_in=%lld ld_out=%lld", (long long)n, nvec,
                (long long)ld_in, (long long)ld_out);
  if (direction != 0 && direction != 1) return fail(HM_EINVAL, "direction must be 0 or 1");
  if (dtype != HM_F64 && dtype != HM_F32) return fail(HM_EDTYPE, "dtype must be HM_F64 or HM_F32");
  hipError_t e = launch_permute(d_perm, n, dtype == HM_F64 ? 8 : 4, direction, nvec, d_in, ld_in, d_out, ld_out,
                                (hipStream_t)stream);
  if (e != hipSuccess) return fail(HM_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  return ok();
}

const char* hm_last_error(void) { return hm::g_err.c_str(); }

}  // extern "C"
