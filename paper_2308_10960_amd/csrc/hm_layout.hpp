// Device-side layout of a packed H-matrix store (shared by the host packer
// and the HIP kernels; plain structs, no HIP types).
//
// The product y += alpha * sum_b E_tau M_b E_sigma^T x is regrouped so that
// every kernel streams contiguous, dtype-homogeneous panels:
//
//  * Row panels.  The row breakpoints of all leaf blocks cut [0, n_rows) into
//    elementary row intervals (at most 64 rows after splitting).  For one
//    such interval rho, every leaf block whose row cluster contains rho
//    contributes its rows restricted to rho: all n_b columns of a dense D_b
//    (source x[sigma]) and the k columns of U_b / W_b (source t_b).  The
//    panel is stored per storage dtype ("section") in column groups of G
//    columns, element (i, c) of group g at ((g*m + i)*G + c): one 16-byte
//    load per lane (lane = row) covers G columns.  A section of a format
//    with a low-byte plane (DFL40, DFL48) has that plane after its groups:
//    the low bytes of group element (g, i) at 16 ngroups m + L (g*m + i),
//    L = lo_bytes (one more 4- or 8-byte load per lane).  The kernel owns y[rho]:
//    y[rho] += alpha * P_rho z_rho, with z the gathered sources.
//  * Column tiles.  The rows of every V_b / X_b are cut into chunks kappa of
//    at most 512 rows: sigma_b itself if small, else its largest sub-clusters
//    of at most 512 rows (the block ranges form the cluster tree).  For each
//    chunk, the rows of V_b restricted to kappa are concatenated over all
//    low-rank blocks that have kappa as a chunk.  The
//    section is cut into tiles of 64 groups of G columns, stored one after
//    another; inside a tile the rows follow each other, each holding the
//    tile's groups contiguously, so a wave (lane = group) streams one
//    contiguous block and accumulates its G columns over the rows:
//    partial(b, kappa, l) = sum_{i in kappa} V_b[i, l] x[i].  A tile with
//    runs of formats with a low-byte plane has the plane after its rows: the
//    low bytes of row i, group g at 16 nrows ngroups + L (i ngroups + g),
//    L = the largest lo_bytes of its runs (entries of groups of the other
//    formats are unused).  AFLP values are stored like DFL values of the
//    same byte count; their per-column decode parameters sit in tables
//    beside the row-source and destination tables.
//  * Reduction.  t_b[l] = s_b[l] * sum over the chunks of sigma_b of the
//    partials, in ascending chunk order.
//  * Single-RHS schedule: phase 1 streams the dense sections of the row
//    panels (y += alpha D x) together with the column tiles in one grouped
//    launch; after the reduction, phase 2 streams the U sections
//    (y += alpha U t).  Each row of y is written by one workgroup per phase,
//    in phase order.
//
// All offsets are in bytes from the start of the store unless noted.

#pragma once
#include <stdint.h>

namespace hm {

constexpr int kMaxPanelRows = 64;   // rows per row panel (one wave's lanes)
constexpr int kMaxTileRows = 64;    // rows per fallback column piece
constexpr int kSegRows = 512;       // rows per column chunk (cluster sub-ranges up to this size)
constexpr int kTileGroups = 64;     // column groups per column tile (one per lane)
constexpr int kLargeSeg = 16;       // blocks with more intervals reduce per workgroup
constexpr int kAlign = 256;

// Storage formats (hm_dtype): F64, F32, F16, BF16, DFL32, DFL40, DFL48,
// DFL16, DFL24, AFLP16, AFLP24, AFLP32, AFLP40, AFLP48, BFL24, BFL40, BFL48.
constexpr int kNumDtypes = 17;
constexpr int kDtDfl32 = 4, kDtDfl40 = 5, kDtDfl48 = 6, kDtDfl16 = 7, kDtDfl24 = 8;
constexpr int kDtAflp16 = 9, kDtAflp24 = 10, kDtAflp32 = 11, kDtAflp40 = 12, kDtAflp48 = 13;
constexpr int kDtBfl24 = 14, kDtBfl40 = 15, kDtBfl48 = 16;

inline constexpr bool is_dfl(int dt) { return dt >= kDtDfl32 && dt <= kDtDfl24; }
inline constexpr bool is_aflp(int dt) { return dt >= kDtAflp16 && dt <= kDtAflp48; }
inline constexpr bool is_bfl(int dt) { return dt >= kDtBfl24 && dt <= kDtBfl48; }
// AFLP and BFL values of B bytes are stored like the DFL values of B bytes
// (a left-aligned B-byte code split into the same leading and low parts).
inline constexpr int storage_dt(int dt) {
  return dt == kDtAflp16 ? kDtDfl16 : dt == kDtAflp24 ? kDtDfl24 : dt == kDtAflp32 ? kDtDfl32
       : dt == kDtAflp40 ? kDtDfl40 : dt == kDtAflp48 ? kDtDfl48 : dt == kDtBfl24 ? kDtDfl24
       : dt == kDtBfl40 ? kDtDfl40 : dt == kDtBfl48 ? kDtDfl48 : dt;
}

// Columns per 16-byte group for a storage dtype.  A DFL value keeps its
// leading 4 bytes (DFL32 / 40 / 48: the high 32-bit word of its FP64
// encoding) or 2 bytes (DFL16 / 24: the high 16 bits) in the group.
inline constexpr int group_width(int dt) {
  return dt == 0 ? 2 : (dt == 2 || dt == 3 || storage_dt(dt) == kDtDfl16 || storage_dt(dt) == kDtDfl24) ? 8 : 4;
}
// Bytes per value inside the 16-byte groups.
inline constexpr int dtype_size(int dt) { return 16 / group_width(dt); }
// DFL40 / DFL48 / DFL24 keep the rest of each value (1 / 2 / 1 bytes: bits
// 31..24 / 31..16 / 47..40 of the encoding) in a low-byte plane: lo_bytes
// per 16-byte group element (4, 8 or 8 values), 0 for the other formats.
inline constexpr int lo_bytes(int dt) {
  return storage_dt(dt) == kDtDfl40 ? 4 : (storage_dt(dt) == kDtDfl48 || storage_dt(dt) == kDtDfl24) ? 8 : 0;
}
// Stored bytes per value.
inline constexpr int value_bytes(int dt) { return dtype_size(dt) + lo_bytes(dt) / group_width(dt); }

// AFLP (Sec. 3.2) of one data block (a dense block, or the columns of one
// column group of U_b or of V_b): with 2^k the power of two at or below the
// block's smallest nonzero magnitude, a value v is stored through
// d = |v| 2^-k + 1 >= 2 rounded to m mantissa bits: a B-byte code holding
// the sign, e bits of the binary exponent of d (1 .. 2^e - 1; 0 is the code
// of zero, d = 1) and the m = 8B - 1 - e leading mantissa bits of d.  With
// the code left-aligned in 64 bits (P, as a DFL encoding), the decoded value
// is sign(P) (d - 1) 2^k with d the FP64 number of bits
// ((P & ~sign) >> (11 - e)) + bits(1.0).  Per column, the store keeps
// aflp_param(k, e): the kernels scale by 2^k where it is exact (x and t
// gathered for a row panel, a column tile's sums) and decode d - 1.
inline constexpr int32_t aflp_param(int k, int e) { return k * 256 + (11 - e); }
inline constexpr int aflp_scale_exp(int32_t p) { return p >> 8; }    // k (arithmetic shift)
inline constexpr int aflp_shift(int32_t p) { return p & 0xff; }      // 11 - e

// BFL (Sec. 3.2): FP32's sign and 8 exponent bits (bias 127) and the
// 8B - 9 leading mantissa bits of a value, rounded to nearest even from
// FP64; B = 2 and 4 are BF16 and FP32, stored as such.  With the code
// left-aligned in 64 bits (P), a nonzero value is the FP64 number of bits
// ((P & ~sign) >> 3) + (896 << 52), sign from P (896 = 1023 - 127); P = 0
// is zero (magnitudes below 2^-126 are stored as zero).
constexpr unsigned long long kBflRebias = 896ull << 52;

struct RowPanel {        // 32 bytes
  int64_t src_off;       // first entry (int32 units) in the row-source table
  int32_t row0, m;       // rows [row0, row0 + m), m <= 64
  int32_t ncols;         // source slots over all sections (each section starts at a multiple of 8)
  int32_t sec0, nsec;    // sections [sec0, sec0 + nsec) in the section table
  int32_t nsec_dense;    // the first nsec_dense sections hold dense blocks (source x),
                         // the rest U factors (source t); dense slots come first
};

struct RowSection {      // 32 bytes
  int64_t data_off;      // byte offset of group 0
  int32_t dtype;         // storage dtype (hm_dtype)
  int32_t ngroups;       // groups of group_width(dtype) columns
  int32_t col0;          // first source slot of the section (a multiple of 8)
  int32_t pad_[3];
};

struct ColTile {         // 32 bytes: nrows rows x ngroups 16-byte groups
  int64_t data_off;      // byte offset of the tile (row 0, first group); row i at + 16 i ngroups
                         // (low-byte plane, if any, from + 16 nrows ngroups)
  int32_t nrows;         // rows of the column chunk (<= 512)
  int32_t x0;            // first x index of the chunk
  int32_t ngroups;       // groups in this tile (<= 64)
  int32_t dst_off;       // first entry (int32 units) of this tile in the destination table
  uint8_t dtype[4];      // storage format of run r of groups (formats in ascending order)
  uint8_t end[4];        // end (exclusive) of run r, in groups; end[3] == ngroups
};

// Run, format and first column (in the tile's column order: run by run,
// group by group) of group g of tile T (constant indices only, so that a
// descriptor in registers stays there).
struct TileGroup { int run, dtype, col; };
inline constexpr TileGroup tile_group(const ColTile& T, int g) {
  const int r = (g >= T.end[0]) + (g >= T.end[1]) + (g >= T.end[2]);
  int col = 0, start = 0, dt = T.dtype[0];
  for (int q = 0; q < 4; ++q) {                     // unrolled: constant indices
    if (q == r) {
      dt = T.dtype[q];
      col += (g - start) * group_width(T.dtype[q]);
    } else if (q < r) {
      col += (T.end[q] - start) * group_width(T.dtype[q]);
      start = T.end[q];
    }
  }
  return TileGroup{r, dt, col};
}

// Destination of a column sum (one int32 per tile column): e >= 0 is the
// partial e; e == -1 is a padding column; e <= -2 is t entry -e - 2 (the
// block lies in one column chunk; the sum, times s_b when kept, is t).
constexpr int32_t kDstPad = -1;
inline constexpr int32_t dst_direct(int32_t t_index) { return -t_index - 2; }
inline constexpr int32_t dst_t_index(int32_t e) { return -e - 2; }

struct TBlock {          // 16 bytes: reduction of one low-rank block's partials
  int32_t pst;           // first partial (acc units); partial (seg, l) at pst + seg*k + l
  int32_t k;             // rank
  int32_t nseg;          // column chunks of sigma_b
  int32_t toff;          // first entry of t_b in t
};

// Header at offset 0 of the store; every table offset is a byte offset.
struct StoreHeader {
  uint64_t magic;
  int64_t n_rows, n_cols;
  int64_t n_row_panels, n_row_sections, n_col_tiles, n_tblocks;
  int64_t n_large, n_large_t, n_t, n_partials;
  int64_t off_row_panels, off_row_sections, off_row_order, off_row_src;
  int64_t off_col_tiles, off_col_dst;
  int64_t off_tblocks, off_large, off_owner, off_sigma;
  int64_t acc_dtype, has_sigma;
  // single-RHS work orders: phase 1 mixes the dense parts of row panels
  // (entry >= 0: panel index) with column tiles (entry < 0: tile -entry-1);
  // phase 2 lists the row panels with U sections
  int64_t off_p1_order, n_p1, off_p2_order, n_p2;
  // t entries [0, n_red_t) come from partials (blocks over several column
  // chunks: the n_large largest first, whose entries are [0, n_large_t));
  // the blocks inside one column chunk, [n_red_t, n_t), get t directly from
  // the column tiles
  int64_t n_red_t;
  // AFLP: one aflp_param per row-source slot (off_row_aflp, n_row_src
  // entries, parallel to the row-source table) and per column-tile column
  // (off_col_aflp, parallel to the destination table); 0 for the columns of
  // other formats.  has_aflp = 0: no AFLP data and no such tables.
  int64_t has_aflp, off_row_aflp, off_col_aflp;
  // column tiles by class: tiles of one storage format f are
  // [tile_class_end[f-1], tile_class_end[f]) (tile_class_end[-1] = 0), tiles
  // with runs of several formats [tile_class_end[kNumDtypes-1],
  // tile_class_end[kNumDtypes])
  int64_t tile_class_end[kNumDtypes + 1];
};

// Low-byte plane entry bytes of a tile: the largest lo_bytes of its runs.
inline constexpr int tile_lo_bytes(const ColTile& T) {
  int L = 0;
  for (int q = 0; q < 4; ++q) L = L > lo_bytes(T.dtype[q]) ? L : lo_bytes(T.dtype[q]);
  return L;
}

// Class of a column tile: its format if it has one, else kNumDtypes.
inline constexpr int tile_class(const ColTile& T) {
  return T.end[0] == T.ngroups ? T.dtype[0] : kNumDtypes;
}

constexpr uint64_t kStoreMagic = 0x484d53544f524535ull;  // "HMSTORE5"

}  // namespace hm
