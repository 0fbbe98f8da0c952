// Host-side plan and matrix objects of libhm (not part of the C-ABI).
#pragma once
#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/hm.h"
#include "hm_layout.hpp"

namespace hm {

// Launch parameters (chosen by the tuner or built-in defaults).
//  schedule 0: column tiles, reduction, whole row panels;
//  schedule 1: grouped launch of dense row-panel sections with the column
//              tiles, reduction, then the U sections.
//  row_unroll: 16-byte groups in flight per wave in the row-panel loop (4, 8).
//  order 0: row panels largest first; order 1: cluster order in 8
//           contiguous ranges, one per XCD (whole-panel kernels).
//  persist 0: one workgroup per work item; P > 0: persistent grids of at
//           most P workgroups per CU looping over the items (single RHS).
//  chunk, tile: the plan's column-tile shape (rows per column chunk, groups
//           per tile); 0 = not given.
//  colb: batched FP32 column tiles as 8-byte slots, 32 per wave (0: 4 row
//           steps in flight, 2: 8), or as 16-byte groups, 32 per wave (1: 4
//           steps, 3: 8).
//  tmix: 0: every column tile holds one storage format (a chunk's runs of
//           different formats start new tiles); 1: a tile may hold runs of
//           up to four formats (part of the plan's tile shape).
struct LaunchParams {
  int schedule = 0;
  int row_unroll = 8;
  int order = 1;
  int persist = 0;
  int chunk = 0;
  int tile = 0;
  int colb = 0;
  int tmix = 0;
  int colw = 1;           // column tiles: 0 a workgroup per tile, 2 a wave per tile, 1 per launch class (col_wave)
};

struct BlockInfo {
  int64_t toff = 0;       // first entry of t_b
  int64_t pst = 0;        // first partial
  int32_t nseg = 0;       // column chunks of sigma_b
};

// A run of consecutive columns of one block inside a panel section.
struct Seg {
  int32_t block;
  int32_t c_first;        // first column of the block (dense col or low-rank l)
  int32_t ncols;
  int32_t src0;           // row panels: source slot of the first column;
                          // column panels: partial index of the first column,
                          // or its t index when direct
  int32_t dtype;
  int32_t seccol;         // column within its section
  int32_t kind;           // HM_DENSE or HM_LOWRANK
  int32_t direct = 0;     // column panels: the block lies in one column chunk,
                          // so its column sums are t itself
};

struct RowSectionHost { int32_t kind = 0, dtype = 0, ngroups = 0, col0 = 0; int64_t data_off = 0; };
struct RowPanelHost {
  int64_t row0 = 0;
  int32_t m = 0, ncols = 0, nsec_dense = 0;
  int64_t src_off = 0;
  std::vector<Seg> segs;
  std::vector<RowSectionHost> secs;
};
// A column panel (one column chunk) stores the groups of all its low-rank
// columns as one sequence ordered by storage format: run r holds the ld
// columns (a multiple of the group width) of one format, from group g0 and
// from column c0 of the panel's column order.
struct ColSectionHost { int32_t dtype = 0, ld = 0, g0 = 0, c0 = 0; };
// Its groups are cut into tiles of at most kTileGroups groups; a run of a
// format with a low-byte plane gets tiles of its own (tile t: groups
// [tile_g0[t], tile_g0[t+1]), bytes from data_off + tile_off[t], low-byte
// plane entry size tile_lo[t]).
struct ColPanelHost {
  int64_t x0 = 0;
  int32_t nrows = 0;
  int32_t ngroups = 0, ncols = 0;    // all runs (ncols counts padding)
  int64_t data_off = 0;
  std::vector<Seg> segs;
  std::vector<ColSectionHost> secs;  // the runs, by format
  std::vector<int32_t> tile_g0;      // n_tiles + 1 entries
  std::vector<int64_t> tile_off;     // n_tiles + 1 entries (the last: the panel's bytes)
  std::vector<int32_t> tile_lo;      // n_tiles entries
};

}  // namespace hm

struct hm_plan {
  int64_t n_rows = 0, n_cols = 0;
  hm_plan_opts opts{};
  std::string tune_path;
  std::vector<hm_block_desc> blocks;
  std::vector<hm::BlockInfo> binfo;
  std::vector<int64_t> rint;              // elementary row interval boundaries (after splitting)
  std::vector<int64_t> chunk_off;         // per block: [chunk_off[b], chunk_off[b+1]) into chunk_list
  std::vector<int32_t> chunk_list;        // column panel (chunk) of each segment of each block
  std::vector<hm::RowPanelHost> rps;
  std::vector<hm::ColPanelHost> cps;
  std::vector<int32_t> lr_order;          // low-rank blocks in t order (large first)
  int64_t n_t = 0, n_partials = 0, n_large = 0, n_large_t = 0, n_red_t = 0;
  int32_t has_sigma = 0;
  hm::StoreHeader hdr{};
  int32_t chunk_rows = hm::kSegRows, tile_groups = hm::kTileGroups;   // column-tile shape
  int32_t rank_class = 0;                 // floor(log2) of the mean low-rank rank (tune key)
  size_t store_bytes = 0, meta_bytes = 0, work_bytes_per_rhs = 0;
  int64_t work_part_off = 0, work_t_off = 0;
  int64_t work_part_bytes = 0, work_t_bytes = 0, work_x_bytes = 0;
  double factor_bytes = 0, alg_bytes = 0, alg_flops = 0, overhead_bytes = 0;
  int64_t n_dense = 0, n_lowrank = 0;
  size_t bytes_by_dtype[hm::kNumDtypes] = {};
  hm::LaunchParams launch;
  // single-RHS column-tile launch classes whose tiles are small enough that
  // a workgroup per tile would leave waves idle (bit 0: the one-format IEEE
  // tiles; bit f: one-format tiles of DFL / AFLP / BFL format f; bit
  // kNumDtypes: several-format tiles)
  uint32_t col_wave = 0;
};

namespace hm {
// Per-call kernel events for hm_profile_begin / hm_profile_end.
struct Profile {
  bool on = false;
  int32_t max_calls = 0, calls = 0;
  std::vector<hipEvent_t> ev;   // 4 per call: before col, before reduce, before row, after row
};
}  // namespace hm

struct hm_matrix {
  hm::StoreHeader hdr{};
  mutable hm::Profile prof;
  const uint8_t* d_store = nullptr;
  size_t store_bytes = 0, work_bytes_per_rhs = 0;
  int64_t work_t_off = 0;
  int64_t work_part_bytes = 0, work_t_bytes = 0, work_x_bytes = 0;
  int32_t acc_dtype = 0, max_nrhs = 1;
  int32_t device = 0, n_cu = 256;       // device of the store and its compute units
  int32_t rank_class = 0;               // of its plan (tune key)
  hm::LaunchParams launch;
  size_t bytes_by_dtype[hm::kNumDtypes] = {};
  uint32_t col_wave = 0;                // of its plan
};

namespace hm {
// Workspace slots (multiples of work_bytes_per_rhs) hm_mvm_batch needs: the
// FP32 path runs right-hand sides in groups of 32 (one group of up to 64 at a
// time); the FP64 path runs them one by one in a single slot.
inline int batch_slots(int acc_dtype, int nrhs) {
  if (acc_dtype == HM_F64) return 1;
  return nrhs <= 32 ? 32 : 64;
}
hm_status fail(hm_status code, const char* fmt, ...);
hm_status ok();

// AFLP parameters (aflp_param) of the data blocks of a plan's factors:
// block b's dense block at prm[base[b]], the columns of its column group g
// of U_b at prm[base[b] + g] and of V_b at prm[base[b] + ngroups + g]
// (base[b] = -1: the block has no AFLP data).  Built from the factor data
// before packing.
struct AflpTable {
  std::vector<int64_t> base;
  std::vector<int32_t> prm;
  hm_status build(const hm_plan* P, const double* const* a, const double* const* bf);
  // parameter of column col of factor `which` (0: D_b / U_b, 1: V_b) of block
  int32_t get(const hm_plan* P, int64_t block, int which, int64_t col) const;
};
hm_status layout_store(hm_plan* P, hm_plan** out);
void read_tune_cache(hm_plan* P);
uint16_t f64_to_f16(double d);
uint16_t f64_to_bf16(double d);

// Kernel launchers (hm_kernels.hip).  profile = false: never record the
// matrix's timing events (used while a stream is being captured).
hipError_t launch_mvm(const hm_matrix& A, double alpha, const void* x, void* y, void* work,
                      hipStream_t s, hipEvent_t* ev = nullptr, bool profile = true);
hipError_t launch_mvm_batch(const hm_matrix& A, int nrhs, double alpha, const void* X, int64_t ldx,
                            void* Y, int64_t ldy, void* work, hipStream_t s, bool profile = true);
hipError_t launch_stream_read(const void* buf, size_t bytes, void* out, hipStream_t s);
// Device address of the fixed workspace of hm_mvm_noalloc on `device`, which
// must be the current device (looked up on the first call per device).
hipError_t scratch_address(int device, void** out);
hipError_t launch_permute(const int64_t* perm, int64_t n, int elem_bytes, int direction, int nvec, const void* in,
                          int64_t ld_in, void* out, int64_t ld_out, hipStream_t s);
}  // namespace hm
