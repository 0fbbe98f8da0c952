// Device-side helpers shared by the single- and multi-right-hand-side
// kernels (gfx950): vector types, the 16-byte streaming load and the
// mapping of launch items to work.
#pragma once

#include <algorithm>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace hm {
namespace {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Index of the calling wave in its workgroup, as a wave-uniform value (so
// that addresses derived from it go through scalar registers and loads).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__device__ __forceinline__ u32x4 ld16(const u32x4* p) { return __builtin_nontemporal_load(p); }

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

}  // namespace
}  // namespace hm
