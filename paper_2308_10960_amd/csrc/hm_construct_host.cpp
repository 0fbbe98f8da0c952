// Host side of the GPU construction of H-matrix leaves (hm_construct.h):
// argument validation, region layout, descriptor upload and the launch.
#include <algorithm>
#include <cmath>
#include <cstdint>

#include <hip/hip_runtime_api.h>

#include "../../include/hm_construct.h"
#include "hm_internal.hpp"

namespace hm {
hipError_t construct_rank_limit(int* rmax);
hipError_t launch_construct(const hm_cblock* d_blocks, int64_t n_blocks, const double* d_points,
                            const hm_construct_opts& o, double* d_out, double* d_scr, int32_t* d_aca_rank,
                            int32_t* d_rank, int r_lds_max, hipStream_t s);
hipError_t launch_construct_pack(const hm_cblock* d_blocks, int64_t n_blocks, const int32_t* d_rank,
                                 const double* d_out, const int64_t* d_off, double* d_packed, int64_t cap,
                                 hipStream_t s);
}  // namespace hm

namespace {

int64_t align2(int64_t v) { return (v + 1) / 2 * 2; }

int64_t out_doubles(const hm_cblock& b) {
  return b.adm ? align2(((int64_t)b.m + b.n) * b.cap + b.cap) : align2((int64_t)b.m * b.n);
}

// U (m x cap), V (n x cap), then m bytes of flags.
int64_t scr_doubles(const hm_cblock& b) {
  return b.adm ? align2(((int64_t)b.m + b.n) * b.cap + ((int64_t)b.m + 7) / 8) : 0;
}

int32_t max_cap(const hm_cblock& b) {
  return (int32_t)std::min<int64_t>(std::min<int64_t>(b.m, b.n), HM_CONSTRUCT_MAX_RANK);
}

}  // namespace

extern "C" {

hm_status hm_construct_layout(hm_cblock* blocks, int64_t n_blocks, int64_t* out_total, int64_t* scr_total) {
  using hm::fail;
  if (!blocks || !out_total || !scr_total || n_blocks < 0) return fail(HM_EINVAL, "bad layout arguments");
  int64_t o = 0, sc = 0;
  for (int64_t i = 0; i < n_blocks; ++i) {
    hm_cblock& b = blocks[i];
    if (b.m < 1 || b.n < 1 || (b.adm != 0 && b.adm != 1))
      return fail(HM_EINVAL, "leaf %lld: m=%d n=%d adm=%d", (long long)i, b.m, b.n, b.adm);
    if (b.adm) {
      if (b.cap == 0) b.cap = max_cap(b);
      if (b.cap < 1 || b.cap > max_cap(b))
        return fail(HM_EINVAL, "leaf %lld: cap %d outside [1, %d]", (long long)i, b.cap, max_cap(b));
    } else {
      b.cap = 0;
    }
    b.out = o;
    b.scr = sc;
    o += out_doubles(b);
    sc += scr_doubles(b);
  }
  *out_total = o;
  *scr_total = sc;
  return hm::ok();
}

hm_status hm_construct_rank_limit(int32_t* rmax) {
  if (!rmax) return hm::fail(HM_EINVAL, "NULL argument");
  int r = 0;
  const hipError_t e = hm::construct_rank_limit(&r);
  if (e != hipSuccess) return hm::fail(HM_EDEVICE, "device query failed: %s", hipGetErrorString(e));
  *rmax = r;
  return hm::ok();
}

hm_status hm_construct(const double* d_points, int64_t n_points, const hm_cblock* h_blocks, int64_t n_blocks,
                       void* d_desc, size_t desc_bytes, const hm_construct_opts* opts, double* d_out,
                       size_t out_bytes, double* d_scr, size_t scr_bytes, int32_t* d_rank, void* stream) {
  using hm::fail;
  if (!d_points || !h_blocks || !d_desc || !opts || !d_out || !d_rank || n_points < 1 || n_blocks < 0)
    return fail(HM_EINVAL, "NULL argument or bad size");
  if (opts->kernel != HM_KERNEL_LAPLACE && opts->kernel != HM_KERNEL_EXP)
    return fail(HM_EINVAL, "unknown kernel %d", opts->kernel);
  if (!(opts->params[0] > 0)) return fail(HM_EINVAL, "params[0] must be > 0");
  if (!(opts->eps_aca > 0) || !(opts->eps > 0)) return fail(HM_EINVAL, "eps_aca and eps must be > 0");
  if (opts->keep_sigma != 0 && opts->keep_sigma != 1) return fail(HM_EINVAL, "keep_sigma must be 0 or 1");
  if (desc_bytes < (size_t)n_blocks * sizeof(hm_cblock)) return fail(HM_ENOMEM, "descriptor buffer too small");
  if ((uintptr_t)d_desc % 16) return fail(HM_EINVAL, "descriptor buffer must be 16-byte aligned");
  const int64_t out_cap = (int64_t)(out_bytes / 8), scr_cap = (int64_t)(scr_bytes / 8);
  bool any_adm = false;
  for (int64_t i = 0; i < n_blocks; ++i) {
    const hm_cblock& b = h_blocks[i];
    if (b.m < 1 || b.n < 1 || (b.adm != 0 && b.adm != 1) || b.rb < 0 || b.cb < 0 || b.rb + b.m > n_points ||
        b.cb + b.n > n_points)
      return fail(HM_EINVAL, "leaf %lld outside the %lld points", (long long)i, (long long)n_points);
    if (b.adm && (b.cap < 1 || b.cap > max_cap(b)))
      return fail(HM_EINVAL, "leaf %lld: cap %d outside [1, %d]", (long long)i, b.cap, max_cap(b));
    if (b.out < 0 || b.out + out_doubles(b) > out_cap || b.scr < 0 || b.scr + scr_doubles(b) > scr_cap)
      return fail(HM_EINVAL, "leaf %lld: region outside its buffer", (long long)i);
    any_adm |= b.adm != 0;
  }
  if (any_adm && !d_scr) return fail(HM_EINVAL, "scratch buffer is NULL");
  int rmax = 0;
  hipError_t e = hm::construct_rank_limit(&rmax);
  if (e != hipSuccess) return fail(HM_EDEVICE, "device query failed: %s", hipGetErrorString(e));
  const hipStream_t s = (hipStream_t)stream;
  e = hipMemcpyAsync(d_desc, h_blocks, (size_t)n_blocks * sizeof(hm_cblock), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hm::launch_construct(static_cast<const hm_cblock*>(d_desc), n_blocks, d_points, *opts, d_out, d_scr,
                             d_rank, d_rank + n_blocks, rmax, s);
  if (e != hipSuccess) return fail(HM_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  return hm::ok();
}

hm_status hm_construct_pack(const void* d_desc, int64_t n_blocks, const int32_t* d_rank, const double* d_out,
                            const int64_t* d_off, double* d_packed, size_t packed_bytes, void* stream) {
  if (!d_desc || !d_rank || !d_out || !d_off || !d_packed || n_blocks < 0)
    return hm::fail(HM_EINVAL, "NULL argument or bad size");
  const hipError_t e = hm::launch_construct_pack(static_cast<const hm_cblock*>(d_desc), n_blocks,
                                                 d_rank + n_blocks, d_out, d_off, d_packed,
                                                 (int64_t)(packed_bytes / 8), (hipStream_t)stream);
  if (e != hipSuccess) return hm::fail(HM_EDEVICE, "launch failed: %s", hipGetErrorString(e));
  return hm::ok();
}

}  // extern "C"
