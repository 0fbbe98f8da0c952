// HIP kernels (gfx950) outside the product: vector reordering between the
// caller's index order and cluster order (hm_permute).

#include <algorithm>

#include <hip/hip_runtime.h>

#include "hm_internal.hpp"

namespace hm {
namespace {

// Gather (direction 0: out[i] = in[perm[i]]) or scatter (1: out[perm[i]] =
// in[i]) of nvec vectors between the caller's order and cluster order; one
// thread per (i, vector), perm read once per i.  Entries outside [0, n) are
// not dereferenced.
template <typename T>
__global__ __launch_bounds__(256) void k_permute(const int64_t* __restrict__ perm, int64_t n, int direction,
                                                 int nvec, const T* __restrict__ in, int64_t ld_in,
                                                 T* __restrict__ out, int64_t ld_out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t p = perm[i];
  const bool ok = p >= 0 && p < n;
  for (int v = (int)blockIdx.y; v < nvec; v += (int)gridDim.y) {
    if (direction == 0)
      out[(int64_t)v * ld_out + i] = ok ? in[(int64_t)v * ld_in + p] : T(__builtin_nan(""));
    else if (ok)
      out[(int64_t)v * ld_out + p] = in[(int64_t)v * ld_in + i];
  }
}

}  // namespace

hipError_t launch_permute(const int64_t* perm, int64_t n, int elem_bytes, int direction, int nvec, const void* in,
                          int64_t ld_in, void* out, int64_t ld_out, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)std::min(nvec, 64));
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_permute<double>, grid, dim3(256), 0, s, perm, n, direction, nvec,
                       static_cast<const double*>(in), ld_in, static_cast<double*>(out), ld_out);
  else
    hipLaunchKernelGGL(k_permute<float>, grid, dim3(256), 0, s, perm, n, direction, nvec,
                       static_cast<const float*>(in), ld_in, static_cast<float*>(out), ld_out);
  return hipGetLastError();
}

}  // namespace hm
