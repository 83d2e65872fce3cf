// Device-side helpers shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace sgk {

// Uniform read of a table the kernels never write: through the constant address
// space so that it becomes a scalar load instead of a vector load plus readfirstlane.
template <typename T>
__device__ __forceinline__ T ld_uniform(const T* p, long i) {
  typedef const __attribute__((address_space(4))) T* cptr;
  return ((cptr)(p))[i];
}

// Whole-wavefront lane shifts (DPP wave_shl / wave_shr by one lane): lane i
// receives the value of lane i + 1 (from_next) or i - 1 (from_prev); the lane
// at the end of the wave receives 0.
__device__ __forceinline__ int dpp_from_next(int v) {  // lane i receives lane i + 1
  return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ int dpp_from_prev(int v) {  // lane i receives lane i - 1
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ double from_next(double v) {
  const int lo = dpp_from_next(__double2loint(v));
  const int hi = dpp_from_next(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_prev(double v) {
  const int lo = dpp_from_prev(__double2loint(v));
  const int hi = dpp_from_prev(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float from_next(float v) { return __int_as_float(dpp_from_next(__float_as_int(v))); }
__device__ __forceinline__ float from_prev(float v) { return __int_as_float(dpp_from_prev(__float_as_int(v))); }

}  // namespace sgk
