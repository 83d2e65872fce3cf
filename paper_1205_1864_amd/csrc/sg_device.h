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

}  // namespace sgk
