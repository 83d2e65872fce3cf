// Allocation-free variant of the inner solve: sg_inner_solve_static keeps the
// inner solver's state vectors, partial sums and counters in a fixed device
// array of this library instead of the handle's workspace, for callers that
// cannot allocate device memory. Each device holds its own copy of the array
// (allocated when the library's code object is loaded on it, kept until the
// process ends); host code reaches it only through the address that
// hipGetSymbolAddress returns on that device.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "sg_host.h"
#include "sg_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, void*> g_addr;  // device -> address of its copy of `scratch`

}  // namespace

namespace sgh {

size_t static_scratch_bytes() { return kScratchBytes; }

int static_scratch_address(void** out) {
  int dev = -1;
  SG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_addr.find(dev);
  if (it != g_addr.end()) {
    *out = it->second;
    return SG_OK;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr)
    return fail(SG_EDEVICE, std::string("static scratch: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
  g_addr[dev] = p;
  *out = p;
  return SG_OK;
}

}  // namespace sgh

extern "C" int sg_inner_solve_static(sg_handle h, const double* B, double* X, int32_t ncols, int32_t* iters) {
  using sgh::fail;
  if (!h || !B || !X) return fail(SG_EINVAL, "null argument");
  if ((const double*)X == B) return fail(SG_EINVAL, "B and X must be distinct");
  if (ncols < 0 || ncols > h->P) return fail(SG_EINVAL, "ncols must be in 0..P");
  if (ncols == 0) return SG_OK;
  const size_t need = sgh::inner_scratch_bytes(h, ncols);
  if (need > kScratchBytes)
    return fail(SG_ENOMEM, "sg_inner_solve_static: " + std::to_string(ncols) + " columns need " +
                               std::to_string(need) + " bytes of scratch, more than the static " +
                               std::to_string(kScratchBytes) + " bytes");
  if (!h->static_scratch) {
    int rc = sgh::static_scratch_address(&h->static_scratch);
    if (rc) return rc;
  }
  return sgh::inner_solve_in(h, B, X, ncols, iters, static_cast<char*>(h->static_scratch));
}
