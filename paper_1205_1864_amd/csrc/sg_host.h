// Host-side internals of the library shared by the single-problem C interface
// and the multi-problem batch driver.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "sg_internal.h"

namespace sgh {

// Record msg as the thread's last error and return code.
int fail(int code, const std::string& msg);

#define SG_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return sgh::fail(SG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

// Y = sum_k K_k U G_k^T on the handle's stream (FP64).
void matvec(sg_ctx* h, const double* U, double* Y);
// R[level l-1] -= B_l V[level l] (dir 0) or R[level l] -= C_l V[level l-1] (dir 1), precision T.
template <typename T>
void coupling(sg_ctx* h, int l, int dir, T* R, const T* V);
// Number of block products of one coupling call (for the work counters).
long coupling_blocks(const sg_ctx* h, int l, int dir);
// Constants of the inner PCG on the handle's grid (stencil weights, Chebyshev recurrence).
template <typename T>
void fill_pcg_consts(const sg_ctx* h, sgk::PcgArgs<T>& a);
// Chebyshev degree actually used, and the inner tile edge for that degree.
int effective_degree(const sg_ctx* h);
// Schedule parameter of the SG operator variant in use (as in sg_tune_report).
int mv_param(const sg_ctx* h);
int choose_tile(const sg_ctx* h, int degree);
// Up to three FP64 dot products over the handle's n x P blocks, read back into h->host_out.
int dots(sg_ctx* h, int nd, const double* a0, const double* b0, const double* a1 = nullptr,
         const double* b1 = nullptr, const double* a2 = nullptr, const double* b2 = nullptr);

// Scratch of the inner solver outside the workspace (sg_inner_solve_static):
// bytes needed for ncols columns, and the solve with every buffer beyond B and
// X inside `scratch` (device, 256-byte aligned, at least that long).
size_t inner_scratch_bytes(const sg_ctx* h, int ncols);
int inner_solve_in(sg_ctx* h, const double* B, double* X, int ncols, int32_t* iters, char* scratch);
// Device address of this device's copy of the library's static scratch array
// (resolved once per device, with that device current), and its size.
int static_scratch_address(void** out);
size_t static_scratch_bytes();

}  // namespace sgh
