// FP64 vector kernels of the outer flexible CG (Section 5) and the precision
// casts at the boundary of the preconditioner. Reductions are two-stage and
// deterministic: a fixed grid writes per-block partials in a fixed order and
// one block sums them in a fixed order.
#include "sg_internal.h"

namespace sgk {

namespace {

constexpr int kT = 256;
constexpr int kMaxDots = 4;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ double block_sum(double v) {
  __shared__ double sred[kT / 64];
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kT / 64; ++w) t += sred[w];
  return t;
}

struct DotArgs {
  const double* a[kMaxDots];
  const double* b[kMaxDots];
  int nd;
  long N;
  double* partials;  // [nd][gridDim.x]
};

__global__ void __launch_bounds__(kT) dots_kernel(DotArgs A) {
  double acc[kMaxDots] = {0.0, 0.0, 0.0, 0.0};
  const long stride = (long)gridDim.x * kT;
  for (long i = (long)blockIdx.x * kT + threadIdx.x; i < A.N; i += stride) {
    for (int d = 0; d < kMaxDots; ++d) {
      if (d < A.nd) acc[d] += A.a[d][i] * A.b[d][i];
    }
  }
  for (int d = 0; d < kMaxDots; ++d) {
    if (d < A.nd) {
      const double t = block_sum(acc[d]);
      if (threadIdx.x == 0) A.partials[(long)d * gridDim.x + blockIdx.x] = t;
    }
  }
}

__global__ void __launch_bounds__(kT) finalize_kernel(const double* partials, int nblocks, int nd, double* out) {
  for (int d = 0; d < nd; ++d) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += kT) v += partials[(long)d * nblocks + i];
    v = block_sum(v);
    if (threadIdx.x == 0) out[d] = v;
  }
}

// x += alpha p, r -= alpha q, partial ||r||^2
__global__ void __launch_bounds__(kT) fcg_update_kernel(double* __restrict__ x, double* __restrict__ r,
                                                         const double* __restrict__ p,
                                                         const double* __restrict__ q, double alpha, long N,
                                                         double* partials) {
  double acc = 0.0;
  const long stride = (long)gridDim.x * kT;
  for (long i = (long)blockIdx.x * kT + threadIdx.x; i < N; i += stride) {
    x[i] += alpha * p[i];
    const double rn = r[i] - alpha * q[i];
    r[i] = rn;
    acc += rn * rn;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kT) xpby_kernel(double* __restrict__ p, const double* __restrict__ z, double beta,
                                                   long N) {
  const long stride = (long)gridDim.x * kT;
  for (long i = (long)blockIdx.x * kT + threadIdx.x; i < N; i += stride) p[i] = z[i] + beta * p[i];
}

__global__ void __launch_bounds__(kT) axpby_kernel(double* __restrict__ y, const double* __restrict__ x, double a,
                                                    double b, long N) {
  const long stride = (long)gridDim.x * kT;
  for (long i = (long)blockIdx.x * kT + threadIdx.x; i < N; i += stride) y[i] = a * x[i] + b * y[i];
}

__global__ void __launch_bounds__(kT) sub_kernel(double* r, const double* f, const double* y, long N) {
  const long stride = (long)gridDim.x * kT;
  for (long i = (long)blockIdx.x * kT + threadIdx.x; i < N; i += stride) r[i] = f[i] - y[i];
}

__global__ void __launch_bounds__(kT) fill_kernel(double* __restrict__ y, double v, long N) {
  const long stride = (long)gridDim.x * kT;
  for (long i = (long)blockIdx.x * kT + threadIdx.x; i < N; i += stride) y[i] = v;
}

template <typename D, typename S>
__global__ void __launch_bounds__(kT) copy_kernel(D* __restrict__ dst, const S* __restrict__ src, long N) {
  const long stride = (long)gridDim.x * kT;
  for (long i = (long)blockIdx.x * kT + threadIdx.x; i < N; i += stride) dst[i] = (D)src[i];
}

int grid_for(long N) {
  long g = (N + kT - 1) / kT;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

void launch_dots(const double* const* a, const double* const* b, int ndots, long N, double* partials, double* out,
                 hipStream_t s) {
  DotArgs A{};
  for (int d = 0; d < ndots; ++d) {
    A.a[d] = a[d];
    A.b[d] = b[d];
  }
  A.nd = ndots;
  A.N = N;
  A.partials = partials;
  hipLaunchKernelGGL(dots_kernel, dim3(kRedBlocks), dim3(kT), 0, s, A);
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kT), 0, s, partials, kRedBlocks, ndots, out);
}

void launch_fcg_update(double* x, double* r, const double* p, const double* q, double alpha, long N,
                       double* partials, double* out, hipStream_t s) {
  hipLaunchKernelGGL(fcg_update_kernel, dim3(kRedBlocks), dim3(kT), 0, s, x, r, p, q, alpha, N, partials);
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kT), 0, s, partials, kRedBlocks, 1, out);
}

void launch_xpby(double* p, const double* z, double beta, long N, hipStream_t s) {
  hipLaunchKernelGGL(xpby_kernel, dim3(grid_for(N)), dim3(kT), 0, s, p, z, beta, N);
}

void launch_axpby(double* y, const double* x, double a, double b, long N, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(N)), dim3(kT), 0, s, y, x, a, b, N);
}

void launch_sub(double* r, const double* f, const double* y, long N, hipStream_t s) {
  hipLaunchKernelGGL(sub_kernel, dim3(grid_for(N)), dim3(kT), 0, s, r, f, y, N);
}

void launch_fill(double* y, double v, long N, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(N)), dim3(kT), 0, s, y, v, N);
}

void launch_copy_d2f(float* dst, const double* src, long N, hipStream_t s) {
  hipLaunchKernelGGL((copy_kernel<float, double>), dim3(grid_for(N)), dim3(kT), 0, s, dst, src, N);
}

void launch_copy_f2d(double* dst, const float* src, long N, hipStream_t s) {
  hipLaunchKernelGGL((copy_kernel<double, float>), dim3(grid_for(N)), dim3(kT), 0, s, dst, src, N);
}

void launch_copy_d2d(double* dst, const double* src, long N, hipStream_t s) {
  hipLaunchKernelGGL((copy_kernel<double, double>), dim3(grid_for(N)), dim3(kT), 0, s, dst, src, N);
}

}  // namespace sgk
