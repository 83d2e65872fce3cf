// Quantity of interest and the parameter contraction of the adjoint gradient.
//
// Q(U) = w_mean . U[:,0] + sum_{j>=1} w_var . U[:,j]^2 (mean of E[u] and the
// integral of Var[u] for a normalised chaos basis). With A Lambda = dQ/dU,
// dQ/dtheta = -<Lambda, (dA/dtheta) U>; for theta0 the derivative of the
// SG matrix is I (x) K_Lap, for the KL amplitude s_k it is
// G_k (x) K[sigma phi_k]. Per element e the contraction is
//   sum_{(a,b): (G_k)_ab = g != 0} g * Lambda_a(e)^T K^e U_b(e) * c_k(e)
// with the Q1 element matrix K^e and c_0 = 1.
#include "sg_internal.h"

namespace sgk {

namespace {

constexpr int kT = 256;

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

__global__ void __launch_bounds__(kT) qoi_kernel(const double* __restrict__ U, const double* __restrict__ wm,
                                                  const double* __restrict__ wv, long n, int P,
                                                  double* partials) {
  double acc = 0.0;
  const long N = n * (long)P;
  const long stride = (long)gridDim.x * kT;
  for (long idx = (long)blockIdx.x * kT + threadIdx.x; idx < N; idx += stride) {
    const long j = idx / n, i = idx - j * n;
    const double u = U[idx];
    acc += j == 0 ? wm[i] * u : wv[i] * u * u;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kT) finalize1_kernel(const double* partials, int nb, double* out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += kT) v += partials[i];
  v = block_sum(v);
  if (threadIdx.x == 0) out[0] = v;
}

__global__ void __launch_bounds__(kT) qoi_grad_kernel(const double* __restrict__ U, const double* __restrict__ wm,
                                                       const double* __restrict__ wv, long n, int P,
                                                       double* __restrict__ G) {
  const long N = n * (long)P;
  const long stride = (long)gridDim.x * kT;
  for (long idx = (long)blockIdx.x * kT + threadIdx.x; idx < N; idx += stride) {
    const long j = idx / n, i = idx - j * n;
    G[idx] = j == 0 ? wm[i] : 2.0 * wv[i] * U[idx];
  }
}

__device__ __forceinline__ double node_val(const double* col, int gx, int gy, int nx) {
  return (gx >= 1 && gx <= nx && gy >= 1 && gy <= nx) ? col[(long)(gy - 1) * nx + (gx - 1)] : 0.0;
}

// lambda^T K^e u for the Q1 element matrix (1/6)[[4,-1,-2,-1],[-1,4,-1,-2],[-2,-1,4,-1],[-1,-2,-1,4]],
// corners counter-clockwise from the lower-left.
__device__ __forceinline__ double elem_form(const double l[4], const double u[4]) {
  const double k0 = 4.0 * u[0] - u[1] - 2.0 * u[2] - u[3];
  const double k1 = -u[0] + 4.0 * u[1] - u[2] - 2.0 * u[3];
  const double k2 = -2.0 * u[0] - u[1] + 4.0 * u[2] - u[3];
  const double k3 = -u[0] - 2.0 * u[1] - u[2] + 4.0 * u[3];
  return (l[0] * k0 + l[1] * k1 + l[2] * k2 + l[3] * k3) / 6.0;
}

__global__ void __launch_bounds__(kT) contract_kernel(const ContractArgs A) {
  const long ne2 = (long)A.n_e * A.n_e;
  const long e = (long)blockIdx.x * kT + threadIdx.x;
  const bool active = e < ne2;
  const int ex = active ? (int)(e % A.n_e) : 0;
  const int ey = active ? (int)(e / A.n_e) : 0;
  const int cx[4] = {0, 1, 1, 0}, cy[4] = {0, 0, 1, 1};
  for (int k = 0; k <= A.M; ++k) {
    double acc = 0.0;
    if (active) {
      if (k == 0) {
        for (int a = 0; a < A.P; ++a) {
          const double* la = A.Lam + (long)a * A.n;
          const double* ua = A.U + (long)a * A.n;
          double l[4], u[4];
          for (int c = 0; c < 4; ++c) {
            l[c] = node_val(la, ex + cx[c], ey + cy[c], A.nx);
            u[c] = node_val(ua, ex + cx[c], ey + cy[c], A.nx);
          }
          acc += elem_form(l, u);
        }
      } else {
        for (int q = A.pair_ptr[k - 1]; q < A.pair_ptr[k]; ++q) {
          const double* la = A.Lam + (long)A.pair_a[q] * A.n;
          const double* ub = A.U + (long)A.pair_b[q] * A.n;
          double l[4], u[4];
          for (int c = 0; c < 4; ++c) {
            l[c] = node_val(la, ex + cx[c], ey + cy[c], A.nx);
            u[c] = node_val(ub, ex + cx[c], ey + cy[c], A.nx);
          }
          acc += A.pair_g[q] * elem_form(l, u);
        }
        acc *= A.c[(long)(k - 1) * ne2 + e];
      }
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) A.partials[(long)blockIdx.x * (A.M + 1) + k] = -t;
  }
}

__global__ void __launch_bounds__(kT) contract_finalize(const double* partials, int nb, int nk, double* out) {
  for (int k = 0; k < nk; ++k) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += kT) v += partials[(long)i * nk + k];
    v = block_sum(v);
    if (threadIdx.x == 0) out[k] = v;
  }
}

}  // namespace

void launch_qoi(const double* U, const double* wm, const double* wv, long n, int P, double* partials, double* out,
                hipStream_t s) {
  hipLaunchKernelGGL(qoi_kernel, dim3(kRedBlocks), dim3(kT), 0, s, U, wm, wv, n, P, partials);
  hipLaunchKernelGGL(finalize1_kernel, dim3(1), dim3(kT), 0, s, partials, kRedBlocks, out);
}

void launch_qoi_grad(const double* U, const double* wm, const double* wv, long n, int P, double* G, hipStream_t s) {
  long g = (n * (long)P + kT - 1) / kT;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(qoi_grad_kernel, dim3((unsigned)g), dim3(kT), 0, s, U, wm, wv, n, P, G);
}

void launch_contract(const ContractArgs& args, hipStream_t s) {
  const long ne2 = (long)args.n_e * args.n_e;
  const int nb = (int)((ne2 + kT - 1) / kT);
  hipLaunchKernelGGL(contract_kernel, dim3(nb), dim3(kT), 0, s, args);
  hipLaunchKernelGGL(contract_finalize, dim3(1), dim3(kT), 0, s, args.partials, nb, args.M + 1, args.out);
}

}  // namespace sgk
