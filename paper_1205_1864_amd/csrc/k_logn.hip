// Kernels of the lognormal-coefficient SG operator (Section 7, second set of
// experiments): the coefficient is expanded in Hermite chaos to twice the
// solution's degree, so every chaos block couples and the operator is
//   Y_a = sum_b K(c_ab) U_b,  c_ab(e) = sum_i E[psi_i psi_a psi_b] k_i(e),
// with K(c) the Q1 stiffness of the element field c (eq. (global-matrix-block)).
#include <hip/hip_runtime.h>

#include "sg_internal.h"

namespace sgk {

// c_ab(e) for every stored block: one thread per (element, block slot),
// summing the block's (term, triple product) list in a fixed order.
__global__ void __launch_bounds__(256) logn_blocks_kernel(const long* __restrict__ ptr, const int* __restrict__ term,
                                                          const double* __restrict__ g,
                                                          const double* __restrict__ kc, int ne2, int nslots,
                                                          double* __restrict__ C) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne2) return;
  for (int s = blockIdx.y; s < nslots; s += gridDim.y) {
    double acc = 0.0;
    for (long j = ptr[s]; j < ptr[s + 1]; ++j) acc += g[j] * kc[(long)term[j] * ne2 + e];
    C[(long)s * ne2 + e] = acc;
  }
}

// Y[:, a] = sum over the stored blocks (a, b) of K(c_ab) U[:, b]: one thread
// per (interior node, chaos row a). The Q1 element matrix of the unit
// coefficient is (4 on the diagonal, -1 along an edge, -2 across) / 6; nodes
// on the boundary carry zero. The node's 3 x 3 neighbourhood offsets and
// boundary masks are fixed per thread, so every load of a block is
// unconditional (a neighbour off the grid reads the node itself, masked to 0).
__global__ void __launch_bounds__(256) logn_matvec_kernel(const int* __restrict__ rptr, const int* __restrict__ rcol,
                                                          const int* __restrict__ rslot,
                                                          const double* __restrict__ C,
                                                          const double* __restrict__ U, int n_e, long n,
                                                          double* __restrict__ Y) {
  const long xi = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (xi >= n) return;
  const int nx = n_e - 1;
  const int ix = (int)(xi % nx) + 1, iy = (int)(xi / nx) + 1;  // grid node, 1..n_e-1
  const long ne2 = (long)n_e * n_e;
  long off[3][3];
  double msk[3][3];
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int gx = ix + dx - 1, gy = iy + dy - 1;
      const bool in = gx >= 1 && gx <= nx && gy >= 1 && gy <= nx;
      off[dy][dx] = in ? (long)(gy - 1) * nx + (gx - 1) : xi;
      msk[dy][dx] = in ? 1.0 : 0.0;
    }
  // elements below-left, below-right, above-left, above-right of the node
  const long e00 = (long)(iy - 1) * n_e + (ix - 1);
  double y = 0.0;
  for (int r = rptr[a]; r < rptr[a + 1]; ++r) {
    const double* __restrict__ u = U + (long)rcol[r] * n;
    const double* __restrict__ c = C + (long)rslot[r] * ne2;
    double v[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) v[dy][dx] = u[off[dy][dx]] * msk[dy][dx];
    const double c00 = c[e00], c01 = c[e00 + 1], c10 = c[e00 + n_e], c11 = c[e00 + n_e + 1];
    const double uc = 4.0 * v[1][1];
    // element (ey, ex) with the node at one corner: edge neighbours (ox, iy),
    // (ix, oy) and the opposite corner (ox, oy)
    y += c00 * (uc - v[1][0] - v[0][1] - 2.0 * v[0][0]);
    y += c01 * (uc - v[1][2] - v[0][1] - 2.0 * v[0][2]);
    y += c10 * (uc - v[1][0] - v[2][1] - 2.0 * v[2][0]);
    y += c11 * (uc - v[1][2] - v[2][1] - 2.0 * v[2][2]);
  }
  Y[(long)a * n + xi] = y * (1.0 / 6.0);
}

void launch_logn_blocks(const long* ptr, const int* term, const double* g, const double* kc, int ne2, int nslots,
                        double* C, hipStream_t s) {
  if (nslots <= 0) return;
  const int gy = nslots < 65535 ? nslots : 65535;
  hipLaunchKernelGGL(logn_blocks_kernel, dim3((ne2 + 255) / 256, gy), dim3(256), 0, s, ptr, term, g, kc, ne2, nslots,
                     C);
}

void launch_logn_matvec(const int* rptr, const int* rcol, const int* rslot, const double* C, const double* U,
                        int n_e, long n, int P, double* Y, hipStream_t s) {
  if (n <= 0 || P <= 0) return;
  hipLaunchKernelGGL(logn_matvec_kernel, dim3((unsigned)((n + 255) / 256), P), dim3(256), 0, s, rptr, rcol, rslot,
                     C, U, n_e, n, Y);
}

}  // namespace sgk
