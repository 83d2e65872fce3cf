// Kernels of the lognormal-coefficient SG operator (Section 6, second set of
// experiments): the coefficient is expanded in Hermite chaos to twice the
// solution's degree, so every chaos block couples and the operator is
//   Y_a = sum_b K(c_ab) U_b,  c_ab(e) = sum_i E[psi_i psi_a psi_b] k_i(e),
// with K(c) the Q1 stiffness of the element field c (eq. (global-matrix-block)).
#include <hip/hip_runtime.h>

#include <algorithm>

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

// Sub-block of the operator for the hierarchical preconditioner: rows
// row0..row0+nrows-1 and columns col0..col1-1 of A (eq. (global-matrix-hierarchy)).
// X holds the columns col0.. (ld n); mode 0: Y = A_sub X; mode 1: Y = R - A_sub X
// (R may be Y). Same element form and summation order as logn_matvec_kernel.
__global__ void __launch_bounds__(256) logn_apply_kernel(const int* __restrict__ rptr, const int* __restrict__ rcol,
                                                         const int* __restrict__ rslot,
                                                         const double* __restrict__ C,
                                                         const double* __restrict__ X, int n_e, long n, int row0,
                                                         int col0, int col1, int mode, const double* R, double* Y) {
  const long xi = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int a = row0 + (int)blockIdx.y;
  if (xi >= n) return;
  const int nx = n_e - 1;
  const int ix = (int)(xi % nx) + 1, iy = (int)(xi / nx) + 1;
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
  const long e00 = (long)(iy - 1) * n_e + (ix - 1);
  double y = 0.0;
  for (int r = rptr[a]; r < rptr[a + 1]; ++r) {
    const int b = rcol[r];
    if (b < col0 || b >= col1) continue;
    const double* __restrict__ u = X + (long)(b - col0) * n;
    const double* __restrict__ c = C + (long)rslot[r] * ne2;
    double v[3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) v[dy][dx] = u[off[dy][dx]] * msk[dy][dx];
    const double c00 = c[e00], c01 = c[e00 + 1], c10 = c[e00 + n_e], c11 = c[e00 + n_e + 1];
    const double uc = 4.0 * v[1][1];
    y += c00 * (uc - v[1][0] - v[0][1] - 2.0 * v[0][0]);
    y += c01 * (uc - v[1][2] - v[0][1] - 2.0 * v[0][2]);
    y += c10 * (uc - v[1][0] - v[2][1] - 2.0 * v[2][0]);
    y += c11 * (uc - v[1][2] - v[2][1] - 2.0 * v[2][2]);
  }
  y *= (1.0 / 6.0);
  const long o = (long)(a - row0) * n + xi;
  Y[o] = mode ? R[o] - y : y;
}

// Y[:, j] = K(c) X[:, j] for ncols columns with one element field c (the
// mean coefficient: the blocks of the mean-based preconditioner).
__global__ void __launch_bounds__(256) logn_mean_apply_kernel(const double* __restrict__ c,
                                                              const double* __restrict__ X, int n_e, long n,
                                                              double* __restrict__ Y) {
  const long xi = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (xi >= n) return;
  const int nx = n_e - 1;
  const int ix = (int)(xi % nx) + 1, iy = (int)(xi / nx) + 1;
  const double* __restrict__ u = X + (long)j * n;
  double v[3][3];
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const int gx = ix + dx - 1, gy = iy + dy - 1;
      const bool in = gx >= 1 && gx <= nx && gy >= 1 && gy <= nx;
      v[dy][dx] = u[in ? (long)(gy - 1) * nx + (gx - 1) : xi] * (in ? 1.0 : 0.0);
    }
  const long e00 = (long)(iy - 1) * n_e + (ix - 1);
  const double c00 = c[e00], c01 = c[e00 + 1], c10 = c[e00 + n_e], c11 = c[e00 + n_e + 1];
  const double uc = 4.0 * v[1][1];
  double y = c00 * (uc - v[1][0] - v[0][1] - 2.0 * v[0][0]);
  y += c01 * (uc - v[1][2] - v[0][1] - 2.0 * v[0][2]);
  y += c10 * (uc - v[1][0] - v[2][1] - 2.0 * v[2][0]);
  y += c11 * (uc - v[1][2] - v[2][1] - 2.0 * v[2][2]);
  Y[(long)j * n + xi] = y * (1.0 / 6.0);
}

// Inverse diagonal of A (Jacobi scaling of the level-block solves): the
// (a, a) block's stencil centre, (4/6) times the sum of c_aa over the four
// elements around the node.
__global__ void __launch_bounds__(256) logn_invdiag_kernel(const int* __restrict__ rptr, const int* __restrict__ rcol,
                                                           const int* __restrict__ rslot,
                                                           const double* __restrict__ C, int n_e, long n,
                                                           double* __restrict__ Dinv) {
  const long xi = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (xi >= n) return;
  const int nx = n_e - 1;
  const int ix = (int)(xi % nx) + 1, iy = (int)(xi / nx) + 1;
  const long e00 = (long)(iy - 1) * n_e + (ix - 1);
  double d = 0.0;
  for (int r = rptr[a]; r < rptr[a + 1]; ++r) {
    if (rcol[r] != a) continue;
    const double* c = C + (long)rslot[r] * n_e * n_e;
    d = (4.0 / 6.0) * (c[e00] + c[e00 + 1] + c[e00 + n_e] + c[e00 + n_e + 1]);
  }
  Dinv[(long)a * n + xi] = d > 0.0 ? 1.0 / d : 0.0;
}

// Partial dot products: block b sums a strided range in a fixed order, then a
// fixed LDS tree; the host adds the partials in index order.
__global__ void __launch_bounds__(256) logn_dot_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                       long len, double* __restrict__ part) {
  __shared__ double sm[256];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x)
    acc += x[i] * y[i];
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// y = a x + b y (b = 0 overwrites y), or y = d * x elementwise with d of
// period dn (mode 1).
__global__ void __launch_bounds__(256) logn_axpby_kernel(long len, double a, const double* __restrict__ x, double b,
                                                         double* __restrict__ y, int mode,
                                                         const double* __restrict__ d, long dn) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x) {
    if (mode == 1) {
      y[i] = d[i % dn] * x[i];
    } else {
      y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
    }
  }
}

// One fused level-solve CG update over a grid-stride range (the grid and
// stride of logn_dot_kernel, so the partial sums have the same order):
//   x += alpha p;  r -= alpha q;  z = d r (d of period dn);
//   partials of r.r into part[0..] and of r.z into part[gridDim.x..].
__global__ void __launch_bounds__(256) logn_cg_update_kernel(long len, double alpha, const double* __restrict__ p,
                                                             const double* __restrict__ q, double* __restrict__ x,
                                                             double* __restrict__ r, const double* __restrict__ d,
                                                             long dn, double* __restrict__ z,
                                                             double* __restrict__ part) {
  __shared__ double sm[2][256];
  double a1 = 0.0, a2 = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x) {
    x[i] = alpha * p[i] + 1.0 * x[i];
    const double ri = -alpha * q[i] + 1.0 * r[i];
    r[i] = ri;
    const double zi = d[i % dn] * ri;
    z[i] = zi;
    a1 += ri * ri;
    a2 += ri * zi;
  }
  sm[0][threadIdx.x] = a1;
  sm[1][threadIdx.x] = a2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sm[0][threadIdx.x] += sm[0][threadIdx.x + w];
      sm[1][threadIdx.x] += sm[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sm[0][0];
    part[gridDim.x + blockIdx.x] = sm[1][0];
  }
}

void launch_logn_cg_update(long len, double alpha, const double* p, const double* q, double* x, double* r,
                           const double* d, long dn, double* z, double* part, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(logn_cg_update_kernel, dim3(nblocks), dim3(256), 0, s, len, alpha, p, q, x, r, d,
                     dn > 0 ? dn : len, z, part);
}

void launch_logn_apply(const int* rptr, const int* rcol, const int* rslot, const double* C, const double* X,
                       int n_e, long n, int row0, int nrows, int col0, int col1, int mode, const double* R, double* Y,
                       hipStream_t s) {
  if (n <= 0 || nrows <= 0) return;
  hipLaunchKernelGGL(logn_apply_kernel, dim3((unsigned)((n + 255) / 256), nrows), dim3(256), 0, s, rptr, rcol, rslot,
                     C, X, n_e, n, row0, col0, col1, mode, R, Y);
}

void launch_logn_invdiag(const int* rptr, const int* rcol, const int* rslot, const double* C, int n_e, long n, int P,
                         double* Dinv, hipStream_t s) {
  if (n <= 0 || P <= 0) return;
  hipLaunchKernelGGL(logn_invdiag_kernel, dim3((unsigned)((n + 255) / 256), P), dim3(256), 0, s, rptr, rcol, rslot, C,
                     n_e, n, Dinv);
}

void launch_logn_dot(const double* x, const double* y, long len, double* part, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(logn_dot_kernel, dim3(nblocks), dim3(256), 0, s, x, y, len, part);
}

void launch_logn_axpby(long len, double a, const double* x, double b, double* y, int mode, const double* d,
                       long dn, hipStream_t s) {
  if (len <= 0) return;
  const long nb = std::min<long>((len + 255) / 256, 4096);
  hipLaunchKernelGGL(logn_axpby_kernel, dim3((unsigned)nb), dim3(256), 0, s, len, a, x, b, y, mode, d,
                     dn > 0 ? dn : len);
}

void launch_logn_mean_apply(const double* c, const double* X, int n_e, long n, int ncols, double* Y, hipStream_t s) {
  if (n <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(logn_mean_apply_kernel, dim3((unsigned)((n + 255) / 256), ncols), dim3(256), 0, s, c, X, n_e, n,
                     Y);
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
