// SG block operator: the MAT-VEC of the stochastic Galerkin matrix (Remark
// after eq. (global-matrix-block)) and the coupling products B_l, C_l of
// Algorithm 1, applied without forming any matrix.
//
// For chaos row a the kernel evaluates
//   out[a] = rcoef * rsrc[a] + diag * K_Lap in[a]
//            + sgn * sum_{(k, b, g) in lists(a)} g * K_k in[b]
// where K_k = sum_e a_k(e) K^e is the Q1 stiffness of the piecewise-constant
// coefficient a_k. At node i the element form is
//   (K_k u)_i = 1/6 sum_{e ni i} a_k(e) (4 u_i - u_adj1 - u_adj2 - 2 u_opp)
// over the four elements sharing i (the Q1 element matrix of a square).
#include "sg_internal.h"

namespace sgk {

namespace {

constexpr int kTile = 16;  // 16 x 16 nodes per block

template <typename T>
__device__ __forceinline__ T load_node(const T* __restrict__ col, int gx, int gy, int nx) {
  // gx, gy are grid coordinates 0..nx+1; the boundary carries no unknowns.
  return (gx >= 1 && gx <= nx && gy >= 1 && gy <= nx) ? col[(long)(gy - 1) * nx + (gx - 1)] : T(0);
}

template <typename T>
__global__ void __launch_bounds__(256) sgop_kernel(const SgOpArgs<T> A) {
  const int tiles_x = (A.nx + kTile - 1) / kTile;
  const int tx = blockIdx.x % tiles_x;
  const int ty = blockIdx.x / tiles_x;
  const int gx = tx * kTile + (threadIdx.x % kTile) + 1;
  const int gy = ty * kTile + (threadIdx.x / kTile) + 1;
  const int row = A.row0 + blockIdx.y;
  if (gx > A.nx || gy > A.nx) return;
  const long node = (long)(gy - 1) * A.nx + (gx - 1);
  const int ne = A.n_e;
  // elements around the node: SW (gx-1, gy-1), SE (gx, gy-1), NW (gx-1, gy), NE (gx, gy)
  const long eSW = (long)(gy - 1) * ne + (gx - 1);
  const long eSE = eSW + 1;
  const long eNW = eSW + ne;
  const long eNE = eNW + 1;

  T acc = T(0);
  if (A.diag != T(0)) {
    const T* col = A.in + (long)row * A.n;
    T c = load_node(col, gx, gy, A.nx);
    T s = load_node(col, gx - 1, gy - 1, A.nx) + load_node(col, gx, gy - 1, A.nx) +
          load_node(col, gx + 1, gy - 1, A.nx) + load_node(col, gx - 1, gy, A.nx) +
          load_node(col, gx + 1, gy, A.nx) + load_node(col, gx - 1, gy + 1, A.nx) +
          load_node(col, gx, gy + 1, A.nx) + load_node(col, gx + 1, gy + 1, A.nx);
    acc = A.diag * (T(8) / T(3) * c - s / T(3));
  }
  T sum = T(0);
  for (int pass = 0; pass < 2; ++pass) {
    const int use = pass == 0 ? A.use_lower : A.use_upper;
    if (!use) continue;
    const int* ptr = pass == 0 ? A.lists.lo_ptr : A.lists.up_ptr;
    const int* ent = pass == 0 ? A.lists.lo_ent : A.lists.up_ent;
    const T* gv = pass == 0 ? A.lists.lo_g : A.lists.up_g;
    for (int e = ptr[row]; e < ptr[row + 1]; ++e) {
      const int pk = ent[e];
      const int b = pk & 0xFFFFF;
      const int k = pk >> 20;
      const T g = gv[e];
      const T* col = A.in + (long)b * A.n;
      const T* ak = A.a + (long)(k - 1) * ne * ne;
      const T aSW = ak[eSW], aSE = ak[eSE], aNW = ak[eNW], aNE = ak[eNE];
      const T uC = load_node(col, gx, gy, A.nx);
      const T uW = load_node(col, gx - 1, gy, A.nx);
      const T uE = load_node(col, gx + 1, gy, A.nx);
      const T uS = load_node(col, gx, gy - 1, A.nx);
      const T uN = load_node(col, gx, gy + 1, A.nx);
      const T uSW = load_node(col, gx - 1, gy - 1, A.nx);
      const T uSE = load_node(col, gx + 1, gy - 1, A.nx);
      const T uNW = load_node(col, gx - 1, gy + 1, A.nx);
      const T uNE = load_node(col, gx + 1, gy + 1, A.nx);
      T v = aSW * (T(4) * uC - uW - uS - T(2) * uSW) + aSE * (T(4) * uC - uE - uS - T(2) * uSE) +
            aNW * (T(4) * uC - uW - uN - T(2) * uNW) + aNE * (T(4) * uC - uE - uN - T(2) * uNE);
      sum += g * v;
    }
  }
  acc += A.sgn * (sum / T(6));
  T* o = A.out + (long)row * A.n + node;
  if (A.rsrc) acc += A.rcoef * A.rsrc[(long)row * A.n + node];
  *o = acc;
}

}  // namespace

template <typename T>
void launch_sgop(const SgOpArgs<T>& args, hipStream_t s) {
  if (args.nrows <= 0) return;
  const int tiles = (args.nx + kTile - 1) / kTile;
  dim3 grid(tiles * tiles, args.nrows);
  hipLaunchKernelGGL(sgop_kernel<T>, grid, dim3(256), 0, s, args);
}

template void launch_sgop<double>(const SgOpArgs<double>&, hipStream_t);
template void launch_sgop<float>(const SgOpArgs<float>&, hipStream_t);

}  // namespace sgk
