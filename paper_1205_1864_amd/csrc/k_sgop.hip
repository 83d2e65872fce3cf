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

// ---------------------------------------------------------------------------
// Register-strip kernel. A block spans the whole grid width: thread ex owns
// element column ex (and node column ex, the left corner of that element) for
// a band of R element rows. Per output chaos row a and KL term k it forms the
// nodal combination w_k = sqrt(a_k) u_{a-e_k} + sqrt(a_k+1) u_{a+e_k} of the
// Galerkin neighbours, adds a_k(e) w_k to the element-corner values V(e), and
// finally applies the Q1 element matrix once per element:
//   (K^e V)_c = (5 V_c - sum V - V_opposite(c)) / 6.
// The right-corner values of an element come from lane + 1 by a DPP wave shift
// (lane 63 loads them itself); the contribution of element ex - 1 to node ex
// comes from lane - 1 by a DPP wave shift, across waves through LDS.
// ---------------------------------------------------------------------------

#ifndef SG_STRIP_R
#define SG_STRIP_R 4
#endif
constexpr int kStripR = SG_STRIP_R;

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

// Node values of column gx for node rows gy0 .. gy0 + R + 1 (grid coordinates; zero outside).
template <typename T, int R>
__device__ __forceinline__ void load_strip(const T* __restrict__ col, int gx, int gy0, int nx, T (&u)[R + 2]) {
  const bool xin = gx >= 1 && gx <= nx;
#pragma unroll
  for (int i = 0; i < R + 2; ++i) {
    const int gy = gy0 + i;
    u[i] = (xin && gy >= 1 && gy <= nx) ? col[(long)(gy - 1) * nx + (gx - 1)] : T(0);
  }
}

template <typename T, int R>
__device__ __forceinline__ void combo_strip(const T* in, long n, int blo, T glo, int bup, T gup, int gx, int gy0,
                                            int nx, T (&w)[R + 2]) {
  T u[R + 2];
#pragma unroll
  for (int i = 0; i < R + 2; ++i) w[i] = T(0);
  if (blo >= 0) {
    load_strip<T, R>(in + (long)blo * n, gx, gy0, nx, u);
#pragma unroll
    for (int i = 0; i < R + 2; ++i) w[i] = glo * u[i];
  }
  if (bup >= 0) {
    load_strip<T, R>(in + (long)bup * n, gx, gy0, nx, u);
#pragma unroll
    for (int i = 0; i < R + 2; ++i) w[i] += gup * u[i];
  }
}

template <typename T, int MT, int R>
__global__ void __launch_bounds__(512) sgop_strip_kernel(const SgOpArgs<T> A, const StripTables<T> tab, int nbands,
                                                          int nchunks, int chunk_rows) {
  __shared__ T xch[2][8][R];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ex = threadIdx.x;
  const int ne = A.n_e, nx = A.nx;
  // XCD-aware mapping: consecutive logical blocks (same band, different row
  // chunks) land on the same XCD so their shared input columns hit its L2.
  const int nblocks = nbands * nchunks;
  const int per_xcd = (nblocks + 7) / 8;
  const int logical = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (logical >= nblocks) return;
  const int band = logical / nchunks, chunk = logical % nchunks;
  const int ey0 = band * R;  // first element row; node rows ey0 .. ey0 + R + 1
  const int r0 = A.row0 + chunk * chunk_rows;
  const int r1 = min(A.row0 + A.nrows, r0 + chunk_rows);
  if (r0 >= r1) return;

  T a[MT > 0 ? MT : 1][R + 1];
#pragma unroll
  for (int k = 0; k < MT; ++k)
#pragma unroll
    for (int j = 0; j < R + 1; ++j) {
      const int ey = ey0 + j;
      a[k][j] = ey < ne ? A.a[(long)k * ne * ne + (long)ey * ne + ex] : T(0);
    }
  const long n = A.n;
  const bool has_right = ex + 1 <= nx;  // node column ex + 1 is interior

  for (int row = r0; row < r1; ++row) {
    T V[R + 1][4];
#pragma unroll
    for (int j = 0; j < R + 1; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) V[j][c] = T(0);

    if (A.diag != T(0)) {
      T w[R + 2];
      load_strip<T, R>(A.in + (long)row * n, ex, ey0, nx, w);
      T wr[R + 2];
#pragma unroll
      for (int i = 0; i < R + 2; ++i) wr[i] = from_next(w[i]);
      if (lane == 63 && has_right) load_strip<T, R>(A.in + (long)row * n, ex + 1, ey0, nx, wr);
#pragma unroll
      for (int j = 0; j < R + 1; ++j) {
        V[j][0] += A.diag * w[j];
        V[j][1] += A.diag * wr[j];
        V[j][2] += A.diag * wr[j + 1];
        V[j][3] += A.diag * w[j + 1];
      }
    }
#pragma unroll
    for (int k = 0; k < MT; ++k) {
      const int blo = A.use_lower ? tab.lo[row * MT + k] : -1;
      const int bup = A.use_upper ? tab.up[row * MT + k] : -1;
      if (blo < 0 && bup < 0) continue;
      const T glo = blo >= 0 ? tab.glo[row * MT + k] : T(0);
      const T gup = bup >= 0 ? tab.gup[row * MT + k] : T(0);
      T w[R + 2];
      combo_strip<T, R>(A.in, n, blo, glo, bup, gup, ex, ey0, nx, w);
      T wr[R + 2];
#pragma unroll
      for (int i = 0; i < R + 2; ++i) wr[i] = from_next(w[i]);
      if (lane == 63 && has_right) combo_strip<T, R>(A.in, n, blo, glo, bup, gup, ex + 1, ey0, nx, wr);
#pragma unroll
      for (int j = 0; j < R + 1; ++j) {
        V[j][0] += a[k][j] * w[j];
        V[j][1] += a[k][j] * wr[j];
        V[j][2] += a[k][j] * wr[j + 1];
        V[j][3] += a[k][j] * w[j + 1];
      }
    }
    // element matrix: o_c = (5 V_c - S - V_opp(c)) / 6, corners 0 BL, 1 BR, 2 TR, 3 TL
    T own[R], right[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      // node row ey0 + 1 + i: top of element i, bottom of element i + 1
      const T S0 = V[i][0] + V[i][1] + V[i][2] + V[i][3];
      const T S1 = V[i + 1][0] + V[i + 1][1] + V[i + 1][2] + V[i + 1][3];
      const T oTL = T(5) * V[i][3] - S0 - V[i][1];
      const T oTR = T(5) * V[i][2] - S0 - V[i][0];
      const T oBL = T(5) * V[i + 1][0] - S1 - V[i + 1][2];
      const T oBR = T(5) * V[i + 1][1] - S1 - V[i + 1][3];
      own[i] = oTL + oBL;
      right[i] = oTR + oBR;
    }
    const int par = row & 1;
    if (lane == 63) {
#pragma unroll
      for (int i = 0; i < R; ++i) xch[par][wave][i] = right[i];
    }
    __syncthreads();
    T left[R];
#pragma unroll
    for (int i = 0; i < R; ++i) left[i] = from_prev(right[i]);
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < R; ++i) left[i] = wave > 0 ? xch[par][wave - 1][i] : T(0);
    }
    if (ex >= 1 && ex <= nx) {
      T* o = A.out + (long)row * n;
      const T* rs = A.rsrc ? A.rsrc + (long)row * n : nullptr;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int gy = ey0 + 1 + i;
        if (gy <= nx) {
          const long idx = (long)(gy - 1) * nx + (ex - 1);
          T v = A.sgn * ((own[i] + left[i]) * T(1.0 / 6.0));
          if (rs) v += A.rcoef * rs[idx];
          o[idx] = v;
        }
      }
    }
  }
}

// Occupancy variant of the strip kernel: the KL coefficients are read per
// entry (they stay in L1/L2, shared by every row of the band) instead of being
// held in registers, and each row walks a compact list of its active KL terms
// without branches, so more waves hide the load latency.
template <typename T, int R>
__global__ void __launch_bounds__(512) sgop_strip_dyn_kernel(const SgOpArgs<T> A, const StripTables<T> tab,
                                                              int nbands, int nchunks, int chunk_rows) {
  __shared__ T xch[2][8][R];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ex = threadIdx.x;
  const int ne = A.n_e, nx = A.nx;
  const int nblocks = nbands * nchunks;
  const int per_xcd = (nblocks + 7) / 8;
  const int logical = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (logical >= nblocks) return;
  const int band = logical / nchunks, chunk = logical % nchunks;
  const int ey0 = band * R;
  const int r0 = A.row0 + chunk * chunk_rows;
  const int r1 = min(A.row0 + A.nrows, r0 + chunk_rows);
  if (r0 >= r1) return;
  const long n = A.n;
  const long ne2 = (long)ne * ne;
  const bool has_right = ex + 1 <= nx;

  for (int row = r0; row < r1; ++row) {
    T V[R + 1][4];
#pragma unroll
    for (int j = 0; j < R + 1; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) V[j][c] = T(0);
    if (A.diag != T(0)) {
      T w[R + 2];
      load_strip<T, R>(A.in + (long)row * n, ex, ey0, nx, w);
      T wr[R + 2];
#pragma unroll
      for (int i = 0; i < R + 2; ++i) wr[i] = from_next(w[i]);
      if (lane == 63 && has_right) load_strip<T, R>(A.in + (long)row * n, ex + 1, ey0, nx, wr);
#pragma unroll
      for (int j = 0; j < R + 1; ++j) {
        V[j][0] += A.diag * w[j];
        V[j][1] += A.diag * wr[j];
        V[j][2] += A.diag * wr[j + 1];
        V[j][3] += A.diag * w[j + 1];
      }
    }
    const int e0 = tab.ent_ptr[row], e1 = tab.ent_ptr[row + 1];
#pragma unroll 2
    for (int e = e0; e < e1; ++e) {
      const int k = tab.ent_k[e];
      const int blo = tab.ent_lo[e], bup = tab.ent_up[e];
      const T glo = A.use_lower ? tab.ent_glo[e] : T(0);
      const T gup = A.use_upper ? tab.ent_gup[e] : T(0);
      if (glo == T(0) && gup == T(0)) continue;
      T a[R + 1];
#pragma unroll
      for (int j = 0; j < R + 1; ++j) {
        const int ey = ey0 + j;
        a[j] = ey < ne ? A.a[(long)k * ne2 + (long)ey * ne + ex] : T(0);
      }
      T ul[R + 2], uu[R + 2], w[R + 2];
      load_strip<T, R>(A.in + (long)blo * n, ex, ey0, nx, ul);
      load_strip<T, R>(A.in + (long)bup * n, ex, ey0, nx, uu);
#pragma unroll
      for (int i = 0; i < R + 2; ++i) w[i] = glo * ul[i] + gup * uu[i];
      T wr[R + 2];
#pragma unroll
      for (int i = 0; i < R + 2; ++i) wr[i] = from_next(w[i]);
      if (lane == 63 && has_right) {
        load_strip<T, R>(A.in + (long)blo * n, ex + 1, ey0, nx, ul);
        load_strip<T, R>(A.in + (long)bup * n, ex + 1, ey0, nx, uu);
#pragma unroll
        for (int i = 0; i < R + 2; ++i) wr[i] = glo * ul[i] + gup * uu[i];
      }
#pragma unroll
      for (int j = 0; j < R + 1; ++j) {
        V[j][0] += a[j] * w[j];
        V[j][1] += a[j] * wr[j];
        V[j][2] += a[j] * wr[j + 1];
        V[j][3] += a[j] * w[j + 1];
      }
    }
    T own[R], right[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const T S0 = V[i][0] + V[i][1] + V[i][2] + V[i][3];
      const T S1 = V[i + 1][0] + V[i + 1][1] + V[i + 1][2] + V[i + 1][3];
      const T oTL = T(5) * V[i][3] - S0 - V[i][1];
      const T oTR = T(5) * V[i][2] - S0 - V[i][0];
      const T oBL = T(5) * V[i + 1][0] - S1 - V[i + 1][2];
      const T oBR = T(5) * V[i + 1][1] - S1 - V[i + 1][3];
      own[i] = oTL + oBL;
      right[i] = oTR + oBR;
    }
    const int par = row & 1;
    if (lane == 63) {
#pragma unroll
      for (int i = 0; i < R; ++i) xch[par][wave][i] = right[i];
    }
    __syncthreads();
    T left[R];
#pragma unroll
    for (int i = 0; i < R; ++i) left[i] = from_prev(right[i]);
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < R; ++i) left[i] = wave > 0 ? xch[par][wave - 1][i] : T(0);
    }
    if (ex >= 1 && ex <= nx) {
      T* o = A.out + (long)row * n;
      const T* rs = A.rsrc ? A.rsrc + (long)row * n : nullptr;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int gy = ey0 + 1 + i;
        if (gy <= nx) {
          const long idx = (long)(gy - 1) * nx + (ex - 1);
          T v = A.sgn * ((own[i] + left[i]) * T(1.0 / 6.0));
          if (rs) v += A.rcoef * rs[idx];
          o[idx] = v;
        }
      }
    }
  }
}

template <typename T>
void launch_strip_dyn(const SgOpArgs<T>& A, const StripTables<T>& tab, hipStream_t s) {
  constexpr int R = kStripR;
  const int nbands = (A.n_e + R - 1) / R;
  int nchunks = tab.blocks_per_band > 0 ? tab.blocks_per_band : 64;
  if (nchunks > A.nrows) nchunks = A.nrows;
  if (nchunks < 1) nchunks = 1;
  const int chunk_rows = (A.nrows + nchunks - 1) / nchunks;
  nchunks = (A.nrows + chunk_rows - 1) / chunk_rows;
  const int nblocks = nbands * nchunks;
  const int grid = (nblocks + 7) / 8 * 8;
  hipLaunchKernelGGL((sgop_strip_dyn_kernel<T, R>), dim3(grid), dim3(A.n_e), 0, s, A, tab, nbands, nchunks,
                     chunk_rows);
}

template <typename T, int MT>
void launch_strip(const SgOpArgs<T>& A, const StripTables<T>& tab, hipStream_t s) {
  constexpr int R = kStripR;
  const int nbands = (A.n_e + R - 1) / R;
  // Row chunks per band: enough blocks per band to fill one XCD (32 CUs, two
  // blocks each), so each XCD works through one band at a time and the band's
  // input columns stay in its L2.
  int nchunks = tab.blocks_per_band > 0 ? tab.blocks_per_band : 64;
  if (nchunks > A.nrows) nchunks = A.nrows;
  if (nchunks < 1) nchunks = 1;
  const int chunk_rows = (A.nrows + nchunks - 1) / nchunks;
  nchunks = (A.nrows + chunk_rows - 1) / chunk_rows;
  const int nblocks = nbands * nchunks;
  const int grid = (nblocks + 7) / 8 * 8;
  hipLaunchKernelGGL((sgop_strip_kernel<T, MT, R>), dim3(grid), dim3(A.n_e), 0, s, A, tab, nbands, nchunks,
                     chunk_rows);
}

template <typename T, int MT>
bool dispatch_strip(const SgOpArgs<T>& A, const StripTables<T>& tab, hipStream_t s) {
  if (tab.M == MT) {
    launch_strip<T, MT>(A, tab, s);
    return true;
  }
  if constexpr (MT > 0) return dispatch_strip<T, MT - 1>(A, tab, s);
  return false;
}

}  // namespace

constexpr int kStripMaxM = 12;

template <typename T>
void launch_sgop(const SgOpArgs<T>& args, const StripTables<T>& tab, hipStream_t s) {
  if (args.nrows <= 0) return;
  const bool shape_ok = args.n_e % 64 == 0 && args.n_e >= 64 && args.n_e <= 512;
  if (shape_ok && tab.variant == 1 && tab.ent_ptr != nullptr) {
    launch_strip_dyn<T>(args, tab, s);
    return;
  }
  const bool strip_ok = shape_ok && tab.M <= kStripMaxM && tab.lo != nullptr;
  if (strip_ok && dispatch_strip<T, kStripMaxM>(args, tab, s)) return;
  const int tiles = (args.nx + kTile - 1) / kTile;
  dim3 grid(tiles * tiles, args.nrows);
  hipLaunchKernelGGL(sgop_kernel<T>, grid, dim3(256), 0, s, args);
}

template void launch_sgop<double>(const SgOpArgs<double>&, const StripTables<double>&, hipStream_t);
template void launch_sgop<float>(const SgOpArgs<float>&, const StripTables<float>&, hipStream_t);

}  // namespace sgk
