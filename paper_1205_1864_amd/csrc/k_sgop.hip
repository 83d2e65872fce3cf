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
#include "sg_device.h"

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
  if (A.active && ld_uniform(A.active, 0) == 0) return;
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
  if (A.active && ld_uniform(A.active, 0) == 0) return;
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
  if (A.active && ld_uniform(A.active, 0) == 0) return;
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

// ---------------------------------------------------------------------------
// y-marching kernel. A block spans the grid width (thread ex owns element
// column ex and node column ex) and walks one segment of node rows upwards for
// a small group of output chaos rows, so every node row of an input column is
// read once per use within the segment. The segments of one XCD are handled by
// all row groups at once, so the columns that several rows share are served
// from that XCD's L2.
//
// At node row gy the block loads, for each output row a of the group, the
// node values of a and of its Galerkin neighbours and forms per node x
//   T  = sum_k a_k(e[x],   gy-1) w_k(x)   top-left corner of element x (row gy-1)
//   Rt = sum_k a_k(e[x-1], gy-1) w_k(x)   top-right corner of element x-1
//   B  = sum_k a_k(e[x],   gy)   w_k(x)   bottom-left corner of element x (row gy)
//   Rb = sum_k a_k(e[x-1], gy)   w_k(x)   bottom-right corner of element x-1
// with w_0 = diag * u_a and w_k = g_lo u_{a-e_k} + g_up u_{a+e_k}. Element x
// of row gy-1 then has all four corner values (B and Rb from the previous node
// row, Rt and Rb of node x+1 from lane x+1) and applies the Q1 element matrix
// o_c = (5 V_c - sum V - V_opp(c)) / 6. Node row gy-1 is complete after that
// and is written one step later, once the contribution across the wave
// boundary has arrived through LDS (one barrier per node row). All loads of a
// step are issued before the first of them is used.
// ---------------------------------------------------------------------------
constexpr int kMarchRGmax = kMarchRGU > kMarchRGL ? kMarchRGU : kMarchRGL;

template <typename T, int NK, int RG, bool LK>
__device__ __forceinline__ void march_body(const SgOpArgs<T>& A, const StripTables<T>& tab, const MarchJob& job,
                                           int g, int ys, int ye, T (*xs)[8][kMarchRGmax][2],
                                           T (*xo)[8][kMarchRGmax][2]) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwaves = blockDim.x >> 6;
  const int ex = threadIdx.x;
  const int ne = A.n_e, nx = A.nx, M = tab.M;
  const long n = A.n;
  const long ne2 = (long)ne * ne;
  const int gbeg = ld_uniform(job.gptr, g);
  const int cnt = ld_uniform(job.gptr, g + 1) - gbeg;
  int rows[RG];
#pragma unroll
  for (int j = 0; j < RG; ++j) rows[j] = j < cnt ? ld_uniform(job.grows, gbeg + j) : -1;
  int ks[NK];
#pragma unroll
  for (int s = 0; s < NK; ++s) ks[s] = LK ? ld_uniform(job.lk, g * kMarchNS + s) : s;
  const bool xin = ex >= 1 && ex <= nx;
  const bool has_left = ex >= 1;
  const int xl = wave * 64 - 1;  // element to the left of lane 0 (-1 for the first wave)
  const bool last_wave = wave + 1 == nwaves;
  const T scale = A.sgn / T(6);
  const T* __restrict__ in = A.in;
  const T* __restrict__ acoef = A.a;

  // Neighbour columns and weights of the group's rows (uniform, read once);
  // a missing neighbour has column -1 and weight 0 and is not loaded (a
  // uniform branch on a scalar register).
  int cl[RG][NK], cu[RG][NK];
  T wl[RG][NK], wu[RG][NK];
#pragma unroll
  for (int j = 0; j < RG; ++j) {
    const int row = rows[j];
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      int lo = -1, up = -1;
      T gl = T(0), gu = T(0);
      if (row >= 0) {
        if constexpr (LK) {
          lo = ld_uniform(job.lcol, (g * kMarchRGL + j) * kMarchNS + s);
          if (lo >= 0) gl = T(ld_uniform(job.lw, (g * kMarchRGL + j) * kMarchNS + s));
        } else {
          if (A.use_lower) {
            lo = ld_uniform(tab.lo, row * M + s);
            if (lo >= 0) gl = ld_uniform(tab.glo, row * M + s);
          }
          if (A.use_upper) {
            up = ld_uniform(tab.up, row * M + s);
            if (up >= 0) gu = ld_uniform(tab.gup, row * M + s);
          }
        }
      }
      cl[j][s] = lo;
      cu[j][s] = up;
      wl[j][s] = gl;
      wu[j][s] = gu;
    }
  }
  const bool has_diag = A.diag != T(0);

  T ac[NK], acp[NK], an[NK], anp[NK];
#pragma unroll
  for (int s = 0; s < NK; ++s) ac[s] = acp[s] = T(0);
  T dc = T(0), dcp = T(0);
  T pend[RG], carry[RG], Bp[RG], Rbp[RG];
#pragma unroll
  for (int j = 0; j < RG; ++j) pend[j] = carry[j] = Bp[j] = Rbp[j] = T(0);

  for (int gy = ys - 1; gy <= ye; ++gy) {
    const int par = gy & 1;
    const bool ev = gy <= ne - 1;  // element row gy (above node row gy) exists
    const long abase = (long)gy * ne + ex;
    const bool nin = xin && gy >= 1 && gy <= nx;
    const long nidx = (long)(gy - 1) * nx + (ex - 1);
    // ---- loads of the step: coefficients of element row gy, then the node values
    T al0[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      const bool use = ev && ks[s] >= 0;
      an[s] = use ? acoef[(long)ks[s] * ne2 + abase] : T(0);
      al0[s] = (use && xl >= 0) ? ld_uniform(acoef, (long)ks[s] * ne2 + (long)gy * ne + xl) : T(0);
    }
    // off-grid lanes read node 0 and discard it
    const long nid = nin ? nidx : 0;
    T ud[RG], ul[RG][NK], uu[RG][NK];
#pragma unroll
    for (int j = 0; j < RG; ++j) {
      const int row = rows[j];
      ud[j] = T(0);
      if (has_diag && row >= 0) ud[j] = in[(long)row * n + nid];
#pragma unroll
      for (int s = 0; s < NK; ++s) {
        ul[j][s] = T(0);
        uu[j][s] = T(0);
        if (row >= 0) {
          if (cl[j][s] >= 0) ul[j][s] = in[(long)cl[j][s] * n + nid];
          if (!LK && cu[j][s] >= 0) uu[j][s] = in[(long)cu[j][s] * n + nid];
        }
      }
    }
    if (!nin) {
#pragma unroll
      for (int j = 0; j < RG; ++j) {
        ud[j] = T(0);
#pragma unroll
        for (int s = 0; s < NK; ++s) ul[j][s] = uu[j][s] = T(0);
      }
    }
    // ---- corner sums
    const T dn = ev ? A.diag : T(0);
    const T dnp = has_left ? dn : T(0);
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      T v = from_prev(an[s]);
      if (lane == 0) v = al0[s];
      anp[s] = v;
    }
    T sT[RG], sB[RG], Rtn[RG], Rbn[RG];
#pragma unroll
    for (int j = 0; j < RG; ++j) {
      sT[j] = sB[j] = Rtn[j] = Rbn[j] = T(0);
      const int row = rows[j];
      if (row < 0) continue;
      T t = dc * ud[j], rt = dcp * ud[j], b = dn * ud[j], rb = dnp * ud[j];
#pragma unroll
      for (int s = 0; s < NK; ++s) {
        T w;
        if constexpr (LK) {
          w = wl[j][s] * ul[j][s];
        } else {
          w = wl[j][s] * ul[j][s] + wu[j][s] * uu[j][s];
        }
        t += ac[s] * w;
        rt += acp[s] * w;
        b += an[s] * w;
        rb += anp[s] * w;
      }
      sT[j] = t;
      sB[j] = b;
      Rtn[j] = from_next(rt);
      Rbn[j] = from_next(rb);
      if (lane == 0) {
        xs[par][wave][j][0] = rt;
        xs[par][wave][j][1] = rb;
      }
    }
    __syncthreads();
    const int orow = gy - 2;  // node row completed one step ago
    const bool wr = xin && orow >= ys && orow < ye;
#pragma unroll
    for (int j = 0; j < RG; ++j) {
      const int row = rows[j];
      if (row < 0) continue;
      if (lane == 63 && !last_wave) {
        Rtn[j] = xs[par][wave + 1][j][0];
        Rbn[j] = xs[par][wave + 1][j][1];
      }
      if (lane == 0 && wave > 0 && gy >= ys) {
        pend[j] += xo[par ^ 1][wave - 1][j][0];
        carry[j] += xo[par ^ 1][wave - 1][j][1];
      }
      if (wr) {
        const long idx = (long)row * n + (long)(orow - 1) * nx + (ex - 1);
        T v = scale * pend[j];
        if (A.rsrc) v += A.rcoef * A.rsrc[idx];
        A.out[idx] = v;
      }
      // element x of element row gy-1: corners BL, BR (node row gy-1), TR, TL (node row gy)
      const T BL = Bp[j], BR = Rbp[j], TR = Rtn[j], TL = sT[j];
      const T S = (BL + BR) + (TR + TL);
      const T oBL = T(5) * BL - S - TR;
      const T oBR = T(5) * BR - S - TL;
      const T oTR = T(5) * TR - S - BL;
      const T oTL = T(5) * TL - S - BR;
      pend[j] = oBL + carry[j] + from_prev(oBR);
      carry[j] = oTL + from_prev(oTR);
      if (lane == 63) {
        xo[par][wave][j][0] = oBR;
        xo[par][wave][j][1] = oTR;
      }
      Bp[j] = sB[j];
      Rbp[j] = Rbn[j];
    }
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      ac[s] = an[s];
      acp[s] = anp[s];
    }
    dc = dn;
    dcp = dnp;
  }
  // node row ye-1 waits for the wave-boundary term of the last step
  __syncthreads();
  const int orow = ye - 1;
  const int lp = ye & 1;
  if (xin && orow >= ys) {
#pragma unroll
    for (int j = 0; j < RG; ++j) {
      const int row = rows[j];
      if (row < 0) continue;
      T pv = pend[j];
      if (lane == 0 && wave > 0) pv += xo[lp][wave - 1][j][0];
      const long idx = (long)row * n + (long)(orow - 1) * nx + (ex - 1);
      T v = scale * pv;
      if (A.rsrc) v += A.rcoef * A.rsrc[idx];
      A.out[idx] = v;
    }
  }
}

template <typename T, int MT>
__global__ void __launch_bounds__(512) sgop_march_kernel(const SgOpArgs<T> A, const StripTables<T> tab,
                                                          const MarchJob job) {
  __shared__ T xs[2][8][kMarchRGmax][2];  // lane 0 of each wave: (Rt, Rb) for lane 63 of the wave before
  __shared__ T xo[2][8][kMarchRGmax][2];  // lane 63 of each wave: (o_BR, o_TR) for lane 0 of the wave after
  if (A.active && ld_uniform(A.active, 0) == 0) return;
  const int nblocks = job.ngroups * job.nseg;
  const int per_xcd = (nblocks + 7) / 8;
  const int logical = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (logical >= nblocks) return;
  const int seg = logical / job.ngroups, g = logical % job.ngroups;
  const int ys = 1 + seg * job.seg_rows;
  const int ye = min(A.nx + 1, ys + job.seg_rows);  // output node rows ys .. ye-1
  if (ys >= ye) return;
  if (ld_uniform(job.gkind, g) == 0) {
    if constexpr (MT > 0) march_body<T, MT, kMarchRGU, false>(A, tab, job, g, ys, ye, xs, xo);
  } else {
    march_body<T, kMarchNS, kMarchRGL, true>(A, tab, job, g, ys, ye, xs, xo);
  }
}

// ---------------------------------------------------------------------------
// Piece kernel. The node grid is cut into pieces of one wavefront of node
// columns by TY node rows: lane 0 and lane W + 1 hold the halo columns of a
// piece, lanes 1..W its W output columns. A block is one wave and marches one
// piece upwards for one row group (the groups of the y-marching kernel), with
// the same corner sums and element matrix as march_body, but without any
// barrier: horizontal neighbours come from DPP lane shifts inside the wave,
// and the halo lanes absorb what the shifts bring in at the ends. Blocks are
// pinned to XCDs (hardware block b runs on XCD b mod 8); XCD x works through a
// contiguous band of pieces, every row group of a piece before the next
// piece, so the input columns of a piece come from HBM about once and are
// then served to the other row groups from that XCD's L2.
//
// Values outside the grid are zero (Dirichlet nodes, and loads of off-grid
// lanes are replaced by zero), so elements that do not exist contribute
// nothing to an output node; their coefficient loads are clamped into the
// array (finite values multiplied by zero).
// ---------------------------------------------------------------------------
template <typename T, int NK, int RG, bool LK>
__device__ __forceinline__ void piece_body(const SgOpArgs<T>& A, const StripTables<T>& tab, const MarchJob& job,
                                           int g, int x0, int ys, int ye, int W) {
  const int lane = threadIdx.x & 63;
  const int ne = A.n_e, nx = A.nx, M = tab.M;
  const long n = A.n;
  const long ne2 = (long)ne * ne;
  const int x = x0 + lane;                          // node column of the lane; its element spans x .. x + 1
  const bool xin = x >= 1 && x <= nx;               // interior node column
  const bool xout = xin && lane >= 1 && lane <= W;  // output column of this piece
  const int xe = x <= ne - 1 ? x : ne - 1;          // element column clamped into the array
  const T scale = A.sgn / T(6);
  const T* __restrict__ in = A.in;
  const T* __restrict__ acoef = A.a;
  const T diag = A.diag;
  const bool has_diag = diag != T(0);

  const int gbeg = ld_uniform(job.gptr, g);
  const int cnt = ld_uniform(job.gptr, g + 1) - gbeg;
  int rows[RG];
#pragma unroll
  for (int j = 0; j < RG; ++j) rows[j] = j < cnt ? ld_uniform(job.grows, gbeg + j) : -1;
  int ks[NK];
#pragma unroll
  for (int s = 0; s < NK; ++s) ks[s] = LK ? ld_uniform(job.lk, g * kMarchNS + s) : s;
  // neighbour columns and weights of the group's rows (uniform); a missing
  // neighbour has column -1 and is not loaded
  int cl[RG][NK], cu[RG][NK];
  T wl[RG][NK], wu[RG][NK];
#pragma unroll
  for (int j = 0; j < RG; ++j) {
    const int row = rows[j];
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      int lo = -1, up = -1;
      T gl = T(0), gu = T(0);
      if (row >= 0) {
        if constexpr (LK) {
          lo = ld_uniform(job.lcol, (g * kMarchRGL + j) * kMarchNS + s);
          if (lo >= 0) gl = T(ld_uniform(job.lw, (g * kMarchRGL + j) * kMarchNS + s));
        } else {
          if (A.use_lower) {
            lo = ld_uniform(tab.lo, row * M + s);
            if (lo >= 0) gl = ld_uniform(tab.glo, row * M + s);
          }
          if (A.use_upper) {
            up = ld_uniform(tab.up, row * M + s);
            if (up >= 0) gu = ld_uniform(tab.gup, row * M + s);
          }
        }
      }
      cl[j][s] = lo;
      cu[j][s] = up;
      wl[j][s] = gl;
      wu[j][s] = gu;
    }
  }

  T ac[NK], acp[NK];
#pragma unroll
  for (int s = 0; s < NK; ++s) ac[s] = acp[s] = T(0);
  T Bp[RG], BRp[RG], carry[RG];
#pragma unroll
  for (int j = 0; j < RG; ++j) Bp[j] = BRp[j] = carry[j] = T(0);

  for (int gy = ys - 1; gy <= ye; ++gy) {
    // ---- loads: coefficients of element row gy (clamped), node values of node row gy
    const int ey = gy < 0 ? 0 : (gy > ne - 1 ? ne - 1 : gy);
    const long abase = (long)ey * ne + xe;
    T an[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) an[s] = ks[s] >= 0 ? acoef[(long)ks[s] * ne2 + abase] : T(0);
    const bool nin = xin && gy >= 1 && gy <= nx;
    const long nid = nin ? (long)(gy - 1) * nx + (x - 1) : 0;
    T ud[RG], ul[RG][NK], uu[RG][NK];
#pragma unroll
    for (int j = 0; j < RG; ++j) {
      const int row = rows[j];
      ud[j] = T(0);
      if (has_diag && row >= 0) ud[j] = in[(long)row * n + nid];
#pragma unroll
      for (int s = 0; s < NK; ++s) {
        ul[j][s] = T(0);
        uu[j][s] = T(0);
        if (row >= 0) {
          if (cl[j][s] >= 0) ul[j][s] = in[(long)cl[j][s] * n + nid];
          if (!LK && cu[j][s] >= 0) uu[j][s] = in[(long)cu[j][s] * n + nid];
        }
      }
    }
    if (!nin) {
#pragma unroll
      for (int j = 0; j < RG; ++j) {
        ud[j] = T(0);
#pragma unroll
        for (int s = 0; s < NK; ++s) ul[j][s] = uu[j][s] = T(0);
      }
    }
    // an at the element to the left (lane 0 is a halo column: its value is unused)
    T anp[NK];
#pragma unroll
    for (int s = 0; s < NK; ++s) anp[s] = from_prev(an[s]);
    const int orow = gy - 1;  // node row completed at this step
    const bool wr = xout && orow >= ys && orow < ye;
#pragma unroll
    for (int j = 0; j < RG; ++j) {
      const int row = rows[j];
      if (row < 0) continue;
      // corner sums at node (x, gy): T / Rt with the element row below (ac, acp),
      // B / Rb with the element row above (an, anp); the diagonal term first
      T t = diag * ud[j];
      T rt = t, b = t, rb = t;
#pragma unroll
      for (int s = 0; s < NK; ++s) {
        T w;
        if constexpr (LK) {
          w = wl[j][s] * ul[j][s];
        } else {
          w = wl[j][s] * ul[j][s] + wu[j][s] * uu[j][s];
        }
        t += ac[s] * w;
        rt += acp[s] * w;
        b += an[s] * w;
        rb += anp[s] * w;
      }
      // element x of element row gy - 1: corners BL, BR (node row gy - 1), TR, TL (node row gy)
      const T BL = Bp[j], BR = BRp[j], TR = from_next(rt), TL = t;
      const T S = (BL + BR) + (TR + TL);
      const T oBL = T(5) * BL - S - TR;
      const T oBR = T(5) * BR - S - TL;
      const T oTR = T(5) * TR - S - BL;
      const T oTL = T(5) * TL - S - BR;
      const T pend = oBL + carry[j] + from_prev(oBR);  // node row gy - 1, complete
      if (wr) {
        const long idx = (long)row * n + (long)(orow - 1) * nx + (x - 1);
        T v = scale * pend;
        if (A.rsrc) v += A.rcoef * A.rsrc[idx];
        A.out[idx] = v;
      }
      carry[j] = oTL + from_prev(oTR);  // node row gy, from element row gy - 1
      Bp[j] = b;
      BRp[j] = from_next(rb);
    }
#pragma unroll
    for (int s = 0; s < NK; ++s) {
      ac[s] = an[s];
      acp[s] = anp[s];
    }
  }
}

template <typename T, int MT>
__global__ void __launch_bounds__(64) sgop_piece_kernel(const SgOpArgs<T> A, const StripTables<T> tab,
                                                         const MarchJob job, const PieceGeom pg) {
  if (A.active && ld_uniform(A.active, 0) == 0) return;
  const int xcd = blockIdx.x % 8;
  const int slot = blockIdx.x / 8;
  const int nslots = ((int)gridDim.x - xcd + 7) / 8;  // blocks on this XCD
  const long npieces = (long)pg.nyseg * pg.nstrips;
  const long p0 = npieces * xcd / 8, p1 = npieces * (xcd + 1) / 8;
  const long ntasks = (p1 - p0) * job.ngroups;
  for (long t = slot; t < ntasks; t += nslots) {
    const long p = p0 + t / job.ngroups;
    const int g = (int)(t % job.ngroups);
    const int yseg = (int)(p / pg.nstrips), strip = (int)(p % pg.nstrips);
    const int x0 = strip * pg.W;
    const int ys = 1 + yseg * pg.TY;
    const int ye = min(A.nx + 1, ys + pg.TY);
    if (ld_uniform(job.gkind, g) == 0) {
      if constexpr (MT > 0) piece_body<T, MT, kMarchRGU, false>(A, tab, job, g, x0, ys, ye, pg.W);
    } else {
      piece_body<T, kMarchNS, kMarchRGL, true>(A, tab, job, g, x0, ys, ye, pg.W);
    }
  }
}

template <typename T, int MT>
void launch_piece(const SgOpArgs<T>& A, const StripTables<T>& tab, const MarchJob& job, const PieceGeom& pg,
                  hipStream_t s) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sgop_piece_kernel<T, MT>, 64, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  int dev = 0, ncu = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const long ntasks = (long)pg.nyseg * pg.nstrips * job.ngroups;
  long grid = (long)per_cu * ncu;
  if (pg.max_waves_per_cu > 0 && pg.max_waves_per_cu < per_cu) grid = (long)pg.max_waves_per_cu * ncu;
  if (grid > ntasks + 7) grid = (ntasks + 7) / 8 * 8;
  grid = (grid + 7) / 8 * 8;
  hipLaunchKernelGGL((sgop_piece_kernel<T, MT>), dim3((unsigned)grid), dim3(64), 0, s, A, tab, job, pg);
}

template <typename T, int MT>
bool dispatch_piece(const SgOpArgs<T>& A, const StripTables<T>& tab, const MarchJob& job, const PieceGeom& pg,
                    hipStream_t s) {
  if (tab.M == MT) {
    launch_piece<T, MT>(A, tab, job, pg, s);
    return true;
  }
  if constexpr (MT > 0) return dispatch_piece<T, MT - 1>(A, tab, job, pg, s);
  return false;
}

template <typename T, int MT>
void launch_march(const SgOpArgs<T>& A, const StripTables<T>& tab, const MarchJob& job, hipStream_t s) {
  const int nblocks = job.ngroups * job.nseg;
  const int grid = (nblocks + 7) / 8 * 8;
  hipLaunchKernelGGL((sgop_march_kernel<T, MT>), dim3(grid), dim3(A.n_e), 0, s, A, tab, job);
}

template <typename T, int MT>
bool dispatch_march(const SgOpArgs<T>& A, const StripTables<T>& tab, const MarchJob& job, hipStream_t s) {
  if (tab.M == MT) {
    launch_march<T, MT>(A, tab, job, s);
    return true;
  }
  if constexpr (MT > 0) return dispatch_march<T, MT - 1>(A, tab, job, s);
  return false;
}

template <int MT>
int march_occ(int M, int block) {
  if (M == MT) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sgop_march_kernel<double, MT>, block, 0) != hipSuccess)
      return 0;
    return nb;
  }
  if constexpr (MT > 0) return march_occ<MT - 1>(M, block);
  return 0;
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

bool march_supported(int n_e, int M) { return n_e % 64 == 0 && n_e >= 64 && n_e <= 512 && M <= kStripMaxM; }

int march_blocks_per_cu(int M, int block) { return march_occ<kStripMaxM>(M, block); }

// ---------------------------------------------------------------------------
// Row-staged full operator (FP64). A block (one per CU: the staged rows take
// most of the LDS) works through pieces of kStageOut node columns by TY node
// rows. For each element row e of a piece (between node rows e - 1 and e) it
// holds node rows e - 1 and e of every chaos column, and the coefficients of
// element row e, in LDS; the next row is loaded into registers while the
// current one is used. Each half wave owns a list of output columns a; for
// every term (b, k, g) of a (b = a: k = 0 and g = 1 with coefficient theta0;
// b = a -+ e_k: the Galerkin weight g of G_k) it forms, lane by lane,
//   R0 += g c_k(right element) U_b(e - 1),  R1 += g c_k(right element) U_b(e),
//   L0 += g c_k(left element) U_b(e - 1),   L1 += g c_k(left element) U_b(e),
// the corner values of sum_terms c g U_b on the element right of the node
// (BL = R0, TL = R1; BR and TR are the next lane's L0, L1). The element matrix
// of the Q1 Laplacian (times 6: 4 on the diagonal, -1 along the edges, -2
// across) turns them into the element's contributions to its four corners,
// which complete node row e - 1 and start node row e of output a.
// ---------------------------------------------------------------------------
size_t stage_lds_bytes(int P, int M, int nterms, int nslots) {
  if (P < 1 || P >= 0xFFFF || M < 0 || M > 255 || nterms < 0 || nterms > 0xFFFF || nslots < 1) return 0;
  if ((long)P * kStageLanes > (long)kStagePre * kStageWaves * 64) return 0;
  if ((M + 1) * kStageLanes > kStageWaves * 64) return 0;
  // node rows [P][32 lanes][2 parities], coefficients [M + 1][32], terms, slots
  const size_t b = sizeof(double) * ((size_t)P * 2 * kStageLanes + (size_t)(M + 1) * kStageLanes) +
                   sizeof(StageTerm) * (size_t)nterms + sizeof(StageSlot) * (size_t)nslots;
  return b <= 160 * 1024 ? b : 0;
}

namespace {

// One element row e of a piece: node rows e - 1 (parity 1 - PE) and e (parity PE)
// and the coefficients of element row e are in LDS; the next node row (parity
// 1 - PE) and coefficient row are loaded meanwhile and stored after the step's
// reads. Completes output node row e - 1 (if e > y0) and starts row e.
template <int PE>
__device__ __forceinline__ void stage_step(const SgOpArgs<double>& A, const StageJob& J, double* Ub, double* Cb,
                                           const StageTerm* Tl, const StageSlot* Sl, int e, int y0, int y1, int x0,
                                           int s_begin, int s_end, double (&Yc)[kStageSlots]) {
  const int tid = threadIdx.x, lane = tid & 63, l32 = lane & 31;
  const int nx = A.nx, n_e = A.n_e;
  const long n = A.n;
  const int P = J.P, MC = J.M + 1;
  const bool more = e < y1;
  // the next rows into registers: thread tid stages lane tid % 32 of chaos
  // columns tid / 32 + 32 j (32-bit offsets: the host enables this kernel only
  // for n P < 2^31)
  const int sb = tid >> 5, sx = x0 - 1 + (tid & 31);
  double nv[kStagePre];
  double nc = 0.0;
  if (more) {
    const int gy = e + 1;
    const bool ok = gy < nx && sx >= 0 && sx < nx;
    const unsigned base = (unsigned)sb * (unsigned)n + (unsigned)(gy * nx + sx);
    const unsigned step = 32u * (unsigned)n;
#pragma unroll
    for (int j = 0; j < kStagePre; ++j) nv[j] = (ok && sb + 32 * j < P) ? A.in[base + (unsigned)j * step] : 0.0;
    if (tid < MC * kStageLanes) {
      const int k = tid >> 5, ex = x0 + (tid & 31);
      if (ex < n_e) nc = k == 0 ? A.diag : A.a[(long)(k - 1) * n_e * n_e + (long)gy * n_e + ex];
    }
  }
  const double2* Ul = reinterpret_cast<const double2*>(Ub) + l32;  // (node row parity 0, parity 1)
  const double* Cl = Cb + l32;                                      // right element of the lane's node
  const unsigned hb = (lane >> 5) * 16u, hk = (lane >> 5) * 8u;
  const int gx = x0 - 1 + l32;
  const double scale = 1.0 / 6.0, theta0 = A.diag;
  auto accumulate = [&](double g, const double2& uv, double cr, double& R0, double& R1, double& L0, double& L1) {
    const double u0 = PE ? uv.x : uv.y, u1 = PE ? uv.y : uv.x;  // node rows e - 1, e
    const double gr = g * cr, gl = from_prev(gr);                 // the left element is the previous lane's right one
    R0 = fma(gr, u0, R0);
    R1 = fma(gr, u1, R1);
    L0 = fma(gl, u0, L0);
    L1 = fma(gl, u1, L1);
  };
  // a term's staged values: U_b at node rows e - 1 and e (one 16-byte read) and
  // the coefficient of k on the right element
  auto term_vals = [&](const uint4& q, double2& uv, double& cr, double& g) {
    const unsigned b = (q.x >> hb) & 0xFFFFu, k = (q.y >> hk) & 0xFFu;
    uv = Ul[b * kStageLanes];
    cr = Cl[k * kStageLanes];
    g = __hiloint2double((int)q.w, (int)q.z);
  };
#pragma unroll
  for (int s = 0; s < kStageSlots; ++s) {
    const int si = s_begin + s;
    if (si < s_end) {
      const uint2 sv = *reinterpret_cast<const uint2*>(Sl + si);
      const int t0 = __builtin_amdgcn_readfirstlane((int)(sv.y & 0xFFFFu));
      const int nt = __builtin_amdgcn_readfirstlane((int)(sv.y >> 16));
      const unsigned oh = (sv.x >> hb) & 0xFFFFu;
      const int out = oh == 0xFFFFu ? -1 : (int)oh;
      // the mean term: coefficient theta0 on both elements, weight 1
      const double2 ud = Ul[(out >= 0 ? out : (int)(sv.x & 0xFFFFu)) * kStageLanes];
      const double d0 = theta0 * (PE ? ud.x : ud.y), d1 = theta0 * (PE ? ud.y : ud.x);
      double R0 = d0, R1 = d1, L0 = d0, L1 = d1;
      const uint4* tq = reinterpret_cast<const uint4*>(Tl + t0);
      int t = 0;
      // two terms at a time: every LDS read of both goes out before the arithmetic
      for (; t + 1 < nt; t += 2) {
        const uint4 qa = tq[t], qb = tq[t + 1];
        double2 ua, ub;
        double ca, cb, ga, gb;
        term_vals(qa, ua, ca, ga);
        term_vals(qb, ub, cb, gb);
        accumulate(ga, ua, ca, R0, R1, L0, L1);
        accumulate(gb, ub, cb, R0, R1, L0, L1);
      }
      if (t < nt) {
        double2 ua;
        double ca, ga;
        term_vals(tq[t], ua, ca, ga);
        accumulate(ga, ua, ca, R0, R1, L0, L1);
      }
      const double BL = R0, TL = R1, BR = from_next(L0), TR = from_next(L1);
      const double S = (BL + BR) + (TR + TL);
      const double oBL = 5.0 * BL - S - TR;
      const double oBR = 5.0 * BR - S - TL;
      const double oTR = 5.0 * TR - S - BL;
      const double oTL = 5.0 * TL - S - BR;
      const double bot = oBL + from_prev(oBR);  // node row e - 1
      const double top = oTL + from_prev(oTR);  // node row e
      if (e > y0 && out >= 0 && l32 >= 1 && l32 <= kStageOut && gx < nx)
        A.out[(unsigned)out * (unsigned)n + (unsigned)((e - 1) * nx + gx)] = scale * (Yc[s] + bot);
      Yc[s] = top;
    }
  }
  __syncthreads();  // every read of node row e - 1 and of element row e is done
  if (more) {
    double* dst = Ub + (sb * kStageLanes + (tid & 31)) * 2 + (1 - PE);
#pragma unroll
    for (int j = 0; j < kStagePre; ++j)
      if (sb + 32 * j < P) dst[j * 32 * (2 * kStageLanes)] = nv[j];
    if (tid < MC * kStageLanes) Cb[tid] = nc;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kStageWaves * 64) sgop_stage_kernel(const SgOpArgs<double> A, const StageJob J) {
  if (A.active && ld_uniform(A.active, 0) == 0) return;
  extern __shared__ double stage_lds[];
  const int P = J.P, MC = J.M + 1;
  double* Ub = stage_lds;                              // [P][32][2]: node rows by parity
  double* Cb = Ub + P * 2 * kStageLanes;               // [M + 1][32]: coefficients of the current element row
  StageTerm* Tl = reinterpret_cast<StageTerm*>(Cb + MC * kStageLanes);
  StageSlot* Sl = reinterpret_cast<StageSlot*>(Tl + J.nterms);
  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nx = A.nx, n_e = A.n_e;
  const long n = A.n;
  const int s_begin = ld_uniform(J.wslot, wv), s_end = ld_uniform(J.wslot, wv + 1);
  // the term and slot tables into LDS (16 and 8 bytes per entry)
  for (int i = tid; i < J.nterms; i += kStageWaves * 64)
    reinterpret_cast<uint4*>(Tl)[i] = reinterpret_cast<const uint4*>(J.terms)[i];
  for (int i = tid; i < J.nslots; i += kStageWaves * 64)
    reinterpret_cast<uint2*>(Sl)[i] = reinterpret_cast<const uint2*>(J.slots)[i];
  // pieces of this block's XCD (block b runs on XCD b mod 8), a contiguous band
  const int xcd = blockIdx.x % 8, bslot = blockIdx.x / 8;
  const int nb = ((int)gridDim.x - xcd + 7) / 8;
  const long npieces = (long)J.nyseg * J.nseg;
  const long p0 = npieces * xcd / 8, p1 = npieces * (xcd + 1) / 8;
  for (long pc = p0 + bslot; pc < p1; pc += nb) {
    const int yseg = (int)(pc / J.nseg), seg = (int)(pc % J.nseg);
    const int x0 = seg * kStageOut;     // first output node column
    const int y0 = yseg * J.TY;
    const int y1 = min(nx, y0 + J.TY);  // output node rows [y0, y1)
    // prologue: node rows y0 - 1 and y0, coefficients of element row y0
    for (int r = 0; r < 2; ++r) {
      const int gy = y0 - 1 + r, par = (y0 + 1 + r) & 1;
      const int sb = tid >> 5, sx = x0 - 1 + (tid & 31);
      const bool ok = gy >= 0 && gy < nx && sx >= 0 && sx < nx;
      const unsigned base = (unsigned)sb * (unsigned)n + (unsigned)(gy * nx + sx);
      double* dst = Ub + (sb * kStageLanes + (tid & 31)) * 2 + par;
      for (int j = 0; j < kStagePre; ++j)
        if (sb + 32 * j < P) dst[j * 32 * (2 * kStageLanes)] = ok ? A.in[base + (unsigned)j * 32u * (unsigned)n] : 0.0;
    }
    if (tid < MC * kStageLanes) {
      const int k = tid >> 5, ex = x0 + (tid & 31);
      double c = 0.0;
      if (ex < n_e) c = k == 0 ? A.diag : A.a[(long)(k - 1) * n_e * n_e + (long)y0 * n_e + ex];
      Cb[tid] = c;
    }
    __syncthreads();
    double Yc[kStageSlots];
#pragma unroll
    for (int s = 0; s < kStageSlots; ++s) Yc[s] = 0.0;
    for (int e = y0; e <= y1; ++e) {
      if (e & 1) stage_step<1>(A, J, Ub, Cb, Tl, Sl, e, y0, y1, x0, s_begin, s_end, Yc);
      else stage_step<0>(A, J, Ub, Cb, Tl, Sl, e, y0, y1, x0, s_begin, s_end, Yc);
    }
  }
}

}  // namespace

void launch_stage(const SgOpArgs<double>& args, const StageJob& job, hipStream_t s) {
  const size_t lds = stage_lds_bytes(job.P, job.M, job.nterms, job.nslots);
  if (lds == 0) return;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(sgop_stage_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int dev = 0, ncu = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const long npieces = (long)job.nyseg * job.nseg;
  long grid = ncu;
  if (grid > npieces) grid = npieces;
  grid = (grid + 7) / 8 * 8;
  hipLaunchKernelGGL(sgop_stage_kernel, dim3((unsigned)grid), dim3(kStageWaves * 64), lds, s, args, job);
}

template <typename T>
void launch_sgop(const SgOpArgs<T>& args, const StripTables<T>& tab, const MarchJob* job, hipStream_t s) {
  if (args.nrows <= 0) return;
  if (job != nullptr && job->piece.W > 0 && tab.lo != nullptr && job->ngroups > 0 &&
      dispatch_piece<T, kStripMaxM>(args, tab, *job, job->piece, s))
    return;
  const bool shape_ok = args.n_e % 64 == 0 && args.n_e >= 64 && args.n_e <= 512;
  if (job != nullptr && shape_ok && tab.lo != nullptr && job->ngroups > 0 &&
      dispatch_march<T, kStripMaxM>(args, tab, *job, s))
    return;
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

template void launch_sgop<double>(const SgOpArgs<double>&, const StripTables<double>&, const MarchJob*,
                                  hipStream_t);
template void launch_sgop<float>(const SgOpArgs<float>&, const StripTables<float>&, const MarchJob*,
                                 hipStream_t);

}  // namespace sgk
