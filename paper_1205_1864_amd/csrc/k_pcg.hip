// Persistent batched PCG for the diagonal-block solves of Algorithm 1
// (Section 5: independent inner Krylov loops on blocks equal to the mean
// matrix K_0 = theta0 * K_Lap). One cooperative launch runs every column of a
// batch to convergence; each column stops on its own.
//
// Preconditioner: d updates of the Chebyshev iteration for
// (D^-1 K_0) z = D^-1 r from z = 0 (D = diag K_0 = theta0 * 8/3), i.e.
// z = p(D^-1 K_0) D^-1 r for a fixed polynomial. Its d - 1 stencil sweeps run
// in LDS on a tile grown by a halo of d - 1 nodes, so a preconditioner
// application reads r and q once and writes z once.
//
// Per PCG iteration every column passes two phases:
//   phase A: p = z + beta p (tile plus a 1-node halo), q = K_0 p, partial p.q;
//   phase B: alpha = gamma / p.q, x += alpha p, r -= alpha q (tile plus the
//            Chebyshev halo), z = M r, partials r.r and r.z.
// A column is split into TS x TS tiles; each block owns a contiguous run of
// tiles (the same tiles in every phase) and works on G tiles at a time, one
// per 256-thread group. Columns synchronise only among the blocks that share
// them, through split-phase counters (no grid-wide barrier). Per-column scalars
// are reduced from per-tile partials in a fixed order, identically in every
// block, so all owners of a column take the same decisions.
//
// The same kernel runs a ragged set of columns from several problems (grids
// of different sizes, own constants, a per-problem skip flag): the tiles of
// all columns form one work list and every column keeps its own arithmetic,
// so a column's iterates do not depend on what else is in the launch.
#include "sg_internal.h"
#include "sg_device.h"

namespace sgk {

namespace {

constexpr int kGroup = 256;                // threads per tile group
constexpr long kSpinLimit = 1L << 26;      // bounded waits: a stuck column aborts the launch

enum { PART_BB = 0, PART_PQ = 1, PART_RR0 = 2, PART_RR1 = 3, PART_RZ0 = 4, PART_RZ1 = 5, PART_N = 6 };

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Split-phase barrier of one column: every block that owns tiles of the column
// adds its tile count to a monotonic arrival counter after finishing its tiles;
// phase k of the column is complete once the counter reaches k * ntiles.
__device__ void column_arrive(unsigned* arr, unsigned count) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(arr, count);
  }
}

__device__ bool column_wait(const unsigned* arr, unsigned target, int* status, int* sflag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    long spins = 0;
    int ok = 1;
    while (__hip_atomic_load(arr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        ok = 0;
        atomicExch(status, 1);
        break;
      }
    }
    __threadfence();
    *sflag = ok;
  }
  __syncthreads();
  return *sflag != 0;
}

// Per-group sum of one value per thread, fixed order; the result is returned
// to every thread of the group. All threads of the block must call it together.
template <int G>
__device__ double group_sum(double v, double (*sred)[4]) {
  v = wave_sum(v);
  const int g = threadIdx.x / kGroup, wv = (threadIdx.x % kGroup) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sred[g][wv] = v;
  __syncthreads();
  return sred[g][0] + sred[g][1] + sred[g][2] + sred[g][3];
}

template <int TS>
struct Interior {
  static constexpr int NI = (TS * TS + kGroup - 1) / kGroup;  // interior nodes per thread
};

// Chebyshev preconditioner on one tile for one group. `rreg(lx, ly)` gives r
// on the region (tile plus halo H = degree - 1; only called inside the
// domain). On return Zi holds z and Ri holds r on this thread's interior
// nodes; the return value is the thread's partial r.z. With `valid` false the
// group only takes part in the block-wide synchronisation.
// The grid, state vectors and constants of one column.
template <typename T>
struct ColView {
  int nx, ntx, ntiles;
  long tbase;  // first index of the column's per-tile partials (and of its work items)
  const T* b;
  T *x, *r0, *r1, *p0, *p1, *q, *z;
  T c0, c1, inv_diag, inv_theta;
  const T* chebA;
  const T* chebB;
};

template <typename T, int TS, int NS, typename RF>
__device__ double cheb_tile(const ColView<T>& A, int degree, bool valid, int x0, int y0, RF rreg, T* W0, T* W1,
                            T (&Zi)[Interior<TS>::NI], T (&Ri)[Interior<TS>::NI]) {
  constexpr int NI = Interior<TS>::NI;
  const int lt = threadIdx.x % kGroup;
  const int H = degree - 1;
  const int RS = TS + 2 * H;
  const int nreg = RS * RS;
  T S[NS];
  // step 0: S = D^-1 r, W = S / theta; r parked in W1 for the interior mapping
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = lt + s * kGroup;
    S[s] = T(0);
    if (valid && i < nreg) {
      const int lx = i % RS, ly = i / RS;
      const int gx = x0 - H + lx, gy = y0 - H + ly;
      const T r = (gx >= 0 && gx < A.nx && gy >= 0 && gy < A.nx) ? rreg(lx, ly) : T(0);
      S[s] = r * A.inv_diag;
      W0[i] = S[s] * A.inv_theta;
      W1[i] = r;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NI; ++k) {
    const int i = lt + k * kGroup;
    Zi[k] = T(0);
    Ri[k] = T(0);
    if (valid && i < TS * TS) {
      const int j = (i / TS + H) * RS + (i % TS + H);
      Zi[k] = W0[j];
      Ri[k] = W1[j];
    }
  }
  T* cur = W0;
  T* nxt = W1;
  for (int j = 1; j < degree; ++j) {
    __syncthreads();  // reads of the buffer about to be overwritten are done
    const T ca = ld_uniform(A.chebA, j), cb = ld_uniform(A.chebB, j);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = lt + s * kGroup;
      if (valid && i < nreg) {
        const int lx = i % RS, ly = i / RS;
        if (lx >= j && lx < RS - j && ly >= j && ly < RS - j) {  // W_j is valid on [j, RS - j)
          const int gx = x0 - H + lx, gy = y0 - H + ly;
          T wn = T(0);
          if (gx >= 0 && gx < A.nx && gy >= 0 && gy < A.nx) {
            const T s8 = cur[i - RS - 1] + cur[i - RS] + cur[i - RS + 1] + cur[i - 1] + cur[i + 1] +
                         cur[i + RS - 1] + cur[i + RS] + cur[i + RS + 1];
            S[s] = S[s] - (cur[i] - T(0.125) * s8);
            wn = ca * cur[i] + cb * S[s];
          }
          nxt[i] = wn;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int i = lt + k * kGroup;
      if (valid && i < TS * TS) Zi[k] += nxt[(i / TS + H) * RS + (i % TS + H)];
    }
    T* t = cur;
    cur = nxt;
    nxt = t;
  }
  double rz = 0.0;
#pragma unroll
  for (int k = 0; k < NI; ++k) rz += (double)Ri[k] * (double)Zi[k];
  return rz;
}

template <typename T, int TS, int NS, int G, bool RAGGED>
__global__ void __launch_bounds__(kGroup* G) pcg_kernel(const PcgArgs<T> A, const PcgCols<T> C) {
  constexpr int NI = Interior<TS>::NI;
  extern __shared__ unsigned char smem_raw[];
  const int grp = threadIdx.x / kGroup;
  const int lt = threadIdx.x % kGroup;
  const int degree = A.degree;
  const int H = degree - 1;
  const int RSa = TS + 2 * (H > 1 ? H : 1);  // phase A needs a 1-node halo
  const int CAP = RSa * RSa;
  T* W0 = reinterpret_cast<T*>(smem_raw) + (long)grp * 2 * CAP;
  T* W1 = W0 + CAP;
  // per-column done flags of this block's columns, after the tile buffers
  int* sdone = reinterpret_cast<int*>(reinterpret_cast<T*>(smem_raw) + (long)G * 2 * CAP);
  __shared__ double sred[G][4];
  __shared__ double s4[4];
  __shared__ int sflag;

  // a compacted ragged launch covers the listed columns only; scratch is indexed by list position
  const bool listed = RAGGED && C.act != nullptr;
  const int ncols = listed ? ld_uniform(C.nact, 0) : A.ncols;
  const long nslots = RAGGED ? C.nwork : (long)A.ncols * A.ntiles;  // stride of the partial arrays
  const long nwork = listed ? ld_uniform(C.nwork_act, 0) : nslots;
  if (ncols <= 0 || nwork <= 0) return;
  double* part = A.sc.part;
  unsigned* arr = A.sc.arrivals;
  auto P = [&](int which) { return part + (long)which * nslots; };
  // the grid, vectors and constants of column c
  auto view = [&](int c) {
    ColView<T> v;
    if constexpr (RAGGED) {
      const int o = listed ? ld_uniform(C.act, c) : c;  // index into the column arrays
      v.nx = ld_uniform(C.nx, o);
      v.ntx = ld_uniform(C.ntx, o);
      v.ntiles = ld_uniform(C.ntiles, o);
      v.tbase = listed ? ld_uniform(C.cbase, c) : ld_uniform(C.tbase, o);
      v.b = ld_uniform(C.b, o);
      v.x = ld_uniform(C.x, o);
      v.r0 = ld_uniform(C.r0, o);
      v.r1 = ld_uniform(C.r1, o);
      v.p0 = ld_uniform(C.p0, o);
      v.p1 = ld_uniform(C.p1, o);
      v.q = ld_uniform(C.q, o);
      v.z = ld_uniform(C.z, o);
      const PcgConsts<T>* k = C.consts + ld_uniform(C.prob, o);
      v.c0 = ld_uniform(&k->c0, 0);
      v.c1 = ld_uniform(&k->c1, 0);
      v.inv_diag = ld_uniform(&k->inv_diag, 0);
      v.inv_theta = ld_uniform(&k->inv_theta, 0);
      v.chebA = k->chebA;
      v.chebB = k->chebB;
    } else {
      const long n = A.n;
      v.nx = A.nx;
      v.ntx = A.ntx;
      v.ntiles = A.ntiles;
      v.tbase = (long)c * A.ntiles;
      v.b = A.B + (long)c * n;
      v.x = A.X + (long)c * n;
      v.r0 = A.R0 + (long)c * n;
      v.r1 = A.R1 + (long)c * n;
      v.p0 = A.P0 + (long)c * n;
      v.p1 = A.P1 + (long)c * n;
      v.q = A.Q + (long)c * n;
      v.z = A.Z + (long)c * n;
      v.c0 = A.c0;
      v.c1 = A.c1;
      v.inv_diag = A.inv_diag;
      v.inv_theta = A.inv_theta;
      v.chebA = A.chebA;
      v.chebB = A.chebB;
    }
    return v;
  };
  // column holding work index w
  auto column_of = [&](long w) {
    if constexpr (RAGGED) {
      const long* base = listed ? C.cbase : C.tbase;
      int lo = 0, hi = ncols - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ld_uniform(base, mid) <= w) lo = mid; else hi = mid - 1;
      }
      return lo;
    } else {
      return (int)(w / A.ntiles);
    }
  };
  const long per_block = (nwork + gridDim.x - 1) / gridDim.x;
  const long w_begin = (long)blockIdx.x * per_block;
  const long w_end = w_begin + per_block < nwork ? w_begin + per_block : nwork;
  if (w_begin >= w_end) return;
  const int c_first = column_of(w_begin), c_last = column_of(w_end - 1);
  // tiles of the column that fall in this block's range [w_begin, w_end)
  auto tiles_of = [&](const ColView<T>& v, int& t0, int& t1) {
    const long lo = v.tbase > w_begin ? v.tbase : w_begin;
    const long hi = v.tbase + v.ntiles < w_end ? v.tbase + v.ntiles : w_end;
    t0 = (int)(lo - v.tbase);
    t1 = (int)(hi - v.tbase);
  };
  auto owner = [&](const ColView<T>& v) { return v.tbase >= w_begin; };  // this block holds tile 0
  // Fixed-order sums of up to four per-tile partial arrays of a column, one wave each.
  auto col_sums = [&](const ColView<T>& v, const double* q0, const double* q1, const double* q2, const double* q3) {
    __syncthreads();
    const int wv = threadIdx.x >> 6;
    const double* src = wv == 0 ? q0 : wv == 1 ? q1 : wv == 2 ? q2 : q3;
    if (wv < 4 && src) {
      double s = 0.0;
      for (int t = threadIdx.x & 63; t < v.ntiles; t += 64) s += src[v.tbase + t];
      s = wave_sum(s);
      if ((threadIdx.x & 63) == 0) s4[wv] = s;
    }
    __syncthreads();
  };
  auto tile_xy = [&](const ColView<T>& v, int t, int& x0, int& y0) {
    x0 = (t % v.ntx) * TS;
    y0 = (t / v.ntx) * TS;
  };
  for (int c = c_first + (int)threadIdx.x; c <= c_last; c += kGroup * G) {
    int skip = 0;
    if constexpr (RAGGED) {
      if (!listed) skip = C.active[C.prob[c]] == 0;
    }
    sdone[c - c_first] = skip;
  }
  __syncthreads();

  T Zi[NI], Ri[NI];

  // ---- start (column phase 1): x = 0, z = M b, partials b.b and b.z
  for (int c = c_first; c <= c_last; ++c) {
    const ColView<T> v = view(c);
    if (sdone[c - c_first]) {
      if (threadIdx.x == 0 && owner(v)) A.sc.iters[c] = 0;
      continue;
    }
    int t0, t1;
    tiles_of(v, t0, t1);
    if (t1 <= t0) continue;
    const int nx = v.nx;
    for (int tb = t0; tb < t1; tb += G) {
      const int t = tb + grp;
      const bool valid = t < t1;
      int x0 = 0, y0 = 0;
      if (valid) tile_xy(v, t, x0, y0);
      __syncthreads();
      auto rreg = [&](int lx, int ly) { return v.b[(long)(y0 - H + ly) * nx + (x0 - H + lx)]; };
      double rz = cheb_tile<T, TS, NS>(v, degree, valid, x0, y0, rreg, W0, W1, Zi, Ri);
      double bb = 0.0;
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const int i = lt + k * kGroup;
        const int gx = x0 + i % TS, gy = y0 + i / TS;
        if (valid && i < TS * TS && gx < nx && gy < nx) {
          const long g = (long)gy * nx + gx;
          bb += (double)Ri[k] * (double)Ri[k];
          v.x[g] = T(0);
          v.z[g] = Zi[k];
        }
      }
      rz = group_sum<G>(rz, sred);
      bb = group_sum<G>(bb, sred);
      if (valid && lt == 0) {
        P(PART_RZ1)[v.tbase + t] = rz;
        P(PART_BB)[v.tbase + t] = bb;
      }
    }
    column_arrive(arr + c, (unsigned)(t1 - t0));
  }

  bool aborted = false;
  for (int it = 0; it < A.maxit && !aborted; ++it) {
    const int par = it & 1;
    bool any_active = false;
    // ---- phase A (column phase 2 + 2 it): p = z + beta p, q = K_0 p, partial p.q
    for (int c = c_first; c <= c_last && !aborted; ++c) {
      if (sdone[c - c_first]) continue;
      const ColView<T> v = view(c);
      int t0, t1;
      tiles_of(v, t0, t1);
      if (t1 <= t0) continue;
      if (!column_wait(arr + c, (unsigned)((1 + 2 * it) * v.ntiles), A.sc.status, &sflag)) {
        aborted = true;
        break;
      }
      col_sums(v, P(PART_BB), it == 0 ? nullptr : P(par ? PART_RR0 : PART_RR1),
               it == 0 ? nullptr : P(par ? PART_RZ0 : PART_RZ1), it == 0 ? nullptr : P(par ? PART_RZ1 : PART_RZ0));
      const double bb = s4[0];
      const double rr = it == 0 ? s4[0] : s4[1];
      if (sqrt(rr) <= A.rtol * sqrt(bb)) {
        __syncthreads();
        if (threadIdx.x == 0) {
          sdone[c - c_first] = 1;
          if (owner(v)) A.sc.iters[c] = it;
        }
        __syncthreads();
        continue;
      }
      const T beta = it == 0 ? T(0) : (T)(s4[2] / s4[3]);
      any_active = true;
      const int nx = v.nx;
      const T* zc = v.z;
      const T* po = par ? v.p0 : v.p1;
      T* pn = par ? v.p1 : v.p0;
      T* qc = v.q;
      const int RS1 = TS + 2;
      for (int tb = t0; tb < t1; tb += G) {
        const int t = tb + grp;
        const bool valid = t < t1;
        int x0 = 0, y0 = 0;
        if (valid) tile_xy(v, t, x0, y0);
        __syncthreads();
        if (valid) {
          for (int i = lt; i < RS1 * RS1; i += kGroup) {
            const int gx = x0 - 1 + i % RS1, gy = y0 - 1 + i / RS1;
            T val = T(0);
            if (gx >= 0 && gx < nx && gy >= 0 && gy < nx) {
              const long g = (long)gy * nx + gx;
              val = it == 0 ? zc[g] : zc[g] + beta * po[g];
            }
            W0[i] = val;
          }
        }
        __syncthreads();
        double pq = 0.0;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
          const int i = lt + k * kGroup;
          const int lx = i % TS + 1, ly = i / TS + 1;
          const int gx = x0 + lx - 1, gy = y0 + ly - 1;
          if (valid && i < TS * TS && gx < nx && gy < nx) {
            const int q = ly * RS1 + lx;
            const T pc = W0[q];
            const T s8 = W0[q - RS1 - 1] + W0[q - RS1] + W0[q - RS1 + 1] + W0[q - 1] + W0[q + 1] +
                         W0[q + RS1 - 1] + W0[q + RS1] + W0[q + RS1 + 1];
            const T qv = v.c0 * pc + v.c1 * s8;
            const long g = (long)gy * nx + gx;
            pn[g] = pc;
            qc[g] = qv;
            pq += (double)pc * (double)qv;
          }
        }
        pq = group_sum<G>(pq, sred);
        if (valid && lt == 0) P(PART_PQ)[v.tbase + t] = pq;
      }
      column_arrive(arr + c, (unsigned)(t1 - t0));
    }
    if (!any_active || aborted) break;
    // ---- phase B (column phase 3 + 2 it): x += alpha p, r -= alpha q, z = M r, partials r.r, r.z
    for (int c = c_first; c <= c_last && !aborted; ++c) {
      if (sdone[c - c_first]) continue;
      const ColView<T> v = view(c);
      int t0, t1;
      tiles_of(v, t0, t1);
      if (t1 <= t0) continue;
      if (!column_wait(arr + c, (unsigned)((2 + 2 * it) * v.ntiles), A.sc.status, &sflag)) {
        aborted = true;
        break;
      }
      col_sums(v, P(PART_PQ), P(par ? PART_RZ0 : PART_RZ1), nullptr, nullptr);
      const double pq = s4[0], gam = s4[1];
      if (!(pq > 0.0) || !isfinite(pq)) {
        // breakdown: keep the current iterate
        __syncthreads();
        if (threadIdx.x == 0) {
          sdone[c - c_first] = 1;
          if (owner(v)) A.sc.iters[c] = it;
        }
        __syncthreads();
        continue;
      }
      const T alpha = (T)(gam / pq);
      const int nx = v.nx;
      const T* pc = par ? v.p1 : v.p0;
      const T* qc = v.q;
      const T* ro = it == 0 ? v.b : (par ? v.r1 : v.r0);
      T* rn = par ? v.r0 : v.r1;
      T* xc = v.x;
      T* zc = v.z;
      for (int tb = t0; tb < t1; tb += G) {
        const int t = tb + grp;
        const bool valid = t < t1;
        int x0 = 0, y0 = 0;
        if (valid) tile_xy(v, t, x0, y0);
        __syncthreads();
        auto rreg = [&](int lx, int ly) {
          const long g = (long)(y0 - H + ly) * nx + (x0 - H + lx);
          return ro[g] - alpha * qc[g];
        };
        double rz = cheb_tile<T, TS, NS>(v, degree, valid, x0, y0, rreg, W0, W1, Zi, Ri);
        double rr = 0.0;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
          const int i = lt + k * kGroup;
          const int gx = x0 + i % TS, gy = y0 + i / TS;
          if (valid && i < TS * TS && gx < nx && gy < nx) {
            const long g = (long)gy * nx + gx;
            xc[g] = it == 0 ? alpha * pc[g] : xc[g] + alpha * pc[g];
            rn[g] = Ri[k];
            zc[g] = Zi[k];
            rr += (double)Ri[k] * (double)Ri[k];
          }
        }
        rz = group_sum<G>(rz, sred);
        rr = group_sum<G>(rr, sred);
        if (valid && lt == 0) {
          P(par ? PART_RZ1 : PART_RZ0)[v.tbase + t] = rz;
          P(par ? PART_RR1 : PART_RR0)[v.tbase + t] = rr;
        }
      }
      column_arrive(arr + c, (unsigned)(t1 - t0));
    }
  }
  // ---- iteration counts of columns that ran out of iterations
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = c_first; c <= c_last; ++c)
      if (!sdone[c - c_first] && owner(view(c))) A.sc.iters[c] = A.maxit;
  }
}

// Zero the per-column arrival counters and the status word before a launch.
__global__ void pcg_reset_kernel(unsigned* arr, int ncols, int* status) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncols; c += gridDim.x * blockDim.x) arr[c] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
}

template <typename T, int TS, int NS, int G, bool RAGGED>
hipError_t launch_cfg(const PcgArgs<T>& args, const PcgCols<T>& cols, int max_blocks, hipStream_t s) {
  const int H = args.degree - 1;
  const int RSa = TS + 2 * (H > 1 ? H : 1);
  if ((TS + 2 * H) * (TS + 2 * H) > NS * kGroup) return hipErrorInvalidValue;
  const size_t tiles_bytes = sizeof(T) * 2 * (size_t)RSa * RSa * G;
  auto kfn = pcg_kernel<T, TS, NS, G, RAGGED>;
  const long nwork = RAGGED ? cols.nwork : (long)args.ncols * args.ntiles;
  if (nwork <= 0) return hipSuccess;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int ncu = 0;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  // Enough blocks to keep every tile group busy, as few as possible beyond
  // that: every block pays a device-wide release per column and phase. The
  // grid must fit on the device at once with the LDS it needs (tile buffers
  // plus one done flag per column a block can touch).
  const long min_tiles = RAGGED ? 1 : args.ntiles;
  long grid = (nwork + 2L * G - 1) / (2L * G);
  if (max_blocks > 0 && grid > max_blocks) grid = max_blocks;
  if (grid < 1) grid = 1;
  size_t sm = 0;
  for (int pass = 0; pass < 8; ++pass) {
    const long per_block = (nwork + grid - 1) / grid;
    const long max_cols = per_block / min_tiles + 2;  // a run of per_block items spans at most this many columns
    sm = tiles_bytes + sizeof(int) * (size_t)max_cols;
    if (sm > 160 * 1024) return hipErrorInvalidValue;
    // the cooperative launch checks co-residency against this attribute, so keep it exact
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kGroup * G, sm);
    if (e != hipSuccess) return e;
    const long cap = (long)per_cu * ncu;
    if (cap < 1) return hipErrorInvalidValue;
    if (grid <= cap) break;
    grid = cap;
    if (pass == 7) return hipErrorInvalidValue;
  }
  PcgArgs<T> a = args;
  PcgCols<T> c = cols;
  hipLaunchKernelGGL(pcg_reset_kernel, dim3(1), dim3(256), 0, s, a.sc.arrivals, a.ncols, a.sc.status);
  if (!RAGGED) {
    void* kargs[] = {&a, &c};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kfn), dim3((unsigned)grid),
                                      dim3(kGroup * G), kargs, (unsigned)sm, s);
  }
  hipLaunchKernelGGL(kfn, dim3((unsigned)grid), dim3(kGroup * G), sm, s, a, c);
  return hipGetLastError();
}

constexpr int slots(int ts, int maxh) { return ((ts + 2 * maxh) * (ts + 2 * maxh) + kGroup - 1) / kGroup; }

template <typename T, bool RAGGED>
hipError_t dispatch_pcg(const PcgArgs<T>& args, const PcgCols<T>& cols, int tile, int max_blocks, hipStream_t s) {
  if (args.ncols <= 0) return hipSuccess;
  const int H = args.degree - 1;
  if (tile == 32) {
    if (H <= 3) return launch_cfg<T, 32, slots(32, 3), 4, RAGGED>(args, cols, max_blocks, s);
    if (H <= 7) return launch_cfg<T, 32, slots(32, 7), 3, RAGGED>(args, cols, max_blocks, s);
  }
  return launch_cfg<T, 16, slots(16, 15), 4, RAGGED>(args, cols, max_blocks, s);
}

}  // namespace

template <typename T>
hipError_t launch_pcg(const PcgArgs<T>& args, int tile, int max_blocks, hipStream_t s) {
  return dispatch_pcg<T, false>(args, PcgCols<T>{}, tile, max_blocks, s);
}

template <typename T>
hipError_t launch_pcg_ragged(const PcgArgs<T>& args, const PcgCols<T>& cols, int tile, hipStream_t s) {
  return dispatch_pcg<T, true>(args, cols, tile, 0, s);
}

template hipError_t launch_pcg_ragged<double>(const PcgArgs<double>&, const PcgCols<double>&, int, hipStream_t);
template hipError_t launch_pcg_ragged<float>(const PcgArgs<float>&, const PcgCols<float>&, int, hipStream_t);
template hipError_t launch_pcg<double>(const PcgArgs<double>&, int, int, hipStream_t);
template hipError_t launch_pcg<float>(const PcgArgs<float>&, int, int, hipStream_t);

}  // namespace sgk
