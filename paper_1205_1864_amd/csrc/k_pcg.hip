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
#include "sg_internal.h"

namespace sgk {

namespace {

constexpr int kGroup = 256;                // threads per tile group
constexpr int kMaxColsPerBlock = 64;
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
template <typename T, int TS, int NS, typename RF>
__device__ double cheb_tile(const PcgArgs<T>& A, bool valid, int x0, int y0, RF rreg, T* W0, T* W1,
                            T (&Zi)[Interior<TS>::NI], T (&Ri)[Interior<TS>::NI]) {
  constexpr int NI = Interior<TS>::NI;
  const int lt = threadIdx.x % kGroup;
  const int H = A.degree - 1;
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
  for (int j = 1; j < A.degree; ++j) {
    __syncthreads();  // reads of the buffer about to be overwritten are done
    const T ca = A.chebA[j], cb = A.chebB[j];
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

template <typename T, int TS, int NS, int G>
__global__ void __launch_bounds__(kGroup* G) pcg_kernel(const PcgArgs<T> A) {
  constexpr int NI = Interior<TS>::NI;
  extern __shared__ unsigned char smem_raw[];
  const int grp = threadIdx.x / kGroup;
  const int lt = threadIdx.x % kGroup;
  const int H = A.degree - 1;
  const int RSa = TS + 2 * (H > 1 ? H : 1);  // phase A needs a 1-node halo
  const int CAP = RSa * RSa;
  T* W0 = reinterpret_cast<T*>(smem_raw) + (long)grp * 2 * CAP;
  T* W1 = W0 + CAP;
  __shared__ double sred[G][4];
  __shared__ double s4[4];
  __shared__ int sdone[kMaxColsPerBlock + 2];  // a run of <= kMaxColsPerBlock * ntiles tiles spans <= kMaxColsPerBlock + 1 columns
  __shared__ int sflag;

  const long n = A.n;
  const int ntiles = A.ntiles;
  const int ncols = A.ncols;
  const long nwork = (long)ncols * ntiles;
  double* part = A.sc.part;
  unsigned* arr = A.sc.arrivals;
  auto P = [&](int which) { return part + (long)which * ncols * ntiles; };
  const long per_block = (nwork + gridDim.x - 1) / gridDim.x;
  const long w_begin = (long)blockIdx.x * per_block;
  const long w_end = w_begin + per_block < nwork ? w_begin + per_block : nwork;
  if (w_begin >= w_end) return;
  const int c_first = (int)(w_begin / ntiles), c_last = (int)((w_end - 1) / ntiles);
  auto tiles_of = [&](int c, int& t0, int& t1) {
    const long lo = (long)c * ntiles > w_begin ? (long)c * ntiles : w_begin;
    const long hi = (long)(c + 1) * ntiles < w_end ? (long)(c + 1) * ntiles : w_end;
    t0 = (int)(lo - (long)c * ntiles);
    t1 = (int)(hi - (long)c * ntiles);
  };
  auto owner = [&](int c) { return (long)c * ntiles >= w_begin; };  // this block holds tile 0 of c
  // Fixed-order sums of up to four per-tile partial arrays of column c, one wave each.
  auto col_sums = [&](int c, const double* q0, const double* q1, const double* q2, const double* q3) {
    __syncthreads();
    const int wv = threadIdx.x >> 6;
    const double* src = wv == 0 ? q0 : wv == 1 ? q1 : wv == 2 ? q2 : q3;
    if (wv < 4 && src) {
      double v = 0.0;
      for (int t = threadIdx.x & 63; t < ntiles; t += 64) v += src[(long)c * ntiles + t];
      v = wave_sum(v);
      if ((threadIdx.x & 63) == 0) s4[wv] = v;
    }
    __syncthreads();
  };
  auto tile_xy = [&](int t, int& x0, int& y0) {
    x0 = (t % A.ntx) * TS;
    y0 = (t / A.ntx) * TS;
  };
  for (int c = c_first + (int)threadIdx.x; c <= c_last; c += kGroup * G) sdone[c - c_first] = 0;

  T Zi[NI], Ri[NI];

  // ---- start (column phase 1): x = 0, z = M b, partials b.b and b.z
  for (int c = c_first; c <= c_last; ++c) {
    int t0, t1;
    tiles_of(c, t0, t1);
    const T* bcol = A.B + (long)c * n;
    T* xcol = A.X + (long)c * n;
    T* zcol = A.Z + (long)c * n;
    for (int tb = t0; tb < t1; tb += G) {
      const int t = tb + grp;
      const bool valid = t < t1;
      int x0 = 0, y0 = 0;
      if (valid) tile_xy(t, x0, y0);
      __syncthreads();
      auto rreg = [&](int lx, int ly) { return bcol[(long)(y0 - H + ly) * A.nx + (x0 - H + lx)]; };
      double rz = cheb_tile<T, TS, NS>(A, valid, x0, y0, rreg, W0, W1, Zi, Ri);
      double bb = 0.0;
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const int i = lt + k * kGroup;
        const int gx = x0 + i % TS, gy = y0 + i / TS;
        if (valid && i < TS * TS && gx < A.nx && gy < A.nx) {
          const long g = (long)gy * A.nx + gx;
          bb += (double)Ri[k] * (double)Ri[k];
          xcol[g] = T(0);
          zcol[g] = Zi[k];
        }
      }
      rz = group_sum<G>(rz, sred);
      bb = group_sum<G>(bb, sred);
      if (valid && lt == 0) {
        P(PART_RZ1)[(long)c * ntiles + t] = rz;
        P(PART_BB)[(long)c * ntiles + t] = bb;
      }
    }
    column_arrive(arr + c, (unsigned)(t1 - t0));
  }

  bool aborted = false;
  for (int it = 0; it < A.maxit && !aborted; ++it) {
    const int par = it & 1;
    T* Pnew = par ? A.P1 : A.P0;
    const T* Pold = par ? A.P0 : A.P1;
    bool any_active = false;
    // ---- phase A (column phase 2 + 2 it): p = z + beta p, q = K_0 p, partial p.q
    for (int c = c_first; c <= c_last && !aborted; ++c) {
      if (sdone[c - c_first]) continue;
      if (!column_wait(arr + c, (unsigned)((1 + 2 * it) * ntiles), A.sc.status, &sflag)) {
        aborted = true;
        break;
      }
      col_sums(c, P(PART_BB), it == 0 ? nullptr : P(par ? PART_RR0 : PART_RR1),
               it == 0 ? nullptr : P(par ? PART_RZ0 : PART_RZ1), it == 0 ? nullptr : P(par ? PART_RZ1 : PART_RZ0));
      const double bb = s4[0];
      const double rr = it == 0 ? s4[0] : s4[1];
      if (sqrt(rr) <= A.rtol * sqrt(bb)) {
        __syncthreads();
        if (threadIdx.x == 0) {
          sdone[c - c_first] = 1;
          if (owner(c)) A.sc.iters[c] = it;
        }
        __syncthreads();
        continue;
      }
      const T beta = it == 0 ? T(0) : (T)(s4[2] / s4[3]);
      any_active = true;
      int t0, t1;
      tiles_of(c, t0, t1);
      const T* zc = A.Z + (long)c * n;
      const T* po = Pold + (long)c * n;
      T* pn = Pnew + (long)c * n;
      T* qc = A.Q + (long)c * n;
      const int RS1 = TS + 2;
      for (int tb = t0; tb < t1; tb += G) {
        const int t = tb + grp;
        const bool valid = t < t1;
        int x0 = 0, y0 = 0;
        if (valid) tile_xy(t, x0, y0);
        __syncthreads();
        if (valid) {
          for (int i = lt; i < RS1 * RS1; i += kGroup) {
            const int gx = x0 - 1 + i % RS1, gy = y0 - 1 + i / RS1;
            T v = T(0);
            if (gx >= 0 && gx < A.nx && gy >= 0 && gy < A.nx) {
              const long g = (long)gy * A.nx + gx;
              v = it == 0 ? zc[g] : zc[g] + beta * po[g];
            }
            W0[i] = v;
          }
        }
        __syncthreads();
        double pq = 0.0;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
          const int i = lt + k * kGroup;
          const int lx = i % TS + 1, ly = i / TS + 1;
          const int gx = x0 + lx - 1, gy = y0 + ly - 1;
          if (valid && i < TS * TS && gx < A.nx && gy < A.nx) {
            const int q = ly * RS1 + lx;
            const T pc = W0[q];
            const T s8 = W0[q - RS1 - 1] + W0[q - RS1] + W0[q - RS1 + 1] + W0[q - 1] + W0[q + 1] +
                         W0[q + RS1 - 1] + W0[q + RS1] + W0[q + RS1 + 1];
            const T qv = A.c0 * pc + A.c1 * s8;
            const long g = (long)gy * A.nx + gx;
            pn[g] = pc;
            qc[g] = qv;
            pq += (double)pc * (double)qv;
          }
        }
        pq = group_sum<G>(pq, sred);
        if (valid && lt == 0) P(PART_PQ)[(long)c * ntiles + t] = pq;
      }
      column_arrive(arr + c, (unsigned)(t1 - t0));
    }
    if (!any_active || aborted) break;
    // ---- phase B (column phase 3 + 2 it): x += alpha p, r -= alpha q, z = M r, partials r.r, r.z
    T* Rnew = par ? A.R0 : A.R1;
    const T* Rold = it == 0 ? A.B : (par ? A.R1 : A.R0);
    for (int c = c_first; c <= c_last && !aborted; ++c) {
      if (sdone[c - c_first]) continue;
      if (!column_wait(arr + c, (unsigned)((2 + 2 * it) * ntiles), A.sc.status, &sflag)) {
        aborted = true;
        break;
      }
      col_sums(c, P(PART_PQ), P(par ? PART_RZ0 : PART_RZ1), nullptr, nullptr);
      const double pq = s4[0], gam = s4[1];
      if (!(pq > 0.0) || !isfinite(pq)) {
        // breakdown: keep the current iterate
        __syncthreads();
        if (threadIdx.x == 0) {
          sdone[c - c_first] = 1;
          if (owner(c)) A.sc.iters[c] = it;
        }
        __syncthreads();
        continue;
      }
      const T alpha = (T)(gam / pq);
      int t0, t1;
      tiles_of(c, t0, t1);
      const T* pc = Pnew + (long)c * n;
      const T* qc = A.Q + (long)c * n;
      const T* ro = Rold + (long)c * n;
      T* rn = Rnew + (long)c * n;
      T* xc = A.X + (long)c * n;
      T* zc = A.Z + (long)c * n;
      for (int tb = t0; tb < t1; tb += G) {
        const int t = tb + grp;
        const bool valid = t < t1;
        int x0 = 0, y0 = 0;
        if (valid) tile_xy(t, x0, y0);
        __syncthreads();
        auto rreg = [&](int lx, int ly) {
          const long g = (long)(y0 - H + ly) * A.nx + (x0 - H + lx);
          return ro[g] - alpha * qc[g];
        };
        double rz = cheb_tile<T, TS, NS>(A, valid, x0, y0, rreg, W0, W1, Zi, Ri);
        double rr = 0.0;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
          const int i = lt + k * kGroup;
          const int gx = x0 + i % TS, gy = y0 + i / TS;
          if (valid && i < TS * TS && gx < A.nx && gy < A.nx) {
            const long g = (long)gy * A.nx + gx;
            xc[g] = it == 0 ? alpha * pc[g] : xc[g] + alpha * pc[g];
            rn[g] = Ri[k];
            zc[g] = Zi[k];
            rr += (double)Ri[k] * (double)Ri[k];
          }
        }
        rz = group_sum<G>(rz, sred);
        rr = group_sum<G>(rr, sred);
        if (valid && lt == 0) {
          P(par ? PART_RZ1 : PART_RZ0)[(long)c * ntiles + t] = rz;
          P(par ? PART_RR1 : PART_RR0)[(long)c * ntiles + t] = rr;
        }
      }
      column_arrive(arr + c, (unsigned)(t1 - t0));
    }
  }
  // ---- iteration counts of columns that ran out of iterations
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = c_first; c <= c_last; ++c)
      if (!sdone[c - c_first] && owner(c)) A.sc.iters[c] = A.maxit;
  }
}

// Zero the per-column arrival counters and the status word before a launch.
__global__ void pcg_reset_kernel(unsigned* arr, int ncols, int* status) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncols; c += gridDim.x * blockDim.x) arr[c] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
}

template <typename T, int TS, int NS, int G>
hipError_t launch_cfg(const PcgArgs<T>& args, int max_blocks, hipStream_t s) {
  const int H = args.degree - 1;
  const int RSa = TS + 2 * (H > 1 ? H : 1);
  if ((TS + 2 * H) * (TS + 2 * H) > NS * kGroup) return hipErrorInvalidValue;
  const size_t sm = sizeof(T) * 2 * (size_t)RSa * RSa * G;
  auto kfn = pcg_kernel<T, TS, NS, G>;
  hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (ea != hipSuccess) return ea;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kGroup * G, sm);
  if (e != hipSuccess) return e;
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int ncu = 0;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const long nwork = (long)args.ncols * args.ntiles;
  // Enough blocks to keep every tile group busy, as few as possible beyond
  // that: every block pays a device-wide release per column and phase.
  long grid = (nwork + 2L * G - 1) / (2L * G);
  const long cap = (long)per_cu * ncu;
  if (grid > cap) grid = cap;
  if (max_blocks > 0 && grid > max_blocks) grid = max_blocks;
  if (grid < 1) grid = 1;
  if ((nwork + grid - 1) / grid > (long)kMaxColsPerBlock * args.ntiles) return hipErrorInvalidValue;
  PcgArgs<T> a = args;
  hipLaunchKernelGGL(pcg_reset_kernel, dim3(1), dim3(256), 0, s, a.sc.arrivals, a.ncols, a.sc.status);
  void* kargs[] = {&a};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kfn), dim3((unsigned)grid), dim3(kGroup * G),
                                    kargs, (unsigned)sm, s);
}

constexpr int slots(int ts, int maxh) { return ((ts + 2 * maxh) * (ts + 2 * maxh) + kGroup - 1) / kGroup; }

}  // namespace

template <typename T>
hipError_t launch_pcg(const PcgArgs<T>& args, int tile, int max_blocks, hipStream_t s) {
  if (args.ncols <= 0) return hipSuccess;
  const int H = args.degree - 1;
  if (tile == 32) {
    if (H <= 3) return launch_cfg<T, 32, slots(32, 3), 4>(args, max_blocks, s);
    if (H <= 7) return launch_cfg<T, 32, slots(32, 7), 2>(args, max_blocks, s);
  }
  return launch_cfg<T, 16, slots(16, 15), 4>(args, max_blocks, s);
}

template hipError_t launch_pcg<double>(const PcgArgs<double>&, int, int, hipStream_t);
template hipError_t launch_pcg<float>(const PcgArgs<float>&, int, int, hipStream_t);

}  // namespace sgk
