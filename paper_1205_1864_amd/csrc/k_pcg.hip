// Persistent batched PCG for the diagonal-block solves of Algorithm 1
// (Section 5: independent inner Krylov loops on blocks equal to the mean
// matrix K_0 = theta0 * K_Lap). One cooperative launch runs every column of
// a batch to convergence with per-column masks.
//
// Preconditioner: d updates of the Chebyshev iteration for
// (D^-1 K_0) z = D^-1 r from z = 0 (D = diag K_0 = theta0 * 8/3), i.e.
// z = p(D^-1 K_0) D^-1 r for a fixed polynomial. Its d - 1 stencil sweeps
// are done in LDS on a tile grown by a halo of d - 1 nodes, so a
// preconditioner application reads r and q once and writes z once.
//
// Per PCG iteration the grid passes two barriers:
//   phase A: p = z + beta p (on the tile plus a 1-node halo), q = K_0 p,
//            partial p.q;
//   phase B: alpha = gamma / p.q, x += alpha p, r -= alpha q (on the tile
//            plus the Chebyshev halo), z = M r, partials r.r and r.z.
// Per-column scalars are reduced from per-tile partials in a fixed order by
// every block that needs them, so all blocks agree bit for bit. p and r are
// double-buffered so halo reads never race with neighbouring tiles.
#include "sg_internal.h"

namespace sgk {

namespace {

constexpr int kThreads = 256;

enum { PART_BB = 0, PART_PQ = 1, PART_RR0 = 2, PART_RR1 = 3, PART_RZ0 = 4, PART_RZ1 = 5, PART_N = 6 };

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the threads of a block in a fixed order; result valid in thread 0.
__device__ double block_sum(double v, double* sred) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < kThreads / 64; ++w) t += sred[w];
  }
  return t;
}

// Chebyshev preconditioner on one tile. `rreg(lx, ly)` gives r on the region
// (tile plus halo H = degree - 1; zero outside the domain). Writes z on the
// tile interior to zcol and returns this thread's partial r.z (interior).
template <typename T, int TS, typename RF>
__device__ double cheb_tile(const PcgArgs<T>& A, int x0, int y0, RF rreg, T* zcol, T* sW0, T* sW1, T* sS,
                            T* sZ, T* sR) {
  const int H = A.degree - 1;
  const int RS = TS + 2 * H;
  const int nreg = RS * RS;
  // step 0: S = D^-1 r, W = S / theta, Z = W
  for (int i = threadIdx.x; i < nreg; i += kThreads) {
    const int lx = i % RS, ly = i / RS;
    const int gx = x0 - H + lx, gy = y0 - H + ly;
    const bool in = gx >= 0 && gx < A.nx && gy >= 0 && gy < A.nx;
    const T r = in ? rreg(lx, ly) : T(0);
    const T s = r * A.inv_diag;
    const T w = s * A.inv_theta;
    sS[i] = s;
    sW0[i] = w;
    if (lx >= H && lx < H + TS && ly >= H && ly < H + TS) {
      const int j = (ly - H) * TS + (lx - H);
      sZ[j] = w;
      sR[j] = r;
    }
  }
  T* cur = sW0;
  T* nxt = sW1;
  for (int j = 1; j < A.degree; ++j) {
    __syncthreads();
    const T ca = A.chebA[j], cb = A.chebB[j];
    const int lo = j, hi = RS - j;  // W_j is valid on [j, RS - j)
    const int w = hi - lo;
    for (int i = threadIdx.x; i < w * w; i += kThreads) {
      const int lx = lo + i % w, ly = lo + i / w;
      const int gx = x0 - H + lx, gy = y0 - H + ly;
      const int k = ly * RS + lx;
      T wn = T(0);
      if (gx >= 0 && gx < A.nx && gy >= 0 && gy < A.nx) {
        const T s8 = cur[k - RS - 1] + cur[k - RS] + cur[k - RS + 1] + cur[k - 1] + cur[k + 1] +
                     cur[k + RS - 1] + cur[k + RS] + cur[k + RS + 1];
        const T s = sS[k] - (cur[k] - T(0.125) * s8);
        sS[k] = s;
        wn = ca * cur[k] + cb * s;
      }
      nxt[k] = wn;
      if (lx >= H && lx < H + TS && ly >= H && ly < H + TS) sZ[(ly - H) * TS + (lx - H)] += wn;
    }
    T* t = cur;
    cur = nxt;
    nxt = t;
  }
  __syncthreads();
  double rz = 0.0;
  for (int i = threadIdx.x; i < TS * TS; i += kThreads) {
    const int lx = i % TS, ly = i / TS;
    const int gx = x0 + lx, gy = y0 + ly;
    if (gx < A.nx && gy < A.nx) {
      const T z = sZ[i];
      zcol[(long)gy * A.nx + gx] = z;
      rz += (double)sR[i] * (double)z;
    }
  }
  return rz;
}

constexpr int kMaxColsPerBlock = 64;
constexpr long kSpinLimit = 1L << 26;  // bounded waits: a stuck column aborts the launch

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

template <typename T, int TS>
__global__ void __launch_bounds__(kThreads) pcg_kernel(const PcgArgs<T> A) {
  // LDS: two W buffers and S over the grown tile; Z and R over the tile.
  extern __shared__ unsigned char smem_raw[];
  T* sW0 = reinterpret_cast<T*>(smem_raw);
  const int H = A.degree - 1;
  const int RSa = TS + 2 * (H > 1 ? H : 1);  // phase A needs a 1-node halo
  const int CAP = RSa * RSa;
  T* sW1 = sW0 + CAP;
  T* sS = sW1 + CAP;
  T* sZ = sS + CAP;
  T* sR = sZ + TS * TS;
  __shared__ double sred[kThreads / 64];
  __shared__ double s4[4];
  __shared__ int sdone[kMaxColsPerBlock + 2];  // a run of < kMaxColsPerBlock * ntiles tiles spans at most kMaxColsPerBlock + 1 columns
  __shared__ int sflag;

  const long n = A.n;
  const int ntiles = A.ntiles;
  const int ncols = A.ncols;
  const long nwork = (long)ncols * ntiles;
  double* part = A.sc.part;
  unsigned* arr = A.sc.arrivals;
  auto P = [&](int which) { return part + (long)which * ncols * ntiles; };
  // Each block owns a contiguous run of work items (tiles); columns progress
  // independently, synchronised only among the blocks that share them.
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
  for (int c = c_first + (int)threadIdx.x; c <= c_last; c += kThreads) sdone[c - c_first] = 0;

  // ---- start (column phase 1): x = 0, z = M b, partials b.b and b.z
  for (int c = c_first; c <= c_last; ++c) {
    int t0, t1;
    tiles_of(c, t0, t1);
    for (int t = t0; t < t1; ++t) {
      __syncthreads();
      const int x0 = (t % A.ntx) * TS, y0 = (t / A.ntx) * TS;
      const T* bcol = A.B + (long)c * n;
      auto rreg = [&](int lx, int ly) { return bcol[(long)(y0 - H + ly) * A.nx + (x0 - H + lx)]; };
      double rz = cheb_tile<T, TS>(A, x0, y0, rreg, A.Z + (long)c * n, sW0, sW1, sS, sZ, sR);
      double bb = 0.0;
      T* xcol = A.X + (long)c * n;
      for (int i = threadIdx.x; i < TS * TS; i += kThreads) {
        const int gx = x0 + i % TS, gy = y0 + i / TS;
        if (gx < A.nx && gy < A.nx) {
          const double b = (double)sR[i];
          bb += b * b;
          xcol[(long)gy * A.nx + gx] = T(0);
        }
      }
      rz = block_sum(rz, sred);
      bb = block_sum(bb, sred);
      if (threadIdx.x == 0) {
        P(PART_RZ1)[(long)c * ntiles + t] = rz;
        P(PART_BB)[(long)c * ntiles + t] = bb;
      }
    }
    column_arrive(arr + c, (unsigned)(t1 - t0));
  }

  bool aborted = false;
  int it = 0;
  for (; it < A.maxit && !aborted; ++it) {
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
      for (int t = t0; t < t1; ++t) {
        const int x0 = (t % A.ntx) * TS, y0 = (t / A.ntx) * TS;
        const int RS1 = TS + 2;
        T* sP = sW0;
        __syncthreads();
        for (int i = threadIdx.x; i < RS1 * RS1; i += kThreads) {
          const int gx = x0 - 1 + i % RS1, gy = y0 - 1 + i / RS1;
          T v = T(0);
          if (gx >= 0 && gx < A.nx && gy >= 0 && gy < A.nx) {
            const long g = (long)gy * A.nx + gx;
            v = it == 0 ? zc[g] : zc[g] + beta * po[g];
          }
          sP[i] = v;
        }
        __syncthreads();
        double pq = 0.0;
        for (int i = threadIdx.x; i < TS * TS; i += kThreads) {
          const int lx = i % TS + 1, ly = i / TS + 1;
          const int gx = x0 + lx - 1, gy = y0 + ly - 1;
          if (gx < A.nx && gy < A.nx) {
            const int k = ly * RS1 + lx;
            const T pc = sP[k];
            const T s8 = sP[k - RS1 - 1] + sP[k - RS1] + sP[k - RS1 + 1] + sP[k - 1] + sP[k + 1] +
                         sP[k + RS1 - 1] + sP[k + RS1] + sP[k + RS1 + 1];
            const T q = A.c0 * pc + A.c1 * s8;
            const long g = (long)gy * A.nx + gx;
            pn[g] = pc;
            qc[g] = q;
            pq += (double)pc * (double)q;
          }
        }
        pq = block_sum(pq, sred);
        if (threadIdx.x == 0) P(PART_PQ)[(long)c * ntiles + t] = pq;
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
      for (int t = t0; t < t1; ++t) {
        const int x0 = (t % A.ntx) * TS, y0 = (t / A.ntx) * TS;
        __syncthreads();
        for (int i = threadIdx.x; i < TS * TS; i += kThreads) {
          const int gx = x0 + i % TS, gy = y0 + i / TS;
          if (gx < A.nx && gy < A.nx) {
            const long g = (long)gy * A.nx + gx;
            xc[g] = it == 0 ? alpha * pc[g] : xc[g] + alpha * pc[g];
          }
        }
        auto rreg = [&](int lx, int ly) {
          const long g = (long)(y0 - H + ly) * A.nx + (x0 - H + lx);
          return ro[g] - alpha * qc[g];
        };
        double rz = cheb_tile<T, TS>(A, x0, y0, rreg, A.Z + (long)c * n, sW0, sW1, sS, sZ, sR);
        double rr = 0.0;
        for (int i = threadIdx.x; i < TS * TS; i += kThreads) {
          const int gx = x0 + i % TS, gy = y0 + i / TS;
          if (gx < A.nx && gy < A.nx) {
            const T r = sR[i];
            rn[(long)gy * A.nx + gx] = r;
            rr += (double)r * (double)r;
          }
        }
        rz = block_sum(rz, sred);
        rr = block_sum(rr, sred);
        if (threadIdx.x == 0) {
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

// Zero the per-column arrival counters before a launch.
__global__ void pcg_reset_kernel(unsigned* arr, int ncols, int* status) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncols; c += gridDim.x * blockDim.x) arr[c] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
}

template <typename T, int TS>
size_t smem_bytes(int degree) {
  const int H = degree - 1;
  const int RSa = TS + 2 * (H > 1 ? H : 1);
  return sizeof(T) * (3 * RSa * RSa + 2 * TS * TS);
}

template <typename T, int TS>
hipError_t launch_tile(const PcgArgs<T>& args, int max_blocks, hipStream_t s) {
  const size_t sm = smem_bytes<T, TS>(args.degree);
  auto kfn = pcg_kernel<T, TS>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kThreads, sm);
  if (e != hipSuccess) return e;
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int ncu = 0;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  long nwork = (long)args.ncols * args.ntiles;
  long grid = (long)per_cu * ncu;
  if (max_blocks > 0 && grid > max_blocks) grid = max_blocks;
  if (grid > nwork) grid = nwork;
  if (grid < 1) grid = 1;
  // every block must own at most kMaxColsPerBlock columns
  if ((nwork + grid - 1) / grid > (long)kMaxColsPerBlock * args.ntiles) return hipErrorInvalidValue;
  PcgArgs<T> a = args;
  hipLaunchKernelGGL(pcg_reset_kernel, dim3(1), dim3(256), 0, s, a.sc.arrivals, a.ncols, a.sc.status);
  void* kargs[] = {&a};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kfn), dim3((unsigned)grid), dim3(kThreads),
                                    kargs, (unsigned)sm, s);
}

}  // namespace

template <typename T>
hipError_t launch_pcg(const PcgArgs<T>& args, int tile, int max_blocks, hipStream_t s) {
  if (args.ncols <= 0) return hipSuccess;
  if (tile == 16) return launch_tile<T, 16>(args, max_blocks, s);
  return launch_tile<T, 32>(args, max_blocks, s);
}

template hipError_t launch_pcg<double>(const PcgArgs<double>&, int, int, hipStream_t);
template hipError_t launch_pcg<float>(const PcgArgs<float>&, int, int, hipStream_t);

}  // namespace sgk
