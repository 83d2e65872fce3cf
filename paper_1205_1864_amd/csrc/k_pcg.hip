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
#include <hip/hip_cooperative_groups.h>

#include "sg_internal.h"

namespace cg = cooperative_groups;

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

// Block-uniform read of a flag that another block may be writing concurrently.
__device__ int block_read(const int* p, int* sbi) {
  __syncthreads();
  if (threadIdx.x == 0) *sbi = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return *sbi;
}

// Column scalar: sum of the per-tile partials of column c, same order in every block.
__device__ double column_sum(const double* part, int c, int ntiles, double* sbc) {
  __syncthreads();
  if (threadIdx.x < 64) {
    double v = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += 64) v += part[(long)c * ntiles + t];
    v = wave_sum(v);
    if (threadIdx.x == 0) *sbc = v;
  }
  __syncthreads();
  return *sbc;
}

template <typename T, int TS>
struct Smem {
  static constexpr int RMAX = TS + 2 * (kMaxCheb - 1);
};

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

template <typename T, int TS>
__global__ void __launch_bounds__(kThreads) pcg_kernel(const PcgArgs<T> A) {
  constexpr int RMAX = Smem<T, TS>::RMAX;
  // LDS: two W buffers, S over the largest region; Z and R over the tile.
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
  __shared__ double sbc;
  __shared__ int sbi;
  (void)RMAX;

  cg::grid_group grid = cg::this_grid();
  const long n = A.n;
  const int ntiles = A.ntiles;
  const long nwork = (long)A.ncols * ntiles;
  double* part = A.sc.part;
  auto P = [&](int which) { return part + (long)which * A.ncols * ntiles; };

  // ---- init: z = M b, partials b.b and b.z (stored as the "iteration -1" r.z)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *A.sc.ndone = 0u;
    *A.sc.status = 0;
  }
  for (long w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int c = (int)(w / ntiles), t = (int)(w % ntiles);
    __syncthreads();
    const int x0 = (t % A.ntx) * TS, y0 = (t / A.ntx) * TS;
    const T* bcol = A.B + (long)c * n;
    auto rreg = [&](int lx, int ly) { return bcol[(long)(y0 - H + ly) * A.nx + (x0 - H + lx)]; };
    double rz = cheb_tile<T, TS>(A, x0, y0, rreg, A.Z + (long)c * n, sW0, sW1, sS, sZ, sR);
    double bb = 0.0;
    for (int i = threadIdx.x; i < TS * TS; i += kThreads) {
      const int gx = x0 + i % TS, gy = y0 + i / TS;
      if (gx < A.nx && gy < A.nx) {
        const double b = (double)sR[i];
        bb += b * b;
      }
    }
    T* xcol = A.X + (long)c * n;
    for (int i = threadIdx.x; i < TS * TS; i += kThreads) {
      const int gx = x0 + i % TS, gy = y0 + i / TS;
      if (gx < A.nx && gy < A.nx) xcol[(long)gy * A.nx + gx] = T(0);
    }
    rz = block_sum(rz, sred);
    bb = block_sum(bb, sred);
    if (threadIdx.x == 0) {
      P(PART_RZ1)[(long)c * ntiles + t] = rz;
      P(PART_BB)[(long)c * ntiles + t] = bb;
      if (t == 0) A.sc.done_at[c] = -1;
    }
  }
  grid.sync();

  for (int it = 0; it < A.maxit; ++it) {
    const int par = it & 1;
    T* Pnew = par ? A.P1 : A.P0;
    const T* Pold = par ? A.P0 : A.P1;
    // ---- phase A
    // Column state done_at[c]: -1 active, >= 0 finished at that iteration,
    // <= -2 broke down in phase B of iteration -(state + 2) (counted here).
    for (long w = blockIdx.x; w < nwork; w += gridDim.x) {
      const int c = (int)(w / ntiles), t = (int)(w % ntiles);
      const int state = block_read(A.sc.done_at + c, &sbi);
      if (state >= 0) continue;
      if (state <= -2) {
        if (threadIdx.x == 0 && t == 0) {
          A.sc.done_at[c] = -(state + 2);
          atomicAdd(A.sc.ndone, 1u);
        }
        continue;
      }
      const int x0 = (t % A.ntx) * TS, y0 = (t / A.ntx) * TS;
      const double bb = column_sum(P(PART_BB), c, ntiles, &sbc);
      const double rr = it == 0 ? bb : column_sum(P(par ? PART_RR0 : PART_RR1), c, ntiles, &sbc);
      if (sqrt(rr) <= A.rtol * sqrt(bb)) {
        if (threadIdx.x == 0 && t == 0) {
          A.sc.done_at[c] = it;
          atomicAdd(A.sc.ndone, 1u);
        }
        continue;
      }
      T beta = T(0);
      if (it > 0) {
        const double gnew = column_sum(P(par ? PART_RZ0 : PART_RZ1), c, ntiles, &sbc);
        const double gold = column_sum(P(par ? PART_RZ1 : PART_RZ0), c, ntiles, &sbc);
        beta = (T)(gnew / gold);
      }
      const T* zc = A.Z + (long)c * n;
      const T* po = Pold + (long)c * n;
      T* pn = Pnew + (long)c * n;
      T* qc = A.Q + (long)c * n;
      const int RS1 = TS + 2;
      T* sP = sW0;
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
    grid.sync();
    if (__hip_atomic_load(A.sc.ndone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (unsigned)A.ncols) break;
    // ---- phase B
    T* Rnew = par ? A.R0 : A.R1;
    const T* Rold = it == 0 ? A.B : (par ? A.R1 : A.R0);
    for (long w = blockIdx.x; w < nwork; w += gridDim.x) {
      const int c = (int)(w / ntiles), t = (int)(w % ntiles);
      if (block_read(A.sc.done_at + c, &sbi) != -1) continue;
      const int x0 = (t % A.ntx) * TS, y0 = (t / A.ntx) * TS;
      const double pq = column_sum(P(PART_PQ), c, ntiles, &sbc);
      if (!(pq > 0.0) || !isfinite(pq)) {
        // breakdown of this column: keep its current iterate; counted in the next phase A
        if (threadIdx.x == 0 && t == 0) A.sc.done_at[c] = -2 - it;
        continue;
      }
      const double gam = column_sum(P(par ? PART_RZ0 : PART_RZ1), c, ntiles, &sbc);
      const T alpha = (T)(gam / pq);
      const T* pc = Pnew + (long)c * n;
      const T* qc = A.Q + (long)c * n;
      const T* ro = Rold + (long)c * n;
      T* rn = Rnew + (long)c * n;
      T* xc = A.X + (long)c * n;
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
    grid.sync();
  }
  // ---- finalize iteration counts
  if (blockIdx.x == 0) {
    for (int c = threadIdx.x; c < A.ncols; c += kThreads) {
      const int d = A.sc.done_at[c];
      A.sc.iters[c] = d >= 0 ? d : (d <= -2 ? -(d + 2) : A.maxit);
    }
  }
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
  PcgArgs<T> a = args;
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
