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
//   phase A: x += alpha' p' (the update of the previous iteration, deferred
//            so that it reuses the p that phase A reads anyway),
//            p = z + beta p' (tile plus a 1-node halo), q = K_0 p, partial p.q;
//   phase B: alpha = gamma / p.q, r -= alpha q (tile plus the Chebyshev
//            halo), z = M r, partials r.r and r.z.
// A column that stops (converged, or out of iterations) applies the pending
// x update to its tiles first. A launch may start every column from the
// contents of X (warm start, banded tiles): the start phase then forms
// r = b - K_0 x on the region grown by one more node.
// A column is split into tiles; each block owns a contiguous run of tiles (the
// same tiles in every phase) and works on G tiles at a time, one per group of
// waves; the waves of a group synchronise among themselves only.
// Columns synchronise only among the blocks that share them, through
// split-phase counters (no grid-wide barrier). Per-column scalars are reduced
// from per-tile partials in a fixed order, identically in every block, so all
// owners of a column take the same decisions.
//
// Two tile shapes. Banded tiles (the default) are tsx x R nodes (R = 64, 128
// or 256 rows by precision and launch size) with tsx chosen so that the tile
// plus its halo is at most 64 columns wide: each lane owns one column of the
// region and each wave one band of its rows, the horizontal stencil
// neighbours come from the neighbouring lanes (DPP) and the vertical ones from
// the wave's own registers (rows just outside its band through a small LDS
// exchange).
// Square 16 x 16 tiles serve Chebyshev degrees whose halo is too wide for that.
//
// The same kernel runs a ragged set of columns from several problems (grids
// of different sizes, own constants, a per-problem skip flag): the tiles of
// all columns form one work list and every column keeps its own arithmetic,
// so a column's iterates do not depend on what else is in the launch.
#include "sg_internal.h"
#include "sg_device.h"

namespace sgk {

namespace {

constexpr int kSquareGroup = 256;          // threads per group of the square tiles
constexpr long kSpinLimit = 1L << 26;      // bounded waits: a stuck column aborts the launch

// Per-tile partial sums: b.b, p.q of even / odd iterations, r.r and r.z of
// even / odd iterations.
enum { PART_BB = 0, PART_PQ0 = 1, PART_PQ1 = 2, PART_RR0 = 3, PART_RR1 = 4, PART_RZ0 = 5, PART_RZ1 = 6, PART_N = 7 };
static_assert(PART_N == kPcgPartials, "partial arrays of the inner solver");

// DPP move of a double within rows of 16 lanes (every source lane exists).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_f64(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum over the 64 lanes of a wave, the same in every lane and in a fixed
// order: butterflies within rows of 16 lanes (neighbour in the quad, the
// other pair of the quad, the other quad of each 8, the other 8 of each 16;
// both partners add the same two values), then the four row sums in order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Split-phase barrier of one column: every block that owns tiles of the column
// adds its tile count to a monotonic arrival counter after finishing its tiles;
// phase k of the column is complete once the counter reaches k * ntiles. The
// arrival releases the block's writes (device scope) and the wait acquires
// them: one L2 write-back per arrival, one invalidation per wait. Every wave
// first waits for its own stores: the barrier does not, and thread 0's
// release (the write-back) covers only stores that have reached the L2.
// A column whose tiles all belong to one block needs neither: its phases are
// ordered by the block's own barriers (see pcg_kernel).
__device__ void column_arrive(unsigned* arr, unsigned count) {
  __builtin_amdgcn_s_waitcnt(0);  // every counter at zero: the wave's stores are done
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    // The write-back the fence issues must be complete before the arrival
    // can be seen. The compiler's own wait after it is dropped when the wave
    // has no other memory operation outstanding, so it is stated here.
    __builtin_amdgcn_s_waitcnt(0);
    __hip_atomic_fetch_add(arr, count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// End of a column phase whose tiles all belong to this block: the block's
// global stores of the phase (vectors and tile partials) are complete before
// any wave goes on to read them. A barrier alone orders only the LDS.
__device__ __forceinline__ void column_end_whole() {
  __builtin_amdgcn_s_waitcnt(0);  // every counter at zero: the wave's stores are done
  __syncthreads();
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
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *sflag = ok;
  }
  __syncthreads();
  return *sflag != 0;
}

// Completes the loads of the given registers here (an empty asm that reads
// them). Vector loads and stores share one in-order counter, so a load
// consumed after later stores would otherwise also wait for those stores.
template <typename T, int N>
__device__ __forceinline__ void ready(const T (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) asm volatile("" ::"v"(v[i]));
}

// Index of this wave within its tile group (uniform, so that values derived
// from it stay in scalar registers).
template <int GT>
__device__ __forceinline__ int wave_in_group() {
  return __builtin_amdgcn_readfirstlane((threadIdx.x % GT) >> 6);
}

// Barrier of the waves of one tile group, so the groups of a block do not run
// in lockstep (one group loads its next tile while another sweeps).
// `bar` is the group's monotonic arrival counter in LDS; `gen` counts the
// arrivals this wave has waited for so far (the same in every wave of the
// group). A wait that does not end within the spin limit sets the status word
// and returns, so a wrong barrier count ends the launch with an error instead
// of a hang.
struct GroupBarrier {
  unsigned* bar;
  unsigned gen;
  unsigned waves;  // waves of the group
  int* status;
  bool dead;   // a wait ran out: later barriers of this wave no longer wait
  bool block;  // the group is the whole block: use the hardware barrier
};

__device__ __forceinline__ void group_sync(GroupBarrier& gb) {
  if (gb.block) {
    __syncthreads();
    return;
  }
  gb.gen += gb.waves;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if ((threadIdx.x & 63) == 0) __hip_atomic_fetch_add(gb.bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  long spins = 0;
  while (!gb.dead && __hip_atomic_load(gb.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < gb.gen) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      if ((threadIdx.x & 63) == 0) atomicExch(gb.status, 1);
      gb.dead = true;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Per-group sums of two values per thread, fixed order; the results are
// returned to every thread of the group. Only the group's threads take part.
template <int GT>
__device__ void group_sum2(double& a, double& b, double (*sred)[GT / 64][2], GroupBarrier& gb) {
  constexpr int NW = GT / 64;
  a = wave_sum(a);
  b = wave_sum(b);
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.x / GT), wv = wave_in_group<GT>();
  group_sync(gb);  // earlier readers of sred[g] are done
  if ((threadIdx.x & 63) == 0) {
    sred[g][wv][0] = a;
    sred[g][wv][1] = b;
  }
  group_sync(gb);
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    sa += sred[g][w][0];
    sb += sred[g][w][1];
  }
  a = sa;
  b = sb;
}

// K_0 v at a node from its column sums: cm, c, cp are v at the node below,
// the node and the node above (one lane per grid column); the horizontal
// neighbours come from the adjacent lanes. c0, c1: centre and neighbour
// weights of K_0. Every product with K_0 of the banded tiles uses this one
// expression, so a value computed twice is the same bit for bit.
template <typename T>
__device__ __forceinline__ T k0_apply(T cm, T c, T cp, T c0, T c1) {
  const T col = (cm + c) + cp;
  const T s8 = (from_prev(col) + from_next(col)) + (cm + cp);
  return c0 * c + c1 * s8;
}

// The grid, state vectors and constants of one column.
template <typename T>
struct ColView {
  int nx, ntx, ntiles, tsx;  // tsx: interior width of an inner banded tile
  int ta;                    // interior width of a banded tile at the grid's left or right edge
  long tbase;  // first index of the column's per-tile partials (and of its work items)
  const T* b;
  T *x, *r0, *r1, *p0, *p1, *q, *z;
  T c0, c1, inv_diag, inv_theta, w8;
  const T* chebA;
  const T* chebB;
};

// Vectors of one PCG iteration as seen by the tile routines.
template <typename T>
struct IterVecs {
  const T* po;  // p of the previous iteration (phase A)
  T* pn;        // p of this iteration
  const T* ro;  // r of the previous iteration (phase B)
  T* rn;        // r of this iteration
  T beta;       // phase A: p = z + beta p (first iteration: p = z)
  T alpha_prev; // phase A: x += alpha_prev po (not in the first iteration)
  T alpha;      // phase B: r -= alpha q
  bool first;
};

// ---------------------------------------------------------------------------
// Square TS x TS tiles: region (tile plus halo) nodes are spread over the
// group's threads in row-major order, NS nodes per thread.
// ---------------------------------------------------------------------------
template <typename T, int TS, int NS>
struct SquareTile {
  static constexpr int kThreads = kSquareGroup;
  static constexpr bool kParkedSums = false;  // tile sums through group_sum2
  __device__ static int ntiles_a(const ColView<T>& v) { return v.ntiles; }  // phase A on the same tiles
  // phase A stores q = K_0 p and phase B reads it
  static constexpr int NI = (TS * TS + kThreads - 1) / kThreads;  // interior nodes per thread
  // elements of T in one group's LDS buffers (two buffers; phase A needs a 1-node halo)
  static int lds_group(int degree) {
    const int h = degree - 1 > 1 ? degree - 1 : 1;
    return 2 * (TS + 2 * h) * (TS + 2 * h);
  }
  static bool fits(int degree, int nx, int ntx, int ntiles) {
    const int H = degree - 1;
    return (TS + 2 * H) * (TS + 2 * H) <= NS * kThreads && ntx == (nx + TS - 1) / TS && ntiles == ntx * ntx;
  }
  __device__ static void origin(const ColView<T>& v, int t, int& x0, int& y0) {
    x0 = (t % v.ntx) * TS;
    y0 = (t / v.ntx) * TS;
  }

  // Chebyshev preconditioner on one tile. `rreg(s, gy * nx + gx)` gives r at
  // grid node (gx, gy) of the region (only called inside the grid). On return Zi holds z and
  // Ri holds r on this thread's interior nodes; returns the partial r.z.
  template <typename RF>
  __device__ static double cheb(const ColView<T>& A, int degree, int x0, int y0, RF rreg, T* W0, T* W1,
                                T (&Zi)[NI], T (&Ri)[NI], GroupBarrier& gb) {
    const int lt = threadIdx.x % kThreads;
    const int H = degree - 1;
    const int RS = TS + 2 * H;
    const int nreg = RS * RS;
    T S[NS];
    // step 0: S = D^-1 r, W = S / theta; r parked in W1 for the interior mapping
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = lt + s * kThreads;
      S[s] = T(0);
      if (i < nreg) {
        const int lx = i % RS, ly = i / RS;
        const int gx = x0 - H + lx, gy = y0 - H + ly;
        const T r = (gx >= 0 && gx < A.nx && gy >= 0 && gy < A.nx) ? rreg(s, (unsigned)(gy * A.nx + gx)) : T(0);
        S[s] = r * A.inv_diag;
        W0[i] = S[s] * A.inv_theta;
        W1[i] = r;
      }
    }
    group_sync(gb);
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int i = lt + k * kThreads;
      Zi[k] = T(0);
      Ri[k] = T(0);
      if (i < TS * TS) {
        const int j = (i / TS + H) * RS + (i % TS + H);
        Zi[k] = W0[j];
        Ri[k] = W1[j];
      }
    }
    T* cur = W0;
    T* nxt = W1;
    for (int j = 1; j < degree; ++j) {
      group_sync(gb);  // reads of the buffer about to be overwritten are done
      const T ca = ld_uniform(A.chebA, j), cb = ld_uniform(A.chebB, j);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int i = lt + s * kThreads;
        if (i < nreg) {
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
      group_sync(gb);
#pragma unroll
      for (int k = 0; k < NI; ++k) {
        const int i = lt + k * kThreads;
        if (i < TS * TS) Zi[k] += nxt[(i / TS + H) * RS + (i % TS + H)];
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

  __device__ static bool warm_fits(const ColView<T>&, int) { return false; }

  // Start of the iteration: x = 0, z = M b; partials b.z, b.b and r.r = b.b.
  __device__ static void start(const ColView<T>& v, int degree, int t, bool, T* W0, T* W1, GroupBarrier& gb,
                               double& rz, double& bb, double& rr) {
    const int lt = threadIdx.x % kThreads;
    const int nx = v.nx;
    int x0, y0;
    origin(v, t, x0, y0);
    T Zi[NI], Ri[NI];
    auto rreg = [&](int, unsigned o) { return v.b[o]; };
    rz = cheb(v, degree, x0, y0, rreg, W0, W1, Zi, Ri, gb);
    bb = 0.0;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int i = lt + k * kThreads;
      const int gx = x0 + i % TS, gy = y0 + i / TS;
      if (i < TS * TS && gx < nx && gy < nx) {
        const long g = (long)gy * nx + gx;
        bb += (double)Ri[k] * (double)Ri[k];
        v.x[g] = T(0);
        v.z[g] = Zi[k];
      }
    }
    rr = bb;
  }

  // Phase A: p = z + beta p on the tile plus a 1-node halo, q = K_0 p; partial p.q.
  __device__ static double phase_a(const ColView<T>& v, int t, const IterVecs<T>& I, T* W0, GroupBarrier& gb) {
    const int lt = threadIdx.x % kThreads;
    const int nx = v.nx;
    constexpr int RS1 = TS + 2;
    int x0, y0;
    origin(v, t, x0, y0);
    for (int i = lt; i < RS1 * RS1; i += kThreads) {
      const int gx = x0 - 1 + i % RS1, gy = y0 - 1 + i / RS1;
      T val = T(0);
      if (gx >= 0 && gx < nx && gy >= 0 && gy < nx) {
        const long g = (long)gy * nx + gx;
        val = I.first ? v.z[g] : v.z[g] + I.beta * I.po[g];
      }
      W0[i] = val;
    }
    group_sync(gb);
    double pq = 0.0;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int i = lt + k * kThreads;
      const int lx = i % TS + 1, ly = i / TS + 1;
      const int gx = x0 + lx - 1, gy = y0 + ly - 1;
      if (i < TS * TS && gx < nx && gy < nx) {
        const int q = ly * RS1 + lx;
        const T pc = W0[q];
        const T s8 = W0[q - RS1 - 1] + W0[q - RS1] + W0[q - RS1 + 1] + W0[q - 1] + W0[q + 1] + W0[q + RS1 - 1] +
                     W0[q + RS1] + W0[q + RS1 + 1];
        const T qv = v.c0 * pc + v.c1 * s8;
        const long g = (long)gy * nx + gx;
        if (!I.first) v.x[g] += I.alpha_prev * I.po[g];
        I.pn[g] = pc;
        v.q[g] = qv;
        pq += (double)pc * (double)qv;
      }
    }
    return pq;
  }

  // x += alpha p on the interior of a tile, the update a stopping column still
  // owes (zero: x = 0 instead).
  __device__ static void finalize(const ColView<T>& v, int t, T alpha, const T* p, bool zero) {
    const int lt = threadIdx.x % kThreads;
    const int nx = v.nx;
    int x0, y0;
    origin(v, t, x0, y0);
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int i = lt + k * kThreads;
      const int gx = x0 + i % TS, gy = y0 + i / TS;
      if (i < TS * TS && gx < nx && gy < nx) {
        const long g = (long)gy * nx + gx;
        if (zero) {
          v.x[g] = T(0);
        } else {
          v.x[g] += alpha * p[g];
        }
      }
    }
  }

  // Phase B: r -= alpha q, z = M r; partials r.z and r.r.
  __device__ static void phase_b(const ColView<T>& v, int degree, int t, const IterVecs<T>& I, T* W0, T* W1,
                                 GroupBarrier& gb, double& rz, double& rr) {
    const int lt = threadIdx.x % kThreads;
    const int nx = v.nx;
    int x0, y0;
    origin(v, t, x0, y0);
    T Zi[NI], Ri[NI];
    auto rreg = [&](int, unsigned o) { return I.ro[o] - I.alpha * v.q[o]; };
    rz = cheb(v, degree, x0, y0, rreg, W0, W1, Zi, Ri, gb);
    rr = 0.0;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int i = lt + k * kThreads;
      const int gx = x0 + i % TS, gy = y0 + i / TS;
      if (i < TS * TS && gx < nx && gy < nx) {
        const long g = (long)gy * nx + gx;
        I.rn[g] = Ri[k];
        v.z[g] = Zi[k];
        rr += (double)Ri[k] * (double)Ri[k];
      }
    }
  }

  __device__ static void run_a(const ColView<T>& v, int t_begin, int t_end, int step, const IterVecs<T>& I, T* W0,
                               GroupBarrier& gb, double (*sred)[kThreads / 64][2], double* part) {
    for (int t = t_begin; t < t_end; t += step) {
      double pq = phase_a(v, t, I, W0, gb), unused = 0.0;
      group_sum2<kThreads>(pq, unused, sred, gb);
      if ((threadIdx.x % kThreads) == 0) part[t] = pq;
    }
  }

  __device__ static void run_b(const ColView<T>& v, int degree, int t_begin, int t_end, int step,
                               const IterVecs<T>& I, T* W0, T* W1, GroupBarrier& gb,
                               double (*sred)[kThreads / 64][2], double* part_rz, double* part_rr) {
    for (int t = t_begin; t < t_end; t += step) {
      double rz, rr;
      phase_b(v, degree, t, I, W0, W1, gb, rz, rr);
      group_sum2<kThreads>(rz, rr, sred, gb);
      if ((threadIdx.x % kThreads) == 0) {
        part_rz[t] = rz;
        part_rr[t] = rr;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// Banded tiles: tsx x TSY nodes. The region (tile plus halo) has one column
// per lane (at most 64) and its rows are split into NW bands of BR rows, one
// per wave of the group. Each wave keeps its band in registers: a stencil
// update takes the horizontal neighbours from the adjacent lanes (DPP), the
// rows above and below from the wave's own registers, and only the rows just
// outside the band from the neighbouring waves, through a small LDS exchange
// area (two rows per wave, two buffers used alternately). r on the interior
// of the tile waits in LDS while the Chebyshev sweeps run.
// ---------------------------------------------------------------------------
template <typename T, int TSY, int HMAX, int NW>
struct BandTile {
  static constexpr int kThreads = 64 * NW;
  static constexpr bool kParkedSums = true;  // tile sums: see TileSums
  // phase B recomputes q = K_0 p from p instead of reading a stored q
  static constexpr int RYMAX = TSY + 2 * HMAX;
  static constexpr int BR = (RYMAX + NW - 1) / NW;     // region rows per wave (Chebyshev)
  static constexpr int BRA = (TSY + 2 + NW - 1) / NW;  // region rows per wave (phase A, halo 1)
  static constexpr int RB = NW * BR;                   // region rows covered by the bands
  static constexpr int kEx = 2 * NW * 2 * 64;          // exchange area: 2 buffers x NW waves x 2 rows
  // the next tile's inputs are loaded during the current one, except where two
  // copies of them do not fit the registers (bands taller than 64 rows)
  static constexpr bool kPrefetch = TSY <= 64;
  // phase B takes the part of the next tile's region that overlaps the
  // current one from the current tile's registers (load_b_next); measured
  // faster in FP32 (one lane shuffle per value), not in FP64 (two)
  static constexpr bool kReuseHalo = sizeof(T) == 4;
  static_assert(NW * BRA <= RB, "phase A rows exceed the bands");
  static_assert(TSY + 2 * (HMAX + 1) <= RB, "phase B needs the Chebyshev halo plus one row");
  // elements of T per group: the exchange area, then r of the region rows
  static int lds_group(int) { return kEx + RB * 64; }

  // Band-edge exchange of an N-row band partition: the row above the band
  // (last row of the wave before) and the row below it (first row of the wave
  // after); zero at the ends of the region. Consecutive exchanges must use
  // alternate buffers: a wave may write buffer b again only after every wave
  // has passed the barrier of an exchange in the other buffer.
  template <int N>
  __device__ static void exchange(const T (&v)[N], T* E, int buf, T& up, T& dn, GroupBarrier& gb) {
    const int lane = threadIdx.x & 63;
    const int wv = wave_in_group<kThreads>();
    T* e = E + buf * (NW * 2 * 64);
    e[(wv * 2 + 0) * 64 + lane] = v[0];
    e[(wv * 2 + 1) * 64 + lane] = v[N - 1];
    group_sync(gb);
    up = wv > 0 ? e[((wv - 1) * 2 + 1) * 64 + lane] : T(0);
    dn = wv + 1 < NW ? e[((wv + 1) * 2 + 0) * 64 + lane] : T(0);
  }
  static bool fits(int degree, int nx, int ntx, int ntiles) {
    if (degree - 1 > HMAX || ntx < 1) return false;
    return ntx == band_ntx(nx, degree) && ntiles == ntx * ((nx + TSY - 1) / TSY);
  }
  // Interior columns [ix0, ix1) and first row y0 of tile t; tx is its column
  // of tiles. The tiles at the grid's left and right edges are ta wide, the
  // others tsx (band_ntx); the last one takes what remains.
  __device__ static void span(const ColView<T>& v, int t, int& tx, int& ix0, int& ix1, int& y0) {
    tx = t % v.ntx;
    y0 = (t / v.ntx) * TSY;
    if (v.ntx == 1) {
      ix0 = 0;
      ix1 = v.nx;
      return;
    }
    ix0 = tx == 0 ? 0 : v.ta + (tx - 1) * v.tsx;
    ix1 = tx == 0 ? v.ta : (tx + 1 == v.ntx ? v.nx : ix0 + v.tsx);
  }
  // First grid column of the 64-lane region of tile column tx with a halo of
  // H columns: at the grid's edges the region ends at the edge, where the
  // lane shifts bring in the zero boundary value.
  __device__ static int region_x(const ColView<T>& v, int tx, int ix0, int H) {
    if (tx == 0) return 0;
    if (tx + 1 == v.ntx) return v.nx - 64;
    return ix0 - H;
  }

  // Per-tile sums without barriers of their own. Each wave adds its lanes
  // (wave_sum) and parks the result in LDS, alternate tiles in alternate
  // buffers; wave 0 adds the waves' values of a tile (a fixed tree over the
  // waves) after the next tile's barriers, when every wave has parked them,
  // and stores the tile's partials. `finish` ends a run of tiles: one
  // barrier, then the last tile. A buffer is parked in again two tiles later,
  // behind the barriers of the tile in between, which wave 0 reaches only
  // after reading it.
  struct TileSums {
    double (*buf)[NW][2];  // [2][NW][2] in LDS
    double* out0;
    double* out1;          // null: one value per tile
    int pend;              // tile whose sums are parked and not yet stored, -1: none
    int pbuf;              // its buffer

    __device__ void settle() {
      if (pend < 0) return;
      if (wave_in_group<kThreads>() == 0) {
        const int lane = threadIdx.x & 63;
        double a = 0.0, c = 0.0;
        if (lane < NW) {
          a = buf[pbuf][lane][0];
          c = buf[pbuf][lane][1];
        }
        static_assert(NW == 16, "one row of 16 lanes holds the wave sums");
        a += dpp_f64<0xB1>(a);
        a += dpp_f64<0x4E>(a);
        a += dpp_f64<0x141>(a);
        a += dpp_f64<0x140>(a);
        c += dpp_f64<0xB1>(c);
        c += dpp_f64<0x4E>(c);
        c += dpp_f64<0x141>(c);
        c += dpp_f64<0x140>(c);
        if (lane == 0) {
          out0[pend] = a;
          if (out1) out1[pend] = c;
        }
      }
      pend = -1;
    }
    __device__ void park(int t, int b, double a, double c) {
      a = wave_sum(a);
      c = wave_sum(c);
      if ((threadIdx.x & 63) == 0) {
        const int wv = wave_in_group<kThreads>();
        buf[b][wv][0] = a;
        buf[b][wv][1] = c;
      }
      pend = t;
      pbuf = b;
    }
    __device__ void finish(GroupBarrier& gb) {
      group_sync(gb);
      settle();
    }
  };

  // Chebyshev preconditioner on one tile (interior columns [ix0, ix1), region
  // columns from rx0): Zi[r] receives z at row
  // wave * BR + r of the region (meaningful only on the interior of the tile;
  // callers mask it) and Rl[(wave * BR + r) * 64 + lane] r on the interior
  // (zero elsewhere; read back by the same thread).
  //
  // Every sweep updates all rows and lanes of the band without branches, so
  // the rows of a band overlap in the pipeline. Values outside the part of
  // the region where W_j is valid ([j, R - j) in both directions) are
  // meaningless but never reach a valid value: a valid node of sweep j + 1
  // reads only nodes valid in sweep j. Nodes outside the grid hold zero
  // (homogeneous Dirichlet values); S is meaningful only inside the grid.
  // `val(r)` gives r at band row r of the region for every lane (it may use
  // DPP, so it runs unmasked); its value at nodes outside the grid is dropped.
  // H is the halo of the region: degree - 1, or degree when r is valid only
  // off the outermost ring of the region (warm start). The caller's exchange
  // for `val` used buffer `eb` of E; the sweeps continue with the other
  // buffer and alternate. `after0()` runs once step 0 has read every value
  // `val` depends on (phase B issues the next tile's loads there, into the
  // registers its inputs leave free, so they stream during the sweeps).
  template <typename VF, typename AF>
  __device__ static void cheb(const ColView<T>& A, int degree, int H, int rx0, int ix0, int ix1, int y0, VF val,
                              T* E, T* Rl, T (&Zi)[BR], GroupBarrier& gb, int eb, AF after0) {
    const int lane = threadIdx.x & 63;
    const int wv = wave_in_group<kThreads>();
    const int nx = A.nx;
    const int RY = TSY + 2 * H;
    const int gx = rx0 + lane;
    const bool xin = gx >= 0 && gx < nx;     // lane holds a grid column
    const bool xint = gx >= ix0 && gx < ix1;  // interior column of the tile
    const int yb = wv * BR;                                    // first region row of this wave
    T S[BR], W[BR];
    // step 0: S = D^-1 r, W = S / theta
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int ly = yb + r;
      const int gy = y0 - H + ly;
      const bool in = xin && ly < RY && gy >= 0 && gy < nx;
      const T v = val(r);
      const T rv = in ? v : T(0);
      S[r] = rv * A.inv_diag;
      W[r] = S[r] * A.inv_theta;
      Zi[r] = W[r];
      const bool interior = xint && ly >= H && ly < H + TSY;
      Rl[ly * 64 + lane] = interior ? rv : T(0);
    }
    after0();
    const T w8 = A.w8;
    // Nodes outside the grid stay at zero without a select per node: a row
    // outside the grid (the same for the whole wave) is not updated at all,
    // and a lane outside it takes zero coefficients, so its new W is
    // 0 * 0 + 0 * S. Inside the grid the arithmetic is the same as with the
    // coefficients themselves.
    bool row_in[BR];
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int gy = y0 - H + yb + r;
      row_in[r] = gy >= 0 && gy < nx;
    }
    // One row of a sweep from the old values of the rows below (cm), at (c0)
    // and above (cp).
    auto row = [&](int r, T cm, T c0, T cp, T ca, T cb) {
      if (!row_in[r]) return;
      const T vs = cm + cp;
      const T col = vs + c0;
      const T s8 = (from_prev(col) + from_next(col)) + vs;
      // S - D^-1 K_0 W, with D^-1 K_0 W = W - s8 / 8
      const T sn = S[r] - (c0 - w8 * s8);
      S[r] = sn;
      const T wn = ca * c0 + cb * sn;
      W[r] = wn;
      Zi[r] += wn;
    };
    static_assert(BR >= 3, "a band has inner rows");
    for (int j = 1; j < degree; ++j) {
      // The band's edge rows go to the neighbouring waves and the inner rows
      // are updated while they travel; the barrier and the reads of the
      // neighbours' edges come before the edge rows only.
      T* e = E + ((eb + j) & 1) * (NW * 2 * 64);
      e[(wv * 2 + 0) * 64 + lane] = W[0];
      e[(wv * 2 + 1) * 64 + lane] = W[BR - 1];
      const T ca_j = ld_uniform(A.chebA, j), cb_j = ld_uniform(A.chebB, j);
      const T ca = xin ? ca_j : T(0), cb = xin ? cb_j : T(0);
      const T w0 = W[0], w1 = W[1], wl = W[BR - 1], wl1 = W[BR - 2];
      T cm = w0;
#pragma unroll
      for (int r = 1; r + 1 < BR; ++r) {
        const T c0 = W[r];
        row(r, cm, c0, W[r + 1], ca, cb);
        cm = c0;
      }
      group_sync(gb);
      const T up = wv > 0 ? e[((wv - 1) * 2 + 1) * 64 + lane] : T(0);
      const T dn = wv + 1 < NW ? e[((wv + 1) * 2 + 0) * 64 + lane] : T(0);
      row(0, up, w0, w1, ca, cb);
      row(BR - 1, wl1, wl, dn, ca, cb);
    }
  }

  // Whether a column can start from the contents of X: the region grown by
  // one more node must fit the band (the tile widths leave that node in x).
  __device__ static bool warm_fits(const ColView<T>&, int degree) {
    const int H1 = degree;  // (degree - 1) + 1
    return TSY + 2 * H1 <= RB;
  }

  // Start of the iteration: z = M r with r = b (x = 0), or r = b - K_0 x from
  // the contents of x (warm). Partials r.z, b.b and r.r; a warm start stores r.
  __device__ static void start(const ColView<T>& v, int degree, int t, bool warm, T* W0, T*, GroupBarrier& gb,
                               double& rz, double& bb, double& rr) {
    T* E = W0;
    T* Rl = W0 + kEx;
    const int lane = threadIdx.x & 63;
    const int wv = wave_in_group<kThreads>();
    const int nx = v.nx;
    const int H = warm ? degree : degree - 1;
    int tx, ix0, ix1, y0;
    span(v, t, tx, ix0, ix1, y0);
    const int rx0 = region_x(v, tx, ix0, H);
    const int RY = TSY + 2 * H;
    const int gx = rx0 + lane;
    const bool xin = gx >= 0 && gx < nx;
    const int yb = wv * BR;
    const bool xint = gx >= ix0 && gx < ix1;
    T bv[BR], xv[BR];
    bb = 0.0;
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int ly = yb + r;
      const int gy = y0 - H + ly;
      const bool in = xin && ly < RY && gy >= 0 && gy < nx;
      bv[r] = xv[r] = T(0);
      if (in) bv[r] = v.b[(unsigned)(gy * nx + gx)];
      if (warm && in) xv[r] = v.x[(unsigned)(gy * nx + gx)];
      if (xint && ly >= H && ly < H + TSY && gy < nx) bb += (double)bv[r] * (double)bv[r];
    }
    // warm: r = b - K_0 x, valid off the outermost ring of the region
    // (exchange buffer 0; the sweeps continue with 1, 0, ...)
    T up = T(0), dn = T(0);
    if (warm) exchange(xv, E, 0, up, dn, gb);
    auto val = [&](int r) {
      if (!warm) return bv[r];
      const T cm = r > 0 ? xv[r - 1] : up;
      const T cp = r + 1 < BR ? xv[r + 1] : dn;
      return bv[r] - k0_apply(cm, xv[r], cp, v.c0, v.c1);
    };
    T Zi[BR];
    cheb(v, degree, H, rx0, ix0, ix1, y0, val, E, Rl, Zi, gb, 0, [] {});
    rz = rr = 0.0;
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int ly = yb + r;
      const int gy = y0 - H + ly;
      if (xint && ly >= H && ly < H + TSY && gy < nx) {
        const unsigned o = (unsigned)(gy * nx + gx);
        const T ri = Rl[ly * 64 + lane];
        rr += (double)ri * (double)ri;
        rz += (double)ri * (double)Zi[r];
        if (warm) {
          v.r0[o] = ri;
        } else {
          v.x[o] = T(0);
        }
        v.z[o] = Zi[r];
      }
    }
  }

  // Phase A needs a one-node halo only, so it has tiles of its own: a
  // wavefront of columns (62 interior ones, 63 at the grid's edges, where the
  // region starts or ends at the edge) by the band's rows. Its p.q partials
  // are per phase-A tile.
  __device__ static int ntx_a(const ColView<T>& v) { return band_cols(v.nx, 1); }
  __device__ static int ntiles_a(const ColView<T>& v) { return ntx_a(v) * ((v.nx + TSY - 1) / TSY); }
  __device__ static void span_a(const ColView<T>& v, int t, int& ix0, int& ix1, int& y0) {
    const int ntx = ntx_a(v), tx = t % ntx;
    y0 = (t / ntx) * TSY;
    if (ntx == 1) {
      ix0 = 0;
      ix1 = v.nx;
      return;
    }
    ix0 = tx == 0 ? 0 : 63 + (tx - 1) * 62;
    ix1 = tx == 0 ? 63 : (tx + 1 == ntx ? v.nx : ix0 + 62);
  }

  // Inputs of phase A on this wave's rows of the region (tile plus a 1-node
  // halo; at the grid's left edge the region starts at the edge).
  struct InA {
    T z[BRA], po[BRA], x[BRA];
  };
  __device__ static int region_a(int ix0) { return ix0 > 0 ? ix0 - 1 : 0; }
  __device__ static void load_a(const ColView<T>& v, int t, const IterVecs<T>& I, InA& in) {
    const int lane = threadIdx.x & 63;
    const int wv = wave_in_group<kThreads>();
    const int nx = v.nx;
    int ix0, ix1, y0;
    span_a(v, t, ix0, ix1, y0);
    const int gx = region_a(ix0) + lane;
    const bool xin = gx <= ix1 && gx < nx;
    const bool xint = gx >= ix0 && gx < ix1;
#pragma unroll
    for (int r = 0; r < BRA; ++r) {
      const int ly = wv * BRA + r;
      const int gy = y0 - 1 + ly;
      in.z[r] = in.po[r] = in.x[r] = T(0);
      if (xin && ly < TSY + 2 && gy >= 0 && gy < nx) {
        const unsigned o = (unsigned)(gy * nx + gx);
        in.z[r] = v.z[o];
        if (!I.first) {
          in.po[r] = I.po[o];
          if (xint && ly >= 1 && ly <= TSY) in.x[r] = v.x[o];
        }
      }
    }
  }

  __device__ static double compute_a(const ColView<T>& v, int t, const IterVecs<T>& I, const InA& in, T* W0,
                                     GroupBarrier& gb, int eb) {
    const int lane = threadIdx.x & 63;
    const int wv = wave_in_group<kThreads>();
    const int nx = v.nx;
    int ix0, ix1, y0;
    span_a(v, t, ix0, ix1, y0);
    const int gx = region_a(ix0) + lane;
    const bool xint = gx >= ix0 && gx < ix1;
    const int yb = wv * BRA;
    T pc[BRA];
#pragma unroll
    for (int r = 0; r < BRA; ++r) {
      const int ly = yb + r;
      const int gy = y0 - 1 + ly;
      pc[r] = I.first ? in.z[r] : in.z[r] + I.beta * in.po[r];
      if (!I.first && xint && ly >= 1 && ly <= TSY && gy < nx)
        v.x[(unsigned)(gy * nx + gx)] = in.x[r] + I.alpha_prev * in.po[r];
    }
    T up, dn;
    exchange(pc, W0, eb, up, dn, gb);
    double pq = 0.0;
#pragma unroll
    for (int r = 0; r < BRA; ++r) {
      const int ly = yb + r;
      const T cm = r > 0 ? pc[r - 1] : up;
      const T cp = r + 1 < BRA ? pc[r + 1] : dn;
      const T qv = k0_apply(cm, pc[r], cp, v.c0, v.c1);
      const int gy = y0 - 1 + ly;
      if (xint && ly >= 1 && ly <= TSY && gy < nx) {
        const unsigned o = (unsigned)(gy * nx + gx);
        I.pn[o] = pc[r];  // q is recomputed in phase B
        pq += (double)pc[r] * (double)qv;
      }
    }
    return pq;
  }

  // Phase A over tiles t_begin, t_begin + step, ... < t_end of a column; the
  // inputs of the next tile are loaded while the current one is computed
  // (short bands, two copies in registers) or once its stores are issued, so
  // the next tile's wait for them does not also wait for those stores.
  // Consecutive tiles exchange through alternate buffers. `sb`: the group's
  // [2][NW][2] sum buffers.
  __device__ static void run_a(const ColView<T>& v, int t_begin, int t_end, int step, const IterVecs<T>& I, T* W0,
                               GroupBarrier& gb, double (*sb)[NW][2], double* part) {
    if (t_begin >= t_end) return;
    TileSums sums{sb, part, nullptr, -1, 0};
    InA cur;
    load_a(v, t_begin, I, cur);
    int k = 0;
    for (int t = t_begin; t < t_end; t += step, ++k) {
      InA nxt;
      const bool more = t + step < t_end;
      if (kPrefetch && more) load_a(v, t + step, I, nxt);
      const double pq = compute_a(v, t, I, cur, W0, gb, k & 1);
      if (!kPrefetch && more) load_a(v, t + step, I, cur);
      sums.settle();
      sums.park(t, k & 1, pq, 0.0);
      if (kPrefetch && more) cur = nxt;
    }
    sums.finish(gb);
  }

  // x += alpha p on the interior of a tile, the update a stopping column still
  // owes (zero: x = 0 instead).
  __device__ static void finalize(const ColView<T>& v, int t, T alpha, const T* p, bool zero) {
    const int lane = threadIdx.x & 63;
    const int wv = wave_in_group<kThreads>();
    const int nx = v.nx;
    int tx, ix0, ix1, y0;
    span(v, t, tx, ix0, ix1, y0);
    const int gx = ix0 + lane;
    constexpr int rows = (TSY + NW - 1) / NW;
#pragma unroll
    for (int r = 0; r < rows; ++r) {
      const int ly = wv * rows + r;
      const int gy = y0 + ly;
      if (gx < ix1 && ly < TSY && gy < nx) {
        const unsigned o = (unsigned)(gy * nx + gx);
        if (zero) {
          v.x[o] = T(0);
        } else {
          v.x[o] += alpha * p[o];
        }
      }
    }
  }

  // Inputs of phase B on this wave's rows of the region: r and p on the tile
  // grown by `degree` nodes (the Chebyshev halo plus one node, so that
  // q = K_0 p is known on the Chebyshev region without storing q).
  struct InB {
    T r[BR], p[BR];
  };
  __device__ static void load_b(const ColView<T>& v, int degree, int t, const IterVecs<T>& I, InB& in) {
    const int lane = threadIdx.x & 63;
    const int wv = wave_in_group<kThreads>();
    const int H = degree, nx = v.nx;
    int tx, ix0, ix1, y0;
    span(v, t, tx, ix0, ix1, y0);
    const int gx = region_x(v, tx, ix0, H) + lane;
    const bool xin = gx >= 0 && gx < nx;
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int ly = wv * BR + r;
      const int gy = y0 - H + ly;
      in.r[r] = in.p[r] = T(0);
      if (xin && ly < TSY + 2 * H && gy >= 0 && gy < nx) {
        const unsigned o = (unsigned)(gy * nx + gx);
        in.r[r] = I.ro[o];
        in.p[r] = I.pn[o];
      }
    }
  }

  // Inputs of tile tn when `in` holds those of tile tc: if tn's region lies
  // s columns to the right of tc's in the same band rows, lanes l < 64 - s
  // take tc's values from lane l + s (the same grid columns; r and p are not
  // written in phase B) and only the last s lanes are loaded; otherwise every
  // lane is loaded (s = 64).
  __device__ static void load_b_next(const ColView<T>& v, int degree, int tc, int tn, const IterVecs<T>& I,
                                     InB& in) {
    int txc, ixc0, ixc1, yc0, txn, ixn0, ixn1, yn0;
    span(v, tc, txc, ixc0, ixc1, yc0);
    span(v, tn, txn, ixn0, ixn1, yn0);
    const int H = degree;
    const int rxn = region_x(v, txn, ixn0, H);
    int sh = rxn - region_x(v, txc, ixc0, H);
    if (yn0 != yc0 || sh <= 0 || sh > 64) sh = 64;
    const int lane = threadIdx.x & 63;
    const int wv = wave_in_group<kThreads>();
    const int nx = v.nx;
    const int gx = rxn + lane;
    const bool fresh = lane >= 64 - sh;
    const bool xin = fresh && gx >= 0 && gx < nx;
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const T rs = __shfl_down(in.r[r], sh & 63, 64), ps = __shfl_down(in.p[r], sh & 63, 64);
      const int ly = wv * BR + r;
      const int gy = yn0 - H + ly;
      in.r[r] = fresh ? T(0) : rs;
      in.p[r] = fresh ? T(0) : ps;
      if (xin && ly < TSY + 2 * H && gy >= 0 && gy < nx) {
        const unsigned o = (unsigned)(gy * nx + gx);
        in.r[r] = I.ro[o];
        in.p[r] = I.pn[o];
      }
    }
  }

  template <typename AF, typename EF>
  __device__ static void compute_b(const ColView<T>& v, int degree, int t, const IterVecs<T>& I, const InB& in,
                                   T* W0, T* W1, GroupBarrier& gb, int eb, double& rz, double& rr, AF after0,
                                   EF before_out) {
    const int lane = threadIdx.x & 63;
    const int wv = wave_in_group<kThreads>();
    const int H = degree, nx = v.nx;
    int tx, ix0, ix1, y0;
    span(v, t, tx, ix0, ix1, y0);
    const int rx0 = region_x(v, tx, ix0, H);
    T* E = W0;
    T* Rl = W0 + kEx;
    // r - alpha q with q = K_0 p on the region, valid off its outermost ring
    // (exchange buffer eb; the sweeps continue with the other one, alternating)
    T up, dn;
    exchange(in.p, E, eb, up, dn, gb);
    auto val = [&](int r) {
      const T cm = r > 0 ? in.p[r - 1] : up;
      const T cp = r + 1 < BR ? in.p[r + 1] : dn;
      return in.r[r] - I.alpha * k0_apply(cm, in.p[r], cp, v.c0, v.c1);
    };
    T Zi[BR];
    cheb(v, degree, H, rx0, ix0, ix1, y0, val, E, Rl, Zi, gb, eb, after0);
    before_out();
    rz = rr = 0.0;
    const int gx = rx0 + lane;
    const bool xint = gx >= ix0 && gx < ix1;
#pragma unroll
    for (int r = 0; r < BR; ++r) {
      const int ly = wv * BR + r;
      const int gy = y0 - H + ly;
      if (xint && ly >= H && ly < H + TSY && gy < nx) {
        const unsigned o = (unsigned)(gy * nx + gx);
        const T ri = Rl[ly * 64 + lane];
        I.rn[o] = ri;
        v.z[o] = Zi[r];
        rr += (double)ri * (double)ri;
        rz += (double)ri * (double)Zi[r];
      }
    }
  }

  // Phase B over tiles t_begin, t_begin + step, ... < t_end of a column; the
  // inputs of the next tile are loaded while the current one is computed:
  // before it (short bands, two copies in registers) or, for tall bands, into
  // the current tile's input registers once its first Chebyshev step has
  // consumed them.
  // A tile makes `degree` exchanges (one for q, then the sweeps), so the
  // next tile's first exchange takes the buffer after the tile's last one.
  __device__ static void run_b(const ColView<T>& v, int degree, int t_begin, int t_end, int step,
                               const IterVecs<T>& I, T* W0, T* W1, GroupBarrier& gb,
                               double (*sb)[NW][2], double* part_rz, double* part_rr) {
    if (t_begin >= t_end) return;
    TileSums sums{sb, part_rz, part_rr, -1, 0};
    InB cur;
    load_b(v, degree, t_begin, I, cur);
    if (!kPrefetch) {
      ready(cur.r);
      ready(cur.p);
    }
    int eb = 0, k = 0;
    for (int t = t_begin; t < t_end; t += step, ++k) {
      InB nxt;
      const bool more = t + step < t_end;
      if (kPrefetch && more) load_b(v, degree, t + step, I, nxt);
      double rz, rr;
      // the next tile's loads, issued after the first Chebyshev step, are
      // complete before this tile's results are stored (a tile start then
      // never waits for the stores of the tile before)
      compute_b(v, degree, t, I, cur, W0, W1, gb, eb, rz, rr, [&] {
        if (!kPrefetch && more) {
          if (kReuseHalo) {
            load_b_next(v, degree, t, t + step, I, cur);
          } else {
            load_b(v, degree, t + step, I, cur);
          }
        }
      }, [&] {
        if (!kPrefetch) {  // unconditional, so every path into the next tile has them ready
          ready(cur.r);
          ready(cur.p);
        }
      });
      eb = (eb + degree) & 1;
      sums.settle();
      sums.park(t, k & 1, rz, rr);
      if (kPrefetch && more) cur = nxt;
    }
    sums.finish(gb);
  }
};

// Tile routines end with a group reduction (two group barriers after the last
// LDS access of the tile), so the next tile of the group may overwrite the
// group's buffers without a further barrier.
template <typename T, typename Tile, int G, bool RAGGED>
__global__ void __launch_bounds__(Tile::kThreads* G) pcg_kernel(const PcgArgs<T> A, const PcgCols<T> C,
                                                                int lds_group) {
  constexpr int GT = Tile::kThreads;
  extern __shared__ unsigned char smem_raw[];
  const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / GT);  // uniform per wave
  const int lt = threadIdx.x % GT;
  const int degree = A.degree;
  T* W0 = reinterpret_cast<T*>(smem_raw) + (long)grp * lds_group;
  T* W1 = W0 + lds_group / 2;
  // per-column done flags of this block's columns, after the tile buffers
  int* sdone = reinterpret_cast<int*>(reinterpret_cast<T*>(smem_raw) + (long)G * lds_group);
  __shared__ double sred[G][GT / 64][2];
  // banded tiles (one group per block) park per-wave tile sums in two buffers
  static_assert(!Tile::kParkedSums || G == 1, "parked tile sums serve one group per block");
  __shared__ double spart[2][GT / 64][2];
  double (*tsums)[GT / 64][2] = Tile::kParkedSums ? spart : sred;
  __shared__ double s4[5];
  static_assert(Tile::kThreads * G >= 5 * 64, "column sums take five waves");
  __shared__ int sflag;
  __shared__ unsigned sgbar[G];
  if (threadIdx.x < G) sgbar[threadIdx.x] = 0u;
  GroupBarrier gb{&sgbar[grp], 0u, GT / 64, A.sc.status, false, G == 1};

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
      v.w8 = ld_uniform(&k->w8, 0);
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
      v.w8 = A.w8;
      v.chebA = A.chebA;
      v.chebB = A.chebB;
    }
    v.ta = 64 - band_halo(degree);
    v.tsx = 64 - 2 * band_halo(degree);
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
  // this block's contiguous range of the work list: per_block items (whole
  // columns), or an even share of the list (shares differ by at most one item,
  // so no block works a tile more than the split needs)
  long w_begin, w_end;
  if (A.per_block > 0) {
    w_begin = (long)blockIdx.x * A.per_block;
    w_end = w_begin + A.per_block < nwork ? w_begin + A.per_block : nwork;
  } else {
    w_begin = (long)blockIdx.x * nwork / gridDim.x;
    w_end = ((long)blockIdx.x + 1) * nwork / gridDim.x;
  }
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
  // this block holds every tile of the column: its phases need only the block's
  // barriers, behind a wait for the block's own global stores (column_end_whole)
  auto whole = [&](const ColView<T>& v, int t0, int t1) { return t0 == 0 && t1 == v.ntiles; };
  // the column starts from the contents of its x
  auto warm_of = [&](const ColView<T>& v) { return A.warm && Tile::warm_fits(v, degree); };
  // Fixed-order sums of up to five per-tile partial arrays of a column, one wave each.
  // (bit w of pq_arrays: array w holds p.q partials, one per phase-A tile)
  auto col_sums = [&](const ColView<T>& v, const double* q0, const double* q1, const double* q2, const double* q3,
                      const double* q4, int pq_arrays) {
    __syncthreads();
    const int wv = threadIdx.x >> 6;
    const double* src = wv == 0 ? q0 : wv == 1 ? q1 : wv == 2 ? q2 : wv == 3 ? q3 : q4;
    if (wv < 5 && src) {
      const int n = (pq_arrays >> wv) & 1 ? Tile::ntiles_a(v) : v.ntiles;
      double s = 0.0;
      for (int t = threadIdx.x & 63; t < n; t += 64) s += src[v.tbase + t];
      s = wave_sum(s);
      if ((threadIdx.x & 63) == 0) s4[wv] = s;
    }
    __syncthreads();
  };
  for (int c = c_first + (int)threadIdx.x; c <= c_last; c += GT * G) {
    int skip = 0;
    if constexpr (RAGGED) {
      if (!listed) skip = C.active[C.prob[c]] == 0;
    }
    sdone[c - c_first] = skip;
  }
  __syncthreads();

  // ---- start (column phase 1): z = M r with r = b (x = 0) or r = b - K_0 x (warm); partials b.b, r.z, r.r
  for (int c = c_first; c <= c_last; ++c) {
    const ColView<T> v = view(c);
    if (sdone[c - c_first]) {
      if (threadIdx.x == 0 && owner(v)) A.sc.iters[c] = 0;
      continue;
    }
    int t0, t1;
    tiles_of(v, t0, t1);
    if (t1 <= t0) continue;
    const bool warm = warm_of(v);
    for (int t = t0 + grp; t < t1; t += G) {
      double rz, bb, rr, unused = 0.0;
      Tile::start(v, degree, t, warm, W0, W1, gb, rz, bb, rr);
      group_sum2<GT>(rz, bb, sred, gb);
      group_sum2<GT>(rr, unused, sred, gb);
      if (lt == 0) {
        P(PART_RZ1)[v.tbase + t] = rz;
        P(PART_BB)[v.tbase + t] = bb;
        P(PART_RR1)[v.tbase + t] = rr;
      }
    }
    if (whole(v, t0, t1)) column_end_whole();
    else column_arrive(arr + c, (unsigned)(t1 - t0));
  }

  bool aborted = false;
  // iteration A.maxit only applies the x update of the last iteration
  for (int it = 0; it <= A.maxit && !aborted; ++it) {
    const int par = it & 1;
    bool any_active = false;
    // ---- phase A (column phase 2 + 2 it): x += alpha' p', p = z + beta p', q = K_0 p, partial p.q
    for (int c = c_first; c <= c_last && !aborted; ++c) {
      if (sdone[c - c_first]) continue;
      const ColView<T> v = view(c);
      int t0, t1;
      tiles_of(v, t0, t1);
      if (t1 <= t0) continue;
      if (whole(v, t0, t1)) __syncthreads();
      else if (!column_wait(arr + c, (unsigned)((1 + 2 * it) * v.ntiles), A.sc.status, &sflag)) {
        aborted = true;
        break;
      }
      const bool first = it == 0;
      col_sums(v, P(PART_BB), P(par ? PART_RR0 : PART_RR1), first ? nullptr : P(par ? PART_RZ0 : PART_RZ1),
               first ? nullptr : P(par ? PART_RZ1 : PART_RZ0), first ? nullptr : P(par ? PART_PQ0 : PART_PQ1), 1 << 4);
      const double bb = s4[0];
      const double rr = s4[1];
      IterVecs<T> I{};
      I.first = first;
      I.po = par ? v.p0 : v.p1;
      I.pn = par ? v.p1 : v.p0;
      I.beta = first ? T(0) : (T)(s4[2] / s4[3]);
      I.alpha_prev = first ? T(0) : (T)(s4[3] / s4[4]);
      if (it == A.maxit || bb == 0.0 || sqrt(rr) <= A.rtol * sqrt(bb)) {
        // stop: apply the pending update x += alpha' p' (a zero right-hand side
        // gives x = 0 also from a warm start)
        const bool zero = first && bb == 0.0 && warm_of(v);
        if (!first || zero)
          for (int t = t0 + grp; t < t1; t += G) Tile::finalize(v, t, I.alpha_prev, I.po, zero);
        __syncthreads();
        if (threadIdx.x == 0) {
          sdone[c - c_first] = 1;
          if (owner(v)) A.sc.iters[c] = it;
        }
        __syncthreads();
        continue;
      }
      any_active = true;
      {
        // this block's phase-A tiles: the same share of the column as its tiles
        const long nta = Tile::ntiles_a(v);
        const int ta0 = (int)(t0 * nta / v.ntiles), ta1 = (int)(t1 * nta / v.ntiles);
        Tile::run_a(v, ta0 + grp, ta1, G, I, W0, gb, tsums, P(par ? PART_PQ1 : PART_PQ0) + v.tbase);
      }
      if (whole(v, t0, t1)) column_end_whole();
      else column_arrive(arr + c, (unsigned)(t1 - t0));
    }
    if (!any_active || aborted) break;
    // ---- phase B (column phase 3 + 2 it): r -= alpha q, z = M r, partials r.r, r.z
    for (int c = c_first; c <= c_last && !aborted; ++c) {
      if (sdone[c - c_first]) continue;
      const ColView<T> v = view(c);
      int t0, t1;
      tiles_of(v, t0, t1);
      if (t1 <= t0) continue;
      if (whole(v, t0, t1)) __syncthreads();
      else if (!column_wait(arr + c, (unsigned)((2 + 2 * it) * v.ntiles), A.sc.status, &sflag)) {
        aborted = true;
        break;
      }
      col_sums(v, P(par ? PART_PQ1 : PART_PQ0), P(par ? PART_RZ0 : PART_RZ1), nullptr, nullptr, nullptr, 1 << 0);
      const double pq = s4[0], gam = s4[1];
      if (!(pq > 0.0) || !isfinite(pq)) {
        // breakdown: keep the current iterate (phase A of this iteration applied the last update)
        __syncthreads();
        if (threadIdx.x == 0) {
          sdone[c - c_first] = 1;
          if (owner(v)) A.sc.iters[c] = it;
        }
        __syncthreads();
        continue;
      }
      IterVecs<T> I{};
      I.first = it == 0;
      I.alpha = (T)(gam / pq);
      I.pn = par ? v.p1 : v.p0;
      I.ro = it == 0 ? (warm_of(v) ? v.r0 : v.b) : (par ? v.r1 : v.r0);
      I.rn = par ? v.r0 : v.r1;
      Tile::run_b(v, degree, t0 + grp, t1, G, I, W0, W1, gb, tsums, P(par ? PART_RZ1 : PART_RZ0) + v.tbase,
                  P(par ? PART_RR1 : PART_RR0) + v.tbase);
      if (whole(v, t0, t1)) column_end_whole();
      else column_arrive(arr + c, (unsigned)(t1 - t0));
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

template <typename T, typename Tile, int G, bool RAGGED>
hipError_t launch_cfg(const PcgArgs<T>& args, const PcgCols<T>& cols, int max_blocks, hipStream_t s) {
  if (!RAGGED && !Tile::fits(args.degree, args.nx, args.ntx, args.ntiles)) return hipErrorInvalidValue;
  const int lds_group = Tile::lds_group(args.degree);
  const size_t tiles_bytes = sizeof(T) * (size_t)lds_group * G;
  auto kfn = pcg_kernel<T, Tile, G, RAGGED>;
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
  long per_block = 0;  // 0: the work list split evenly over the grid
  size_t sm = 0;
  if (!RAGGED && max_blocks < 0) {
    // Whole columns per block: each block owns k consecutive columns, k the
    // smallest count with which the grid fits on the device at once, so no
    // column phase needs the device-scope arrival counters. Taken when the
    // columns keep at least three quarters of the k * (resident blocks) column
    // places busy; other launches take the automatic grid.
    max_blocks = 0;
    for (long k = 1; k <= 8; ++k) {
      sm = tiles_bytes + sizeof(int) * (size_t)(k + 2);
      if (sm > 160 * 1024) return hipErrorInvalidValue;
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
      if (e != hipSuccess) return e;
      int per_cu = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, Tile::kThreads * G, sm);
      if (e != hipSuccess) return e;
      const long cap = (long)per_cu * ncu;
      if (cap < 1) break;
      if ((args.ncols + k - 1) / k <= cap) {
        if (4L * args.ncols >= 3L * k * cap) per_block = k * args.ntiles;
        break;
      }
    }
  }
  // a launch with no more tile groups than compute units gives each block one
  // group's worth (the column chain then waits on one tile per phase);
  // otherwise two, so that a block's next tile can load during the current one
  const long per_auto = nwork <= (long)ncu * G ? G : 2L * G;
  long grid = per_block > 0 ? (nwork + per_block - 1) / per_block : (nwork + per_auto - 1) / per_auto;
  if (max_blocks > 0 && grid > max_blocks) grid = max_blocks;
  if (grid < 1) grid = 1;
  for (int pass = 0; pass < 8 && per_block == 0; ++pass) {
    const long pb = (nwork + grid - 1) / grid;
    const long max_cols = pb / min_tiles + 2;  // a run of pb items spans at most this many columns
    sm = tiles_bytes + sizeof(int) * (size_t)max_cols;
    if (sm > 160 * 1024) return hipErrorInvalidValue;
    // the cooperative launch checks co-residency against this attribute, so keep it exact
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, Tile::kThreads * G, sm);
    if (e != hipSuccess) return e;
    const long cap = (long)per_cu * ncu;
    if (cap < 1) return hipErrorInvalidValue;
    if (grid <= cap) break;
    grid = cap;
    if (pass == 7) return hipErrorInvalidValue;
  }
  PcgArgs<T> a = args;
  a.per_block = per_block;
  PcgCols<T> c = cols;
  int lg = lds_group;
  hipLaunchKernelGGL(pcg_reset_kernel, dim3(1), dim3(256), 0, s, a.sc.arrivals, a.ncols, a.sc.status);
  if (!RAGGED && !args.no_coop) {
    void* kargs[] = {&a, &c, &lg};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kfn), dim3((unsigned)grid),
                                      dim3(Tile::kThreads * G), kargs, (unsigned)sm, s);
  }
  hipLaunchKernelGGL(kfn, dim3((unsigned)grid), dim3(Tile::kThreads * G), sm, s, a, c, lg);
  return hipGetLastError();
}

constexpr int slots(int ts, int maxh) {
  return ((ts + 2 * maxh) * (ts + 2 * maxh) + kSquareGroup - 1) / kSquareGroup;
}

template <typename T, bool RAGGED>
hipError_t dispatch_pcg(const PcgArgs<T>& args, const PcgCols<T>& cols, int tile, int max_blocks, hipStream_t s) {
  if (args.ncols <= 0) return hipSuccess;
  const int H = args.degree - 1;
  if (tile != 16) {
    // banded tiles, one group of 16 waves per block, of the band height the
    // host tiled with: the precision's default or, for small launches, 64 rows
    // (and 128 in FP32 when a single problem's launch has few tiles)
    constexpr int TSY = kBandRowsOf<T>;
    constexpr int TS = kBandRowsSmall;
    if constexpr (sizeof(T) == 4 && !RAGGED) {
      constexpr int TM = kBandRowsMid;
      if (args.rows == TM) {
        if (H > 15) return hipErrorInvalidValue;
        if (H <= 3) return launch_cfg<T, BandTile<T, TM, 3, 16>, 1, RAGGED>(args, cols, max_blocks, s);
        if (H <= 7) return launch_cfg<T, BandTile<T, TM, 7, 16>, 1, RAGGED>(args, cols, max_blocks, s);
        if (H <= 11) return launch_cfg<T, BandTile<T, TM, 11, 16>, 1, RAGGED>(args, cols, max_blocks, s);
        return launch_cfg<T, BandTile<T, TM, 15, 16>, 1, RAGGED>(args, cols, max_blocks, s);
      }
    }
    if (H > 15) return hipErrorInvalidValue;
    if (args.rows == TSY) {
      if (H <= 3) return launch_cfg<T, BandTile<T, TSY, 3, 16>, 1, RAGGED>(args, cols, max_blocks, s);
      if (H <= 7) return launch_cfg<T, BandTile<T, TSY, 7, 16>, 1, RAGGED>(args, cols, max_blocks, s);
      if (H <= 11) return launch_cfg<T, BandTile<T, TSY, 11, 16>, 1, RAGGED>(args, cols, max_blocks, s);
      return launch_cfg<T, BandTile<T, TSY, 15, 16>, 1, RAGGED>(args, cols, max_blocks, s);
    }
    if (args.rows == TS) {
      if (H <= 3) return launch_cfg<T, BandTile<T, TS, 3, 16>, 1, RAGGED>(args, cols, max_blocks, s);
      if (H <= 7) return launch_cfg<T, BandTile<T, TS, 7, 16>, 1, RAGGED>(args, cols, max_blocks, s);
      if (H <= 11) return launch_cfg<T, BandTile<T, TS, 11, 16>, 1, RAGGED>(args, cols, max_blocks, s);
      return launch_cfg<T, BandTile<T, TS, 15, 16>, 1, RAGGED>(args, cols, max_blocks, s);
    }
    return hipErrorInvalidValue;
  }
  return launch_cfg<T, SquareTile<T, 16, slots(16, 15)>, 4, RAGGED>(args, cols, max_blocks, s);
}

}  // namespace

template <typename T>
hipError_t launch_pcg(const PcgArgs<T>& args, int tile, int max_blocks, hipStream_t s) {
  return dispatch_pcg<T, false>(args, PcgCols<T>{}, tile, max_blocks, s);
}

template <typename T>
hipError_t launch_pcg_ragged(const PcgArgs<T>& args, const PcgCols<T>& cols, int tile, int max_blocks, hipStream_t s) {
  return dispatch_pcg<T, true>(args, cols, tile, max_blocks, s);
}

template hipError_t launch_pcg_ragged<double>(const PcgArgs<double>&, const PcgCols<double>&, int, int, hipStream_t);
template hipError_t launch_pcg_ragged<float>(const PcgArgs<float>&, const PcgCols<float>&, int, int, hipStream_t);
template hipError_t launch_pcg<double>(const PcgArgs<double>&, int, int, hipStream_t);
template hipError_t launch_pcg<float>(const PcgArgs<float>&, int, int, hipStream_t);

}  // namespace sgk
