// Batched vector kernels of the multi-problem flexible CG (Section 5, one
// instance per problem). Every launch covers all problems of the batch: grid
// dimension y is the problem, x the kBatchBlocks blocks that stride over its
// n x P entries. Reductions are two-stage with a fixed order per problem, and
// the scalars alpha, beta and the stopping test are evaluated on the device,
// identically in every block, so that an outer iteration needs no host round
// trip. A problem whose active flag is 0 is skipped by every launch.
#include "sg_internal.h"

namespace sgk {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum of two values; thread 0 gets the result.
__device__ void block_sum2(double& a, double& b) {
  __shared__ double sa[kThreads / 64], sb[kThreads / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sa[w] = a;
    sb[w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0.0;
    b = 0.0;
    for (int i = 0; i < kThreads / 64; ++i) {
      a += sa[i];
      b += sb[i];
    }
  }
}

__device__ __forceinline__ long stride_begin() { return (long)blockIdx.x * kThreads + threadIdx.x; }
__device__ __forceinline__ long stride_step() { return (long)gridDim.x * kThreads; }

// Partial sums of a0.b0 and a1.b1 of problem blockIdx.y.
__device__ void dot_partials(const BatchVecs& V, const double* a0, const double* b0, const double* a1,
                             const double* b1) {
  const int b = blockIdx.y;
  const long N = V.N[b];
  double s0 = 0.0, s1 = 0.0;
  for (long i = stride_begin(); i < N; i += stride_step()) {
    s0 += a0[i] * b0[i];
    if (a1) s1 += a1[i] * b1[i];
  }
  block_sum2(s0, s1);
  if (threadIdx.x == 0) {
    V.part[((long)b * kBatchBlocks + blockIdx.x) * 2 + 0] = s0;
    V.part[((long)b * kBatchBlocks + blockIdx.x) * 2 + 1] = s1;
  }
}

// Fixed-order sum of the kBatchBlocks partials of problem b (one block per problem).
__device__ void final_sums(const BatchVecs& V, int b, double& s0, double& s1) {
  double a = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < kBatchBlocks; i += kThreads) {
    a += V.part[((long)b * kBatchBlocks + i) * 2 + 0];
    c += V.part[((long)b * kBatchBlocks + i) * 2 + 1];
  }
  block_sum2(a, c);
  s0 = a;
  s1 = c;
}

__global__ void __launch_bounds__(kThreads) init_kernel(const BatchVecs V) {
  const int b = blockIdx.y;
  const long N = V.N[b];
  const double* f = V.f[b];
  double* r = V.r[b];
  double* x = V.x[b];
  double* p = V.p[b];
  double s0 = 0.0, s1 = 0.0;
  for (long i = stride_begin(); i < N; i += stride_step()) {
    const double fi = f[i];
    r[i] = fi;
    x[i] = 0.0;
    p[i] = 0.0;
    s0 += fi * fi;
  }
  block_sum2(s0, s1);
  if (threadIdx.x == 0) V.part[((long)b * kBatchBlocks + blockIdx.x) * 2 + 0] = s0;
}

__global__ void __launch_bounds__(kThreads) init_final_kernel(const BatchVecs V, double rtol) {
  const int b = blockIdx.x;
  double fn2, unused;
  final_sums(V, b, fn2, unused);
  if (threadIdx.x == 0) {
    BatchScal& S = V.sc[b];
    S.fn2 = fn2;
    S.rr = fn2;
    S.pq = S.pr = S.zq = S.pq_prev = 0.0;
    S.rtol2 = rtol * rtol * fn2;
    S.it = 0;
    S.inner_it = 0;
    const bool done = !(fn2 > S.rtol2);  // zero right-hand side (or rtol >= 1): x = 0 is the answer
    S.status = !isfinite(fn2) ? SG_BREAKDOWN : done ? SG_OK : SG_NOT_CONVERGED;
    V.active[b] = S.status == SG_NOT_CONVERGED ? 1 : 0;
  }
}

__global__ void __launch_bounds__(kThreads) dot_zq_kernel(const BatchVecs V) {
  if (!V.active[blockIdx.y]) return;
  dot_partials(V, V.z[blockIdx.y], V.q[blockIdx.y], nullptr, nullptr);
}

__global__ void __launch_bounds__(kThreads) zq_final_kernel(const BatchVecs V) {
  const int b = blockIdx.x;
  if (!V.active[b]) return;
  double zq, unused;
  final_sums(V, b, zq, unused);
  if (threadIdx.x == 0) V.sc[b].zq = zq;
}

// p = z + beta p with beta = -z.q / (p.q of the previous iteration); p = z at the first iteration.
__global__ void __launch_bounds__(kThreads) dirupdate_kernel(const BatchVecs V) {
  const int b = blockIdx.y;
  if (!V.active[b]) return;
  const BatchScal& S = V.sc[b];
  const double beta = S.it == 0 ? 0.0 : -S.zq / S.pq_prev;
  const long N = V.N[b];
  const double* z = V.z[b];
  double* p = V.p[b];
  for (long i = stride_begin(); i < N; i += stride_step()) p[i] = S.it == 0 ? z[i] : z[i] + beta * p[i];
}

__global__ void __launch_bounds__(kThreads) dot_pq_pr_kernel(const BatchVecs V) {
  const int b = blockIdx.y;
  if (!V.active[b]) return;
  dot_partials(V, V.p[b], V.q[b], V.p[b], V.r[b]);
}

__global__ void __launch_bounds__(kThreads) pq_pr_final_kernel(const BatchVecs V) {
  const int b = blockIdx.x;
  if (!V.active[b]) return;
  double pq, pr;
  final_sums(V, b, pq, pr);
  if (threadIdx.x == 0) {
    V.sc[b].pq = pq;
    V.sc[b].pr = pr;
  }
}

__device__ __forceinline__ bool curvature_ok(const BatchScal& S) {
  return S.pq > 0.0 && isfinite(S.pq) && isfinite(S.pr);
}

// alpha = p.r / p.q; x += alpha p, r -= alpha q; partial r.r.
__global__ void __launch_bounds__(kThreads) update_kernel(const BatchVecs V) {
  const int b = blockIdx.y;
  if (!V.active[b]) return;
  const BatchScal& S = V.sc[b];
  if (!curvature_ok(S)) return;
  const double alpha = S.pr / S.pq;
  const long N = V.N[b];
  double* x = V.x[b];
  double* r = V.r[b];
  const double* p = V.p[b];
  const double* q = V.q[b];
  double s0 = 0.0, s1 = 0.0;
  for (long i = stride_begin(); i < N; i += stride_step()) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    s0 += ri * ri;
  }
  block_sum2(s0, s1);
  if (threadIdx.x == 0) V.part[((long)b * kBatchBlocks + blockIdx.x) * 2 + 0] = s0;
}

// r.r, the iteration count and the stopping test; a problem that stops is masked from here on.
__global__ void __launch_bounds__(kThreads) update_final_kernel(const BatchVecs V) {
  const int b = blockIdx.x;
  if (!V.active[b]) return;
  BatchScal& S = V.sc[b];
  if (!curvature_ok(S)) {
    if (threadIdx.x == 0) {
      S.status = SG_BREAKDOWN;
      V.active[b] = 0;
    }
    return;
  }
  double rr, unused;
  final_sums(V, b, rr, unused);
  if (threadIdx.x == 0) {
    S.rr = rr;
    S.pq_prev = S.pq;
    S.it += 1;
    if (!isfinite(rr)) {
      S.status = SG_BREAKDOWN;
      V.active[b] = 0;
    } else if (rr <= S.rtol2) {
      S.status = SG_OK;
      V.active[b] = 0;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) to_inner_kernel(const BatchVecs V) {
  const int b = blockIdx.y;
  if (!V.active[b]) return;
  const long N = V.N[b];
  const double* r = V.r[b];
  T* w = reinterpret_cast<T*>(V.rw[b]);
  for (long i = stride_begin(); i < N; i += stride_step()) w[i] = (T)r[i];
}

__global__ void __launch_bounds__(kThreads) from_inner_kernel(const BatchVecs V) {
  const int b = blockIdx.y;
  if (!V.active[b]) return;
  const long N = V.N[b];
  const float* w = reinterpret_cast<const float*>(V.zw[b]);
  double* z = V.z[b];
  for (long i = stride_begin(); i < N; i += stride_step()) z[i] = (double)w[i];
}

// Adds the inner iteration counts of a ragged PCG launch to their problems and
// keeps a sticky copy of the launch's wait status.
// Adds the inner iteration counts of a ragged PCG launch (over the listed
// columns) to their problems and keeps a sticky copy of the wait status.
__global__ void count_iters_kernel(const int* iters, const int* act, const int* nact, const int* prob, BatchScal* sc,
                                   const int* pcg_status, int* sticky) {
  const int n = *nact;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    atomicAdd(reinterpret_cast<unsigned long long*>(&sc[prob[act[i]]].inner_it), (unsigned long long)iters[i]);
  if (blockIdx.x == 0 && threadIdx.x == 0 && *pcg_status != 0) *sticky = 1;
}

// One block: order-preserving list of the columns whose problem is active and
// the exclusive prefix sums of their tile counts.
__global__ void __launch_bounds__(1024) compact_kernel(const int* prob, const int* ntiles, int ncols,
                                                       const int* active, const int* pdeg, int pmin, int* act,
                                                       int* nact, long* cbase, long* nwork_act) {
  auto keep = [&](int c) { return active[prob[c]] != 0 && pdeg[prob[c]] >= pmin; };
  __shared__ int cnt[1024];
  __shared__ long tiles[1024];
  const int per = (ncols + 1023) / 1024;
  const int c0 = threadIdx.x * per;
  const int c1 = min(ncols, c0 + per);
  int k = 0;
  long t = 0;
  for (int c = c0; c < c1; ++c)
    if (keep(c)) {
      ++k;
      t += ntiles[c];
    }
  cnt[threadIdx.x] = k;
  tiles[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    int rk = 0;
    long rt = 0;
    for (int i = 0; i < 1024; ++i) {
      const int vk = cnt[i];
      const long vt = tiles[i];
      cnt[i] = rk;
      tiles[i] = rt;
      rk += vk;
      rt += vt;
    }
    *nact = rk;
    *nwork_act = rt;
  }
  __syncthreads();
  int pos = cnt[threadIdx.x];
  long base = tiles[threadIdx.x];
  for (int c = c0; c < c1; ++c)
    if (keep(c)) {
      act[pos] = c;
      cbase[pos] = base;
      ++pos;
      base += ntiles[c];
    }
}

dim3 vec_grid(const BatchVecs& V) {
  long need = (V.maxN + kThreads - 1) / kThreads;
  if (need > kBatchBlocks) need = kBatchBlocks;
  if (need < 1) need = 1;
  return dim3((unsigned)need, (unsigned)V.nprob);
}

}  // namespace

// Launches that reduce always start all kBatchBlocks blocks of a problem, so
// that every partial slot is written; the others use only as many blocks as
// the largest problem needs.
void launch_batch_init(const BatchVecs& V, double rtol, hipStream_t s) {
  hipLaunchKernelGGL(init_kernel, dim3(kBatchBlocks, V.nprob), dim3(kThreads), 0, s, V);
  hipLaunchKernelGGL(init_final_kernel, dim3(V.nprob), dim3(kThreads), 0, s, V, rtol);
}

void launch_batch_dot_zq(const BatchVecs& V, hipStream_t s) {
  hipLaunchKernelGGL(dot_zq_kernel, dim3(kBatchBlocks, V.nprob), dim3(kThreads), 0, s, V);
  hipLaunchKernelGGL(zq_final_kernel, dim3(V.nprob), dim3(kThreads), 0, s, V);
}

void launch_batch_dirupdate(const BatchVecs& V, hipStream_t s) {
  hipLaunchKernelGGL(dirupdate_kernel, vec_grid(V), dim3(kThreads), 0, s, V);
}

void launch_batch_dot_pq_pr(const BatchVecs& V, hipStream_t s) {
  hipLaunchKernelGGL(dot_pq_pr_kernel, dim3(kBatchBlocks, V.nprob), dim3(kThreads), 0, s, V);
  hipLaunchKernelGGL(pq_pr_final_kernel, dim3(V.nprob), dim3(kThreads), 0, s, V);
}

void launch_batch_update(const BatchVecs& V, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel, dim3(kBatchBlocks, V.nprob), dim3(kThreads), 0, s, V);
  hipLaunchKernelGGL(update_final_kernel, dim3(V.nprob), dim3(kThreads), 0, s, V);
}

template <typename T>
void launch_batch_to_inner(const BatchVecs& V, hipStream_t s) {
  hipLaunchKernelGGL(to_inner_kernel<T>, vec_grid(V), dim3(kThreads), 0, s, V);
}
template void launch_batch_to_inner<double>(const BatchVecs&, hipStream_t);
template void launch_batch_to_inner<float>(const BatchVecs&, hipStream_t);

void launch_batch_from_inner(const BatchVecs& V, hipStream_t s) {
  hipLaunchKernelGGL(from_inner_kernel, vec_grid(V), dim3(kThreads), 0, s, V);
}

void launch_batch_count_iters(const int* iters, const int* act, const int* nact, const int* prob, int ncols,
                              BatchScal* sc, const int* pcg_status, int* sticky_status, hipStream_t s) {
  if (ncols <= 0) return;
  const int blocks = (ncols + 255) / 256 < 64 ? (ncols + 255) / 256 : 64;
  hipLaunchKernelGGL(count_iters_kernel, dim3(blocks), dim3(256), 0, s, iters, act, nact, prob, sc, pcg_status,
                     sticky_status);
}

void launch_batch_compact(const int* prob, const int* ntiles, int ncols, const int* active, const int* pdeg, int pmin,
                          int* act, int* nact, long* cbase, long* nwork_act, hipStream_t s) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(1024), 0, s, prob, ntiles, ncols, active, pdeg, pmin, act, nact,
                     cbase, nwork_act);
}

}  // namespace sgk
