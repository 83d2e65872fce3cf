// Multi-problem batch: many independent SG problems solved together by the
// flexible CG (Section 5) with the hierarchical Schur complement
// preconditioner (Algorithm 1) or the mean-based one (Section 6).
//
// Every problem keeps its own handle (chaos tables, coefficients and vectors
// in its own part of the workspace). What is shared is the schedule: one
// outer iteration of the whole batch is a fixed sequence of launches in which
//   - all diagonal-block solves of one step of Algorithm 1 (the columns of
//     degree l of every problem that has that degree) run in one persistent
//     ragged PCG launch,
//   - the vector updates and reductions of the outer CG run in batched
//     launches with their scalars (alpha, beta, the stopping test) on the
//     device,
//   - each problem's SG operator launches do nothing once its solve stopped.
// Because the sequence does not depend on host decisions it is captured once
// into a HIP graph and replayed; the host only reads the per-problem active
// flags after each iteration to know when every solve has stopped.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sg_host.h"
#include "sg_internal.h"

struct sg_batch_ctx {
  int nprob = 0;
  int pmax = 0;
  int inner = 64;
  int degree = 1;
  int tile = 32;
  int rows = 0;        // band height of banded inner tiles
  int max_blocks = 0;  // cap on the blocks of a ragged inner launch (0 = as many as fit)
  sg_opts opts{};
  hipStream_t stream = nullptr;
  std::vector<sg_ctx*> h;
  // ragged column sets: set l (0..pmax) holds the degree-l columns of every
  // problem with p >= l; set pmax + 1 holds all columns (mean-based preconditioner)
  std::vector<sgk::PcgCols<double>> cols64;
  std::vector<sgk::PcgCols<float>> cols32;
  std::vector<int> set_ncols;
  std::vector<long> set_nwork_cap;  // planned work items per set (largest over the tilings)
  std::vector<size_t> set_off;      // byte offset of each set in the set region
  char* sets_base = nullptr;
  const void* sets_consts = nullptr;  // per-problem inner constants (device)
  sgk::PcgScratch sc{};
  int* sticky = nullptr;  // set if a bounded wait of an inner launch expired
  int* pdeg = nullptr;    // chaos degree of each problem (device)
  sgk::BatchVecs V{};
  double** x_tab = nullptr;        // device tables of the solution and right-hand-side addresses
  const double** f_tab = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_pc = -1;
};

namespace {

using sgh::fail;

struct Layout {
  size_t total = 0;
  size_t take(size_t bytes) {
    size_t o = total;
    total += (bytes + 255) / 256 * 256;
    return o;
  }
};

long nchaos(int M, int p) {
  long r = 1;
  for (int i = 1; i <= p; ++i) r = r * (M + i) / i;
  return r;
}

// Level offsets of a problem (graded basis: level l has C(M+l-1, l) functions).
std::vector<int> level_offsets(int M, int p) {
  std::vector<int> off(1, 0);
  for (int l = 0; l <= p; ++l) off.push_back(off.back() + (int)(nchaos(M, l) - (l > 0 ? nchaos(M, l - 1) : 0)));
  return off;
}

int batch_tile(const sg_opts& op) {
  if (op.tile == 16) return 16;
  return op.cheb_degree <= sgk::kBandMaxDegree ? 32 : 16;
}

// Inner tilings (tile kind, band rows) a batch may run with: the default
// first, then the other kinds the options allow (the autotuner's candidates).
std::vector<std::pair<int, int>> batch_tilings(const sg_opts& op) {
  const int def_rows = sgk::band_rows(op.inner_precision, op.cheb_degree);
  std::vector<std::pair<int, int>> t;
  if (batch_tile(op) == 32) {
    t.push_back({32, def_rows});
    t.push_back({32, sgk::kBandRowsSmall});
    if (op.tile == 0) t.push_back({16, 0});
  } else {
    t.push_back({16, 0});
  }
  return t;
}

// Byte layout of the batch: the problems' own workspaces first, then the
// shared region. Returns false if a problem is rejected.
struct BatchPlan {
  std::vector<size_t> ws_off, ws_size;
  size_t o_N, o_tab, o_sc, o_active, o_pdeg, o_part, o_consts, o_sets, o_pcg_part, o_arr, o_iters, o_status, o_sticky;
  std::vector<int> set_ncols;
  std::vector<long> set_nwork;
  size_t set_bytes = 0;
  long ncols_max = 0, nwork_max = 0;
  size_t total = 0;
};

size_t set_stride(long ncols) {
  // per column: nx, ntx, ntiles, prob, list entry (int), tbase, list base (long) and eight
  // pointers; plus the two list totals and the alignment of the 17 arrays
  return (size_t)ncols * (5 * sizeof(int) + 2 * sizeof(long) + 8 * sizeof(void*)) + 20 * 256;
}

int make_batch_plan(int count, const sg_problem* probs, const sg_opts* op, BatchPlan& bp) {
  if (count <= 0) return fail(SG_EINVAL, "batch needs at least one problem");
  if (!probs || !op) return fail(SG_EINVAL, "null problems or options");
  if (op->precond != SG_PC_HSC && op->precond != SG_PC_MEAN && op->precond != SG_PC_BGS)
    return fail(SG_EINVAL, "a batch uses the HSC, the mean-based or the block Gauss-Seidel preconditioner");
  Layout L;
  int pmax = 0;
  for (int b = 0; b < count; ++b) {
    size_t bytes = 0;
    int rc = sg_workspace_bytes(&probs[b], op, &bytes);
    if (rc) return rc;
    bp.ws_off.push_back(L.take(bytes));
    bp.ws_size.push_back(bytes);
    pmax = std::max(pmax, probs[b].p);
  }
  bp.set_ncols.assign(pmax + 2, 0);
  bp.set_nwork.assign(pmax + 2, 0);
  const std::vector<std::pair<int, int>> tilings = batch_tilings(*op);
  for (int b = 0; b < count; ++b) {
    const std::vector<int> off = level_offsets(probs[b].M, probs[b].p);
    // tiles per column: the most over the tilings the autotuner may choose
    int nt = 0;
    for (const auto& tr : tilings) {
      int ntx = 0, ntt = 0;
      sgk::pcg_tiling(probs[b].n_e - 1, op->cheb_degree, tr.first, tr.second, ntx, ntt);
      nt = std::max(nt, ntt);
    }
    for (int l = 0; l <= probs[b].p; ++l) {
      bp.set_ncols[l] += off[l + 1] - off[l];
      bp.set_nwork[l] += (long)(off[l + 1] - off[l]) * nt;
    }
    bp.set_ncols[pmax + 1] += off.back();
    bp.set_nwork[pmax + 1] += (long)off.back() * nt;
  }
  for (int s = 0; s <= pmax + 1; ++s) {
    bp.ncols_max = std::max<long>(bp.ncols_max, bp.set_ncols[s]);
    bp.nwork_max = std::max(bp.nwork_max, bp.set_nwork[s]);
    bp.set_bytes += set_stride(bp.set_ncols[s]);
  }
  bp.o_N = L.take(sizeof(long) * count);
  bp.o_tab = L.take(sizeof(void*) * 8 * count);
  bp.o_sc = L.take(sizeof(sgk::BatchScal) * count);
  bp.o_active = L.take(sizeof(int) * count);
  bp.o_pdeg = L.take(sizeof(int) * count);
  bp.o_part = L.take(sizeof(double) * 2 * sgk::kBatchBlocks * count);
  bp.o_consts = L.take(sizeof(sgk::PcgConsts<double>) * count);
  bp.o_sets = L.take(bp.set_bytes);
  bp.o_pcg_part = L.take(sizeof(double) * sgk::kPcgPartials * std::max<long>(1, bp.nwork_max));
  bp.o_arr = L.take(sizeof(unsigned) * std::max<long>(1, bp.ncols_max));
  bp.o_iters = L.take(sizeof(int) * std::max<long>(1, bp.ncols_max));
  bp.o_status = L.take(sizeof(int));
  bp.o_sticky = L.take(sizeof(int));
  bp.total = L.total;
  return SG_OK;
}

// Device column set s for inner precision T, built on the host and uploaded
// into the set's part of the workspace.
template <typename T>
int build_set(sg_batch_ctx* B, int s, char* base, std::vector<char>& host, sgk::PcgCols<T>& cols, long& nwork) {
  std::vector<int> nx, ntx, ntiles, prob;
  std::vector<long> tbase;
  std::vector<const T*> pb;
  std::vector<T*> px, pr0, pr1, pp0, pp1, pq, pz;
  long w = 0;
  for (int b = 0; b < B->nprob; ++b) {
    sg_ctx* h = B->h[b];
    int j0, j1;
    if (s <= B->pmax) {
      if (h->p < s) continue;
      j0 = h->off[s];
      j1 = h->off[s + 1];
    } else {
      j0 = 0;
      j1 = h->P;
    }
    const long n = h->n;
    int t = 0, nt = 0;
    sgk::pcg_tiling(h->nx, B->degree, B->tile, B->rows, t, nt);
    T* rw = (T*)h->rw;
    T* zw = B->inner == 32 ? (T*)h->zw : (T*)h->z;
    for (int j = j0; j < j1; ++j) {
      const long slot = j - j0;
      nx.push_back(h->nx);
      ntx.push_back(t);
      ntiles.push_back(nt);
      tbase.push_back(w);
      w += nt;
      prob.push_back(b);
      pb.push_back(rw + (long)j * n);
      px.push_back(zw + (long)j * n);
      pr0.push_back((T*)h->pR0 + slot * n);
      pr1.push_back((T*)h->pR1 + slot * n);
      pp0.push_back((T*)h->pP0 + slot * n);
      pp1.push_back((T*)h->pP1 + slot * n);
      pq.push_back((T*)h->pQ + slot * n);
      pz.push_back((T*)h->pZ + slot * n);
    }
  }
  nwork = w;
  Layout L;
  auto put = [&](const void* src, size_t bytes) {
    const size_t o = L.take(bytes);
    if (host.size() < o + bytes) host.resize(o + bytes);
    if (bytes) std::memcpy(host.data() + o, src, bytes);
    return base + o;
  };
  const size_t nc = nx.size();
  cols.nx = (const int*)put(nx.data(), sizeof(int) * nc);
  cols.ntx = (const int*)put(ntx.data(), sizeof(int) * nc);
  cols.ntiles = (const int*)put(ntiles.data(), sizeof(int) * nc);
  cols.tbase = (const long*)put(tbase.data(), sizeof(long) * nc);
  cols.prob = (const int*)put(prob.data(), sizeof(int) * nc);
  cols.b = (const T* const*)put(pb.data(), sizeof(void*) * nc);
  cols.x = (T* const*)put(px.data(), sizeof(void*) * nc);
  cols.r0 = (T* const*)put(pr0.data(), sizeof(void*) * nc);
  cols.r1 = (T* const*)put(pr1.data(), sizeof(void*) * nc);
  cols.p0 = (T* const*)put(pp0.data(), sizeof(void*) * nc);
  cols.p1 = (T* const*)put(pp1.data(), sizeof(void*) * nc);
  cols.q = (T* const*)put(pq.data(), sizeof(void*) * nc);
  cols.z = (T* const*)put(pz.data(), sizeof(void*) * nc);
  cols.nwork = w;
  // list of the active columns, rebuilt on the device before every launch
  const std::vector<int> zero_i(nc + 1, 0);
  const std::vector<long> zero_l(nc + 1, 0);
  cols.act = (const int*)put(zero_i.data(), sizeof(int) * nc);
  cols.nact = (const int*)put(zero_i.data(), sizeof(int));
  cols.cbase = (const long*)put(zero_l.data(), sizeof(long) * nc);
  cols.nwork_act = (const long*)put(zero_l.data(), sizeof(long));
  B->set_ncols[s] = (int)nc;
  if (L.total > set_stride((long)nc)) return fail(SG_EINVAL, "internal: column set larger than planned");
  return SG_OK;
}

template <typename T>
std::vector<sgk::PcgCols<T>>& sets(sg_batch_ctx* B);
template <>
std::vector<sgk::PcgCols<double>>& sets<double>(sg_batch_ctx* B) { return B->cols64; }
template <>
std::vector<sgk::PcgCols<float>>& sets<float>(sg_batch_ctx* B) { return B->cols32; }

// Builds every ragged column set for the batch's current tiling (B->tile,
// B->rows) and uploads them into the set region; synchronises the stream.
int upload_sets(sg_batch_ctx* B) {
  B->cols64.clear();
  B->cols32.clear();
  B->set_ncols.assign(B->pmax + 2, 0);
  const auto* consts = B->sets_consts;
  for (int s = 0; s <= B->pmax + 1; ++s) {
    std::vector<char> blob;
    long nwork = 0;
    char* base = B->sets_base + B->set_off[s];
    int rc;
    if (B->inner == 32) {
      sgk::PcgCols<float> c{};
      rc = build_set<float>(B, s, base, blob, c, nwork);
      c.consts = (const sgk::PcgConsts<float>*)consts;
      c.active = B->V.active;
      B->cols32.push_back(c);
    } else {
      sgk::PcgCols<double> c{};
      rc = build_set<double>(B, s, base, blob, c, nwork);
      c.consts = (const sgk::PcgConsts<double>*)consts;
      c.active = B->V.active;
      B->cols64.push_back(c);
    }
    if (rc == SG_OK && nwork > B->set_nwork_cap[s]) rc = fail(SG_EINVAL, "inner tiling exceeds the planned work list");
    if (rc) return rc;
    if (!blob.empty()) SG_HIP(hipMemcpyAsync(base, blob.data(), blob.size(), hipMemcpyHostToDevice, B->stream));
    // the host blob is freed at the end of this iteration: wait for its copy
    SG_HIP(hipStreamSynchronize(B->stream));
  }
  return SG_OK;
}

// Ragged inner launch over column set s, restricted to problems of degree >= pmin;
// warm: start from the contents of X where the options allow it.
template <typename T>
int run_set(sg_batch_ctx* B, int s, int pmin = 0, bool warm = false) {
  const int ncols = B->set_ncols[s];
  if (ncols <= 0) return SG_OK;
  sgk::PcgArgs<T> a{};
  a.ncols = ncols;
  a.degree = B->degree;
  a.rows = B->rows;
  a.maxit = B->opts.inner_maxit;
  a.rtol = B->opts.inner_rtol > 0.0 ? B->opts.inner_rtol : 0.0;
  a.warm = warm && B->opts.warm_start && B->tile != 16;
  a.sc = B->sc;
  const sgk::PcgCols<T>& cols = sets<T>(B)[s];
  // only the columns of problems that still iterate take part in the launch
  sgk::launch_batch_compact(cols.prob, cols.ntiles, ncols, B->V.active, B->pdeg, pmin, const_cast<int*>(cols.act),
                            const_cast<int*>(cols.nact), const_cast<long*>(cols.cbase),
                            const_cast<long*>(cols.nwork_act), B->stream);
  SG_HIP(sgk::launch_pcg_ragged<T>(a, cols, B->tile, B->max_blocks, B->stream));
  sgk::launch_batch_count_iters(B->sc.iters, cols.act, cols.nact, cols.prob, ncols, B->V.sc, B->sc.status,
                                B->sticky, B->stream);
  return SG_OK;
}

// Algorithm 1 for every active problem, level steps shared across the batch.
template <typename T>
int batch_hsc(sg_batch_ctx* B) {
  auto zw = [&](sg_ctx* h) { return B->inner == 32 ? (T*)h->zw : (T*)h->z; };
  for (int l = B->pmax; l >= 1; --l) {
    int rc = run_set<T>(B, l);  // y_l = D_l^-1 r_l^l
    if (rc) return rc;
    for (sg_ctx* h : B->h)
      if (h->p >= l) sgh::coupling<T>(h, l, 0, (T*)h->rw, zw(h));  // g_{l-1} = r_l^{l-1} - B_l y_l
  }
  int rc = run_set<T>(B, 0);  // A_0 u_0 = g_0
  if (rc) return rc;
  for (int l = 1; l <= B->pmax; ++l) {
    for (sg_ctx* h : B->h)
      if (h->p >= l) sgh::coupling<T>(h, l, 1, (T*)h->rw, zw(h));  // w = r_l^l - C_l u_{l-1}
    rc = run_set<T>(B, l, 0, true);  // u_l^l = D_l^-1 w, warm from y_l
    if (rc) return rc;
  }
  return SG_OK;
}

// Block symmetric Gauss-Seidel for every active problem, level steps shared
// across the batch (forward l = 0..pmax, backward l = pmax-1..0).
template <typename T>
int batch_bgs(sg_batch_ctx* B) {
  auto zw = [&](sg_ctx* h) { return B->inner == 32 ? (T*)h->zw : (T*)h->z; };
  int rc = run_set<T>(B, 0);
  if (rc) return rc;
  for (int l = 1; l <= B->pmax; ++l) {
    for (sg_ctx* h : B->h)
      if (h->p >= l) sgh::coupling<T>(h, l, 1, (T*)h->rw, zw(h));
    rc = run_set<T>(B, l);
    if (rc) return rc;
  }
  for (int l = B->pmax - 1; l >= 0; --l) {
    // problems whose top level is l keep their forward values on level l
    for (sg_ctx* h : B->h)
      if (h->p >= l + 1) sgh::coupling<T>(h, l + 1, 0, (T*)h->rw, zw(h));
    rc = run_set<T>(B, l, l + 1, true);  // z_l, warm from z'_l
    if (rc) return rc;
  }
  return SG_OK;
}

// One outer iteration of every active problem (no host synchronisation).
int iteration(sg_batch_ctx* B, int pc) {
  int rc = SG_OK;
  if (B->inner == 32) {
    sgk::launch_batch_to_inner<float>(B->V, B->stream);
    rc = pc == SG_PC_HSC ? batch_hsc<float>(B) : pc == SG_PC_BGS ? batch_bgs<float>(B) : run_set<float>(B, B->pmax + 1);
    if (rc) return rc;
    sgk::launch_batch_from_inner(B->V, B->stream);
  } else {
    sgk::launch_batch_to_inner<double>(B->V, B->stream);
    rc = pc == SG_PC_HSC ? batch_hsc<double>(B) : pc == SG_PC_BGS ? batch_bgs<double>(B) : run_set<double>(B, B->pmax + 1);
    if (rc) return rc;
  }
  sgk::launch_batch_dot_zq(B->V, B->stream);
  sgk::launch_batch_dirupdate(B->V, B->stream);
  for (sg_ctx* h : B->h) sgh::matvec(h, h->pv, h->q);
  sgk::launch_batch_dot_pq_pr(B->V, B->stream);
  sgk::launch_batch_update(B->V, B->stream);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

void drop_graph(sg_batch_ctx* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  B->graph_pc = -1;
}

int capture(sg_batch_ctx* B, int pc) {
  drop_graph(B);
  SG_HIP(hipStreamBeginCapture(B->stream, hipStreamCaptureModeRelaxed));
  const int rc = iteration(B, pc);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(B->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(SG_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  B->graph = g;
  SG_HIP(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0));
  B->graph_pc = pc;
  return SG_OK;
}

}  // namespace

extern "C" {

int sg_batch_workspace_bytes(int32_t count, const sg_problem* probs, const sg_opts* opts, size_t* bytes) {
  if (!bytes) return fail(SG_EINVAL, "null bytes");
  BatchPlan bp;
  int rc = make_batch_plan(count, probs, opts, bp);
  if (rc) return rc;
  *bytes = bp.total;
  return SG_OK;
}

int sg_batch_setup(int32_t count, const sg_problem* probs, const sg_opts* opts, void* workspace,
                   size_t workspace_bytes, void* stream, sg_batch* out) {
  if (!out || !workspace) return fail(SG_EINVAL, "null workspace or handle pointer");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(SG_EINVAL, "workspace must be 256-byte aligned");
  BatchPlan bp;
  int rc = make_batch_plan(count, probs, opts, bp);
  if (rc) return rc;
  if (workspace_bytes < bp.total) return fail(SG_ENOMEM, "workspace too small");
  sg_batch_ctx* B = new (std::nothrow) sg_batch_ctx();
  if (!B) return fail(SG_ENOMEM, "host allocation failed");
  char* w = (char*)workspace;
  B->nprob = count;
  B->opts = *opts;
  B->stream = (hipStream_t)stream;
  B->inner = opts->inner_precision;
  B->tile = batch_tile(*opts);
  B->rows = sgk::band_rows(opts->inner_precision, opts->cheb_degree);
  for (int b = 0; b < count; ++b) {
    sg_handle hb = nullptr;
    rc = sg_setup(&probs[b], opts, w + bp.ws_off[b], bp.ws_size[b], stream, &hb);
    if (rc) {
      sg_batch_destroy(B);
      return rc;
    }
    B->h.push_back(hb);
    B->pmax = std::max(B->pmax, hb->p);
  }
  // one Chebyshev degree for the whole batch
  B->degree = sgh::effective_degree(B->h[0]);
  for (sg_ctx* h : B->h)
    if (sgh::effective_degree(h) != B->degree) {
      sg_batch_destroy(B);
      return fail(SG_EINVAL, "all problems of a batch need the same effective Chebyshev degree");
    }
  // shared region
  std::vector<long> N(count);
  std::vector<void*> tab(8 * (size_t)count, nullptr);
  for (int b = 0; b < count; ++b) {
    sg_ctx* h = B->h[b];
    N[b] = h->n * (long)h->P;
    tab[0 * count + b] = nullptr;  // x: set per solve
    tab[1 * count + b] = nullptr;  // f: set per solve
    tab[2 * count + b] = h->r;
    tab[3 * count + b] = h->z;
    tab[4 * count + b] = h->pv;
    tab[5 * count + b] = h->q;
    tab[6 * count + b] = h->rw;
    tab[7 * count + b] = h->zw;
  }
  void** tab_d = (void**)(w + bp.o_tab);
  B->x_tab = (double**)(tab_d + 0 * count);
  B->f_tab = (const double**)(tab_d + 1 * count);
  sgk::BatchVecs& V = B->V;
  V.nprob = count;
  V.N = (const long*)(w + bp.o_N);
  V.x = (double* const*)(tab_d + 0 * count);
  V.f = (const double* const*)(tab_d + 1 * count);
  V.r = (double* const*)(tab_d + 2 * count);
  V.z = (double* const*)(tab_d + 3 * count);
  V.p = (double* const*)(tab_d + 4 * count);
  V.q = (double* const*)(tab_d + 5 * count);
  V.rw = (void* const*)(tab_d + 6 * count);
  V.zw = (void* const*)(tab_d + 7 * count);
  V.sc = (sgk::BatchScal*)(w + bp.o_sc);
  V.active = (int*)(w + bp.o_active);
  V.part = (double*)(w + bp.o_part);
  V.maxN = *std::max_element(N.begin(), N.end());
  for (int b = 0; b < count; ++b) B->h[b]->mask = V.active + b;
  // inner PCG constants per problem
  std::vector<char> consts(sizeof(sgk::PcgConsts<double>) * count);
  for (int b = 0; b < count; ++b) {
    if (B->inner == 32) {
      sgk::PcgArgs<float> a{};
      sgh::fill_pcg_consts<float>(B->h[b], a);
      sgk::PcgConsts<float> k{};
      k.c0 = a.c0;
      k.c1 = a.c1;
      k.inv_diag = a.inv_diag;
      k.inv_theta = a.inv_theta;
      k.w8 = a.w8;
      std::copy(a.chebA, a.chebA + sgk::kMaxCheb, k.chebA);
      std::copy(a.chebB, a.chebB + sgk::kMaxCheb, k.chebB);
      std::memcpy(consts.data() + sizeof(k) * b, &k, sizeof(k));
    } else {
      sgk::PcgArgs<double> a{};
      sgh::fill_pcg_consts<double>(B->h[b], a);
      sgk::PcgConsts<double> k{};
      k.c0 = a.c0;
      k.c1 = a.c1;
      k.inv_diag = a.inv_diag;
      k.inv_theta = a.inv_theta;
      k.w8 = a.w8;
      std::copy(a.chebA, a.chebA + sgk::kMaxCheb, k.chebA);
      std::copy(a.chebB, a.chebB + sgk::kMaxCheb, k.chebB);
      std::memcpy(consts.data() + sizeof(k) * b, &k, sizeof(k));
    }
  }
  // ragged column sets (built and uploaded after the shared tables)
  B->sets_base = w + bp.o_sets;
  B->sets_consts = w + bp.o_consts;
  B->set_nwork_cap = bp.set_nwork;
  B->set_off.clear();
  size_t set_off = 0;
  for (int s = 0; s <= B->pmax + 1; ++s) {
    B->set_off.push_back(set_off);
    set_off += set_stride(bp.set_ncols[s]);
  }
  B->sc.part = (double*)(w + bp.o_pcg_part);
  B->sc.arrivals = (unsigned*)(w + bp.o_arr);
  B->sc.iters = (int*)(w + bp.o_iters);
  B->sc.status = (int*)(w + bp.o_status);
  B->sticky = (int*)(w + bp.o_sticky);
  B->pdeg = (int*)(w + bp.o_pdeg);
  std::vector<int> pdeg(count);
  for (int b = 0; b < count; ++b) pdeg[b] = B->h[b]->p;
  hipStream_t s = B->stream;
  hipError_t e = hipMemcpyAsync(w + bp.o_N, N.data(), sizeof(long) * count, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(tab_d, tab.data(), sizeof(void*) * tab.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(w + bp.o_consts, consts.data(), consts.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(B->pdeg, pdeg.data(), sizeof(int) * count, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    sg_batch_destroy(B);
    return fail(SG_EDEVICE, std::string("batch upload failed: ") + hipGetErrorString(e));
  }
  rc = upload_sets(B);
  if (rc) {
    sg_batch_destroy(B);
    return rc;
  }
  *out = B;
  return SG_OK;
}

int sg_batch_sizes(sg_batch B, int32_t i, int64_t* n, int32_t* P) {
  if (!B || i < 0 || i >= B->nprob) return fail(SG_EINVAL, "bad batch or index");
  return sg_sizes(B->h[i], n, P, nullptr, nullptr);
}

int sg_batch_solve(sg_batch B, const double* const* F, double* const* U, double rtol, int32_t maxit,
                   int32_t use_graph, sg_stats* stats, double* ms_total) {
  if (!B || !F || !U) return fail(SG_EINVAL, "null batch or vector list");
  if (!(rtol >= 0.0) || maxit < 0) return fail(SG_EINVAL, "rtol must be >= 0 and maxit >= 0");
  for (int b = 0; b < B->nprob; ++b)
    if (!F[b] || !U[b]) return fail(SG_EINVAL, "null right-hand side or solution pointer");
  if (use_graph && B->stream == nullptr) return fail(SG_EINVAL, "graph capture needs a non-default stream");
  const int pc = B->opts.precond;
  const int nb = B->nprob;
  hipStream_t s = B->stream;
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<const void*> xs(U, U + nb), fs(F, F + nb);
  SG_HIP(hipMemcpyAsync(B->x_tab, xs.data(), sizeof(void*) * nb, hipMemcpyHostToDevice, s));
  SG_HIP(hipMemcpyAsync(B->f_tab, fs.data(), sizeof(void*) * nb, hipMemcpyHostToDevice, s));
  SG_HIP(hipMemsetAsync(B->sticky, 0, sizeof(int), s));
  sgk::launch_batch_init(B->V, rtol, s);
  std::vector<int> active(nb, 1);
  SG_HIP(hipMemcpyAsync(active.data(), B->V.active, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
  SG_HIP(hipStreamSynchronize(s));
  int iters = 0;
  for (int it = 0; it < maxit; ++it) {
    if (std::none_of(active.begin(), active.end(), [](int a) { return a != 0; })) break;
    if (use_graph && it >= 1) {
      if (!B->exec || B->graph_pc != pc) {
        int rc = capture(B, pc);
        if (rc) return rc;
      }
      SG_HIP(hipGraphLaunch(B->exec, s));
    } else {
      int rc = iteration(B, pc);
      if (rc) return rc;
    }
    ++iters;
    SG_HIP(hipMemcpyAsync(active.data(), B->V.active, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
    SG_HIP(hipStreamSynchronize(s));
  }
  int sticky = 0;
  SG_HIP(hipMemcpyAsync(&sticky, B->sticky, sizeof(int), hipMemcpyDeviceToHost, s));
  std::vector<sgk::BatchScal> S(nb);
  SG_HIP(hipMemcpyAsync(S.data(), B->V.sc, sizeof(sgk::BatchScal) * nb, hipMemcpyDeviceToHost, s));
  SG_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (ms_total) *ms_total = ms;
  if (sticky) return fail(SG_EDEVICE, "inner solver: a bounded column wait expired");
  int worst = SG_OK;
  for (int b = 0; b < nb; ++b) {
    sg_ctx* h = B->h[b];
    if (S[b].status == SG_BREAKDOWN) worst = SG_BREAKDOWN;
    else if (S[b].status == SG_NOT_CONVERGED && worst == SG_OK) worst = SG_NOT_CONVERGED;
    if (!stats) continue;
    sg_stats st{};
    st.outer_it = S[b].it;
    st.status = S[b].status;
    st.inner_it_total = S[b].inner_it;
    long nbmv = 0;
    for (int l = 1; l <= h->p; ++l) nbmv += sgh::coupling_blocks(h, l, 0) + sgh::coupling_blocks(h, l, 1);
    const long top = h->off[h->p + 1] - h->off[h->p];
    st.n_blockmv = pc == SG_PC_MEAN ? 0 : (long)S[b].it * nbmv;
    st.n_blocksolve = (long)S[b].it * (pc == SG_PC_HSC ? 2L * (h->P - 1) + 1 : pc == SG_PC_BGS ? 2L * h->P - top : (long)h->P);
    st.relres = S[b].fn2 > 0.0 ? std::sqrt(S[b].rr / S[b].fn2) : 0.0;
    st.ms = ms;
    // true residual ||f - A u|| / ||f|| of the returned iterate
    const int* mask = h->mask;
    h->mask = nullptr;
    sgh::matvec(h, U[b], h->tmp);
    sgk::launch_sub(h->tmp, F[b], h->tmp, h->n * (long)h->P, s);
    h->mask = mask;
    int rc = sgh::dots(h, 1, h->tmp, h->tmp);
    if (rc) return rc;
    st.true_relres = S[b].fn2 > 0.0 ? std::sqrt(h->host_out[0] / S[b].fn2) : 0.0;
    stats[b] = st;
  }
  (void)iters;
  if (worst == SG_NOT_CONVERGED) sgh::fail(SG_NOT_CONVERGED, "a batch member did not converge");
  if (worst == SG_BREAKDOWN) sgh::fail(SG_BREAKDOWN, "breakdown in a batch member");
  return worst;
}

int sg_batch_autotune(sg_batch B, int32_t flags, sg_tune_report* report) {
  if (!B) return fail(SG_EINVAL, "null batch");
  if (flags & ~3) return fail(SG_EINVAL, "flags: bit 0 = SG operators, bit 1 = inner launches");
  drop_graph(B);  // a new schedule needs a new capture
  hipStream_t s = B->stream;
  sg_tune_report R{};
  // every problem takes part while the candidates are timed
  std::vector<int> ones(B->nprob, 1);
  SG_HIP(hipMemcpyAsync(B->V.active, ones.data(), sizeof(int) * B->nprob, hipMemcpyHostToDevice, s));
  SG_HIP(hipStreamSynchronize(s));
  if (flags & 1)
    for (sg_ctx* h : B->h) {
      sg_tune_report r{};
      const int rc = sg_autotune(h, 1, &r);
      if (rc) return rc;
      R.candidates += r.candidates;
      R.mv_ms += r.mv_ms;
    }
  if (flags & 2) {
    // a constant right-hand side in every problem's inner input
    for (sg_ctx* h : B->h) {
      const long N = h->n * (long)h->P;
      sgk::launch_fill(h->pv, 1.0, N, s);
      if (B->inner == 32) sgk::launch_copy_d2f((float*)h->rw, h->pv, N, s);
      else sgk::launch_copy_d2d((double*)h->rw, h->pv, N, s);
    }
    const int pc = B->opts.precond;
    hipEvent_t e0 = B->h[0]->ev0, e1 = B->h[0]->ev1;
    // one inner solve of every set a preconditioner action works on: the
    // degree levels (HSC, block Gauss-Seidel) or all columns (mean-based)
    auto pass = [&]() -> int {
      const int first = pc == SG_PC_MEAN ? B->pmax + 1 : 0, last = pc == SG_PC_MEAN ? B->pmax + 1 : B->pmax;
      for (int set = first; set <= last; ++set) {
        const int rc = B->inner == 32 ? run_set<float>(B, set) : run_set<double>(B, set);
        if (rc) return rc;
      }
      return SG_OK;
    };
    int bt = B->tile, br = B->rows, bb = B->max_blocks;
    double best = 1e300;
    const int ncu = B->h[0]->num_cu;
    for (const auto& tr : batch_tilings(B->opts))
      for (int mb : {0, std::max(1, ncu / 2)}) {
        B->tile = tr.first;
        B->rows = tr.first == 16 ? B->rows : tr.second;
        B->max_blocks = mb;
        int rc = upload_sets(B);
        if (rc) return rc;
        if ((rc = pass())) return rc;  // warm-up
        std::vector<float> t;
        for (int rep = 0; rep < 3; ++rep) {
          SG_HIP(hipEventRecord(e0, s));
          if ((rc = pass())) return rc;
          SG_HIP(hipEventRecord(e1, s));
          SG_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          SG_HIP(hipEventElapsedTime(&ms, e0, e1));
          t.push_back(ms);
        }
        std::sort(t.begin(), t.end());
        ++R.candidates;
        if (t[1] < best) {
          best = t[1];
          bt = B->tile;
          br = B->rows;
          bb = mb;
        }
      }
    B->tile = bt;
    B->rows = br;
    B->max_blocks = bb;
    const int rc = upload_sets(B);
    if (rc) return rc;
    R.pcg_ms = best;
  }
  // the schedule of the largest member stands for the SG operators
  sg_ctx* big = B->h[0];
  for (sg_ctx* h : B->h)
    if (h->n * (long)h->P > big->n * (long)big->P) big = h;
  R.mv_variant = big->mv_variant;
  R.mv_param = sgh::mv_param(big);
  R.pcg_tile = B->tile;
  R.pcg_max_blocks = B->max_blocks;
  R.pcg_rows = B->tile == 16 ? 16 : B->rows;
  if (report) *report = R;
  return SG_OK;
}

void sg_batch_destroy(sg_batch B) {
  if (!B) return;
  drop_graph(B);
  for (sg_ctx* h : B->h) sg_destroy(h);
  delete B;
}

}  // extern "C"
