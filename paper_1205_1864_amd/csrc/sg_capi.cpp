// C interface of the SG solver library: setup of the chaos tables and the
// workspace, and the host drivers of the flexible CG (Section 5), the
// hierarchical Schur complement preconditioner (Algorithm 1), the mean-based
// and block symmetric Gauss-Seidel preconditioners (Section 6) and the
// adjoint gradient.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "sg_host.h"
#include "sg_internal.h"

namespace sgh {

thread_local std::string g_last_error = "no error";

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

long binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Multi-indices of total degree <= p, graded, descending lexicographic within a degree.
void multi_indices(int M, int p, std::vector<int>& out, std::vector<int>& off) {
  out.clear();
  off.assign(1, 0);
  std::vector<int> cur(M, 0);
  for (int d = 0; d <= p; ++d) {
    long count = 0;
    if (M == 0) {
      if (d == 0) count = 1;
    } else {
      // iterative enumeration: fill positions left to right with the largest value first
      std::vector<int> rem(M + 1, 0);
      std::function<void(int, int)> rec = [&](int k, int remaining) {
        if (k == M - 1) {
          cur[k] = remaining;
          out.insert(out.end(), cur.begin(), cur.end());
          ++count;
          return;
        }
        for (int v = remaining; v >= 0; --v) {
          cur[k] = v;
          rec(k + 1, remaining - v);
        }
      };
      rec(0, d);
    }
    off.push_back(off.back() + (int)count);
  }
}

struct Layout {
  size_t total = 0;
  size_t take(size_t bytes) {
    size_t o = total;
    total += (bytes + 255) / 256 * 256;
    return o;
  }
};

struct Plan {
  int P, nx;
  long n;
  int nlo, nup, npairs;
  int maxcols, ntiles_max;
  size_t o_a64, o_a32, o_c64;
  size_t o_lo_ptr, o_lo_ent, o_lo_g64, o_lo_g32, o_up_ptr, o_up_ent, o_up_g64, o_up_g32;
  size_t o_st_lo, o_st_up, o_st_glo64, o_st_gup64, o_st_glo32, o_st_gup32;
  size_t o_en_ptr, o_en_k, o_en_lo, o_en_up, o_en_glo64, o_en_gup64, o_en_glo32, o_en_gup32;
  size_t o_pair_ptr, o_pair_a, o_pair_b, o_pair_g;
  size_t o_mj_ptr, o_mj_rows, o_mj_kind, o_mj_lk, o_mj_lcol, o_mj_lw;
  size_t o_stg_terms, o_stg_slots, o_stg_wslot;
  size_t o_vec[7];
  size_t o_rw, o_zw;
  size_t o_pcg[6];
  size_t o_part, o_arr, o_iters, o_status;
  size_t o_red_part, o_red_out;
  size_t total;
};

int validate(const sg_problem* pr, const sg_opts* op) {
  if (!pr || !op) return fail(SG_EINVAL, "null problem or options");
  if (pr->n_e < 3) return fail(SG_EINVAL, "n_e must be >= 3");
  if (pr->n_e > 8192) return fail(SG_EINVAL, "n_e must be <= 8192");
  if (pr->M < 0 || pr->p < 0) return fail(SG_EINVAL, "M and p must be >= 0");
  if (pr->p + 1 > sgk::kMaxLevels) return fail(SG_EINVAL, "p must be < 16");
  if (binom(pr->M + pr->p, pr->p) > (1L << 20)) return fail(SG_EINVAL, "P = C(M+p, p) exceeds 2^20");
  if (pr->M > 2047) return fail(SG_EINVAL, "M must be < 2048");
  if (!(pr->theta0 > 0.0) || !std::isfinite(pr->theta0)) return fail(SG_EINVAL, "theta0 must be positive");
  if (!(pr->sigma >= 0.0) || !std::isfinite(pr->sigma)) return fail(SG_EINVAL, "sigma must be >= 0");
  if (pr->family != SG_FAMILY_HERMITE && pr->family != SG_FAMILY_LEGENDRE)
    return fail(SG_EINVAL, "family must be SG_FAMILY_HERMITE or SG_FAMILY_LEGENDRE");
  if (pr->M > 0 && (!pr->s || !pr->phi)) return fail(SG_EINVAL, "null s or phi");
  if (op->inner_precision != 32 && op->inner_precision != 64)
    return fail(SG_EINVAL, "inner_precision must be 32 or 64");
  if (op->cheb_degree < 1 || op->cheb_degree > sgk::kMaxCheb) return fail(SG_EINVAL, "cheb_degree must be 1..16");
  if (op->inner_maxit < 1) return fail(SG_EINVAL, "inner_maxit must be >= 1");
  if (op->precond < SG_PC_NONE || op->precond > SG_PC_BGS) return fail(SG_EINVAL, "unknown preconditioner");
  if (op->tile != 0 && op->tile != 16 && op->tile != 32) return fail(SG_EINVAL, "tile must be 0, 16 or 32");
  if (op->warm_start != 0 && op->warm_start != 1) return fail(SG_EINVAL, "warm_start must be 0 or 1");
  if (!(op->inner_rtol < 1.0) || std::isnan(op->inner_rtol)) return fail(SG_EINVAL, "inner_rtol must be < 1");
  if (op->use_graph != 0 && op->use_graph != 1) return fail(SG_EINVAL, "use_graph must be 0 or 1");
  if (op->reserved != 0) return fail(SG_EINVAL, "reserved must be 0");
  return SG_OK;
}

void make_plan(const sg_problem* pr, const sg_opts* op, Plan& pl) {
  const int M = pr->M, p = pr->p;
  pl.P = (int)binom(M + p, p);
  pl.nx = pr->n_e - 1;
  pl.n = (long)pl.nx * pl.nx;
  const long ne2 = (long)pr->n_e * pr->n_e;
  // each row has at most M lower and M upper neighbours; exact counts from the level sizes
  long nlo = 0;
  std::vector<int> al, off;
  multi_indices(M, p, al, off);
  for (int a = 0; a < pl.P; ++a)
    for (int k = 0; k < M; ++k)
      if (al[(long)a * M + k] > 0) ++nlo;
  pl.nlo = (int)nlo;
  pl.nup = (int)nlo;  // every lower entry (a, a - e_k) is an upper entry of a - e_k
  pl.npairs = 2 * (int)nlo;
  pl.maxcols = pl.P;
  pl.ntiles_max = (int)(((pl.nx + 15) / 16) * ((pl.nx + 15) / 16));
  const size_t isz = op->inner_precision == 32 ? 4 : 8;
  const long nP = pl.n * (long)pl.P;
  Layout L;
  pl.o_a64 = L.take(sizeof(double) * M * ne2);
  pl.o_a32 = L.take(sizeof(float) * M * ne2);
  pl.o_c64 = L.take(sizeof(double) * M * ne2);
  pl.o_lo_ptr = L.take(sizeof(int) * (pl.P + 1));
  pl.o_lo_ent = L.take(sizeof(int) * std::max(1, pl.nlo));
  pl.o_lo_g64 = L.take(sizeof(double) * std::max(1, pl.nlo));
  pl.o_lo_g32 = L.take(sizeof(float) * std::max(1, pl.nlo));
  pl.o_up_ptr = L.take(sizeof(int) * (pl.P + 1));
  pl.o_up_ent = L.take(sizeof(int) * std::max(1, pl.nup));
  pl.o_up_g64 = L.take(sizeof(double) * std::max(1, pl.nup));
  pl.o_up_g32 = L.take(sizeof(float) * std::max(1, pl.nup));
  const long PM = std::max<long>(1, (long)pl.P * M);
  pl.o_st_lo = L.take(sizeof(int) * PM);
  pl.o_st_up = L.take(sizeof(int) * PM);
  pl.o_st_glo64 = L.take(sizeof(double) * PM);
  pl.o_st_gup64 = L.take(sizeof(double) * PM);
  pl.o_st_glo32 = L.take(sizeof(float) * PM);
  pl.o_st_gup32 = L.take(sizeof(float) * PM);
  pl.o_en_ptr = L.take(sizeof(int) * (pl.P + 1));
  pl.o_en_k = L.take(sizeof(int) * PM);
  pl.o_en_lo = L.take(sizeof(int) * PM);
  pl.o_en_up = L.take(sizeof(int) * PM);
  pl.o_en_glo64 = L.take(sizeof(double) * PM);
  pl.o_en_gup64 = L.take(sizeof(double) * PM);
  pl.o_en_glo32 = L.take(sizeof(float) * PM);
  pl.o_en_gup32 = L.take(sizeof(float) * PM);
  pl.o_pair_ptr = L.take(sizeof(int) * (M + 1));
  pl.o_pair_a = L.take(sizeof(int) * std::max(1, pl.npairs));
  pl.o_pair_b = L.take(sizeof(int) * std::max(1, pl.npairs));
  pl.o_pair_g = L.take(sizeof(double) * std::max(1, pl.npairs));
  // row groups of the y-marching operator: the matvec (P rows) and the 2p coupling
  // products (two levels each), at most one group per row
  const long mj_rows = 3L * pl.P;
  pl.o_mj_ptr = L.take(sizeof(int) * (mj_rows + 2L * p + 2));
  pl.o_mj_rows = L.take(sizeof(int) * mj_rows);
  pl.o_mj_kind = L.take(sizeof(int) * mj_rows);
  pl.o_mj_lk = L.take(sizeof(int) * mj_rows * sgk::kMarchNS);
  pl.o_mj_lcol = L.take(sizeof(int) * mj_rows * sgk::kMarchRGL * sgk::kMarchNS);
  pl.o_mj_lw = L.take(sizeof(double) * mj_rows * sgk::kMarchRGL * sgk::kMarchNS);
  // row-staged operator: output pairs and their (padded) term lists
  const long stg_slots = std::max(1, pl.P);
  pl.o_stg_terms = L.take(sizeof(sgk::StageTerm) * (pl.P + 1L) * (2L * M + 1));
  pl.o_stg_slots = L.take(sizeof(sgk::StageSlot) * stg_slots);
  pl.o_stg_wslot = L.take(sizeof(int) * (sgk::kStageWaves + 1));
  for (int i = 0; i < 7; ++i) pl.o_vec[i] = L.take(sizeof(double) * nP);
  pl.o_rw = L.take(isz * nP);
  pl.o_zw = L.take(op->inner_precision == 32 ? isz * nP : 0);
  for (int i = 0; i < 6; ++i) pl.o_pcg[i] = L.take(isz * pl.n * (long)pl.maxcols);
  pl.o_part = L.take(sizeof(double) * sgk::kPcgPartials * (long)pl.maxcols * pl.ntiles_max);
  pl.o_arr = L.take(sizeof(unsigned) * pl.maxcols);
  pl.o_iters = L.take(sizeof(int) * pl.maxcols);
  pl.o_status = L.take(sizeof(int));
  const long nb_contract = (ne2 + 255) / 256;
  pl.o_red_part = L.take(sizeof(double) * std::max<long>(4L * sgk::kRedBlocks, nb_contract * (M + 1)));
  pl.o_red_out = L.take(sizeof(double) * std::max(64, M + 1));
  pl.total = L.total;
}

// Row groups of one use of the y-marching SG operator. Rows that use upper
// neighbours go into groups of kMarchRGU rows that carry all KL terms; the
// other rows are packed greedily, in order, into groups of at most kMarchRGL
// rows whose lower neighbours use at most kMarchNS distinct KL terms. The
// number of grid segments aims at one resident wave of blocks (cap_blocks).
struct HostMarchJob {
  std::vector<int> ptr, rows, kind, lk, lcol;
  std::vector<double> lw;
  int nseg = 8, seg_rows = 1;
};

void build_march_job(int M, int nx, const std::vector<int>& rows, bool lower, bool upper,
                     const std::vector<int>& st_lo, const std::vector<int>& st_up,
                     const std::vector<double>& st_glo, long cap_blocks, int seg_per_xcd, HostMarchJob& J) {
  const int RGU = sgk::kMarchRGU, RGL = sgk::kMarchRGL, NS = sgk::kMarchNS;
  std::vector<int> ru, rl;
  for (int r : rows) {
    bool has_up = false;
    for (int k = 0; k < M && upper; ++k) has_up = has_up || st_up[(size_t)r * M + k] >= 0;
    (has_up ? ru : rl).push_back(r);
  }
  J.ptr.assign(1, 0);
  J.rows.clear();
  J.kind.clear();
  J.lk.clear();
  J.lcol.clear();
  J.lw.clear();
  auto close = [&](int kind, const std::vector<int>& grp, const std::vector<int>& slots) {
    J.rows.insert(J.rows.end(), grp.begin(), grp.end());
    J.ptr.push_back((int)J.rows.size());
    J.kind.push_back(kind);
    for (int s = 0; s < NS; ++s) J.lk.push_back(s < (int)slots.size() ? slots[s] : -1);
    for (int j = 0; j < RGL; ++j)
      for (int s = 0; s < NS; ++s) {
        int col = -1;
        double w = 0.0;
        if (kind == 1 && j < (int)grp.size() && s < (int)slots.size() && lower) {
          const size_t e = (size_t)grp[j] * M + slots[s];
          col = st_lo[e];
          w = col >= 0 ? st_glo[e] : 0.0;
        }
        J.lcol.push_back(col);
        J.lw.push_back(w);
      }
  };
  for (size_t i = 0; i < ru.size(); i += RGU) {
    std::vector<int> grp(ru.begin() + i, ru.begin() + std::min(ru.size(), i + RGU));
    close(0, grp, {});
  }
  std::vector<int> grp, slots;
  for (int r : rl) {
    std::vector<int> need;
    for (int k = 0; k < M && lower; ++k)
      if (st_lo[(size_t)r * M + k] >= 0) need.push_back(k);
    std::vector<int> merged = slots;
    for (int k : need)
      if (std::find(merged.begin(), merged.end(), k) == merged.end()) merged.push_back(k);
    if (!grp.empty() && ((int)grp.size() == RGL || (int)merged.size() > NS)) {
      close(1, grp, slots);
      grp.clear();
      slots.clear();
      merged = need;
    }
    grp.push_back(r);
    slots = merged;
  }
  if (!grp.empty()) close(1, grp, slots);
  const long ng = std::max<long>(1, (long)J.kind.size());
  // segments per XCD: as many as one resident wave of blocks allows (or the requested
  // number), each at least 8 node rows tall
  long spx = seg_per_xcd > 0 ? seg_per_xcd : std::min<long>(nx / 64, cap_blocks / (8 * ng));
  spx = std::max<long>(1, std::min<long>(spx, nx / 64 > 0 ? nx / 64 : 1));
  J.nseg = (int)(8 * spx);
  J.seg_rows = (nx + J.nseg - 1) / J.nseg;
}

// Row groups of the y-marching SG operator for every use: job 0 is the matvec,
// job 1 + 2 (l - 1) + dir the coupling product of level l in direction dir.
// seg_per_xcd = 0 chooses the number of grid segments per XCD automatically.
// Tables of the row-staged full operator. The slot of an output applies its
// mean term (its own column, coefficient theta0); the term list holds the
// Galerkin neighbours (b, k, g), b = a -+ e_k with the weight g of G_k (which
// is symmetric), in ascending order of g. Two outputs share a slot (one per
// half wave) when their weight sequences are equal, so a term's weight is one
// value for both halves; an output left without a partner takes a slot alone.
// The slots go, largest first, to the least loaded wave. Uploads into the
// workspace and waits.
int build_stage_tables(sg_ctx* h, sgk::StageTerm* terms_d, sgk::StageSlot* slots_d, int* wslot_d) {
  h->stage_ok = false;
  const int P = h->P, M = h->M;
  // the kernel addresses the n x P blocks with 32-bit offsets; the tables use 16-bit indices
  if (P >= 0xFFFF || M > 255 || h->n * (long)P >= (1L << 31)) return SG_OK;
  struct Term {
    int b, k;
    double g;
  };
  std::vector<std::vector<Term>> tl(P);
  for (int a = 0; a < P; ++a) {
    for (int k = 0; k < M; ++k) {
      const int lo = h->st_lo_h[(size_t)a * M + k], up = h->st_up_h[(size_t)a * M + k];
      if (lo >= 0) tl[a].push_back({lo, k + 1, h->st_glo_h[(size_t)a * M + k]});
      if (up >= 0) tl[a].push_back({up, k + 1, h->st_glo_h[(size_t)up * M + k]});
    }
    std::stable_sort(tl[a].begin(), tl[a].end(), [](const Term& x, const Term& y) { return x.g < y.g; });
  }
  auto same_sig = [&](int x, int y) {
    if (tl[x].size() != tl[y].size()) return false;
    for (size_t t = 0; t < tl[x].size(); ++t)
      if (tl[x][t].g != tl[y][t].g) return false;
    return true;
  };
  auto sig_less = [&](int x, int y) {  // longer lists first, then by weight sequence
    if (tl[x].size() != tl[y].size()) return tl[x].size() > tl[y].size();
    for (size_t t = 0; t < tl[x].size(); ++t)
      if (tl[x][t].g != tl[y][t].g) return tl[x][t].g < tl[y][t].g;
    return x < y;
  };
  std::vector<int> order(P);
  for (int a = 0; a < P; ++a) order[a] = a;
  std::sort(order.begin(), order.end(), sig_less);
  struct Pair {
    int out[2];
    int nt;
  };
  std::vector<Pair> pairs;
  for (int i = 0; i < P;) {
    const bool two = i + 1 < P && same_sig(order[i], order[i + 1]);
    pairs.push_back({{order[i], two ? order[i + 1] : -1}, (int)tl[order[i]].size()});
    i += two ? 2 : 1;
  }
  std::stable_sort(pairs.begin(), pairs.end(), [](const Pair& x, const Pair& y) { return x.nt > y.nt; });
  // each slot goes to the least loaded wave with a free slot (a slot also costs
  // about eight terms of mean-term and element work)
  constexpr int NW = sgk::kStageWaves;
  std::vector<std::vector<int>> wav(NW);
  std::vector<long> load(NW, 0);
  for (size_t q = 0; q < pairs.size(); ++q) {
    int best = -1;
    for (int w2 = 0; w2 < NW; ++w2)
      if ((int)wav[w2].size() < sgk::kStageSlots && (best < 0 || load[w2] < load[best])) best = w2;
    if (best < 0) return SG_OK;  // more slots than the waves hold: the kernel is not used
    wav[best].push_back((int)q);
    load[best] += pairs[q].nt + 8;
  }
  std::vector<sgk::StageTerm> terms;
  std::vector<sgk::StageSlot> slots;
  std::vector<int> wslot(NW + 1, 0);
  for (int w2 = 0; w2 < NW; ++w2) {
    wslot[w2] = (int)slots.size();
    for (int q : wav[w2]) {
      const Pair& pr = pairs[q];
      if (terms.size() + pr.nt > 0xFFFF) return SG_OK;  // 16-bit term indices
      sgk::StageSlot sl{};
      sl.out[0] = (unsigned short)pr.out[0];
      sl.out[1] = pr.out[1] >= 0 ? (unsigned short)pr.out[1] : (unsigned short)0xFFFF;
      sl.t0 = (unsigned short)terms.size();
      sl.nt = (unsigned short)pr.nt;
      slots.push_back(sl);
      for (int t = 0; t < pr.nt; ++t) {
        sgk::StageTerm tm{};
        tm.g = tl[pr.out[0]][t].g;
        for (int hf = 0; hf < 2; ++hf) {
          const int a = pr.out[hf] >= 0 ? pr.out[hf] : pr.out[0];  // a lone output's idle half repeats it
          tm.b[hf] = (unsigned short)tl[a][t].b;
          tm.k[hf] = (unsigned char)tl[a][t].k;
        }
        terms.push_back(tm);
      }
    }
  }
  wslot[NW] = (int)slots.size();
  if ((long)terms.size() > (P + 1L) * (2L * M + 1) || (long)slots.size() > (long)P)
    return fail(SG_EINVAL, "internal: staged term list larger than planned");
  if (sgk::stage_lds_bytes(P, M, (int)terms.size(), (int)slots.size()) == 0) return SG_OK;  // does not fit LDS
  if (!terms.empty())
    SG_HIP(hipMemcpyAsync(terms_d, terms.data(), sizeof(sgk::StageTerm) * terms.size(), hipMemcpyHostToDevice,
                          h->stream));
  SG_HIP(hipMemcpyAsync(slots_d, slots.data(), sizeof(sgk::StageSlot) * slots.size(), hipMemcpyHostToDevice,
                        h->stream));
  SG_HIP(hipMemcpyAsync(wslot_d, wslot.data(), sizeof(int) * wslot.size(), hipMemcpyHostToDevice, h->stream));
  SG_HIP(hipStreamSynchronize(h->stream));
  h->stage.terms = terms_d;
  h->stage.slots = slots_d;
  h->stage.wslot = wslot_d;
  h->stage.P = P;
  h->stage.M = M;
  h->stage.nterms = (int)terms.size();
  h->stage.nslots = (int)slots.size();
  h->stage_ok = true;
  return SG_OK;
}

// Node rows per piece of the row-staged operator (0 turns it off).
void set_stage_rows(sg_ctx* h, int rows) {
  h->mv_stage = h->stage_ok && rows > 0 ? rows : 0;
  if (!h->mv_stage) return;
  h->stage.TY = rows;
  h->stage.nseg = (h->nx + sgk::kStageOut - 1) / sgk::kStageOut;
  h->stage.nyseg = (h->nx + rows - 1) / rows;
}

int build_march_jobs(sg_ctx* h, int seg_per_xcd) {
  h->march_ok = false;
  h->mjobs.clear();
  const bool piece = h->mv_variant == 3 && h->M <= sgk::kPieceMaxM;
  if (!piece && (!sgk::march_supported(h->n_e, h->M) || h->mv_variant != 2)) return SG_OK;
  const int occ = piece ? 1 : sgk::march_blocks_per_cu(h->M, h->n_e);
  if (occ <= 0) return SG_OK;
  const long cap = (long)occ * h->num_cu;
  const int M = h->M, P = h->P;
  std::vector<HostMarchJob> jobs(1 + 2 * h->p);
  std::vector<int> all(P);
  for (int a = 0; a < P; ++a) all[a] = a;
  build_march_job(M, h->nx, all, true, true, h->st_lo_h, h->st_up_h, h->st_glo_h, cap, seg_per_xcd, jobs[0]);
  for (int l = 1; l <= h->p; ++l)
    for (int dir = 0; dir < 2; ++dir) {
      const int rl = dir == 0 ? l - 1 : l;
      std::vector<int> rows;
      for (int a = h->off[rl]; a < h->off[rl + 1]; ++a) rows.push_back(a);
      build_march_job(M, h->nx, rows, dir == 1, dir == 0, h->st_lo_h, h->st_up_h, h->st_glo_h, cap, seg_per_xcd,
                      jobs[1 + 2 * (l - 1) + dir]);
    }
  std::vector<int> ptr, rws, knd, lk, lcol;
  std::vector<double> lw;
  for (const HostMarchJob& J : jobs) {
    sgk::MarchJob mj{};
    mj.gptr = h->mj_ptr_d + ptr.size();
    mj.grows = h->mj_rows_d;
    mj.gkind = h->mj_kind_d + knd.size();
    mj.lk = h->mj_lk_d + lk.size();
    mj.lcol = h->mj_lcol_d + lcol.size();
    mj.lw = h->mj_lw_d + lw.size();
    mj.ngroups = (int)J.kind.size();
    mj.nseg = J.nseg;
    mj.seg_rows = J.seg_rows;
    mj.piece = sgk::PieceGeom{0, 0, 0, 0, 0};
    if (piece) {
      // pieces of at most 62 output columns (one wavefront with its two halo
      // columns), as many as the grid width needs and equally wide
      const int nst = (h->nx + 61) / 62;
      const int W = (h->nx + nst - 1) / nst;
      const int TY = std::max(1, std::min(h->mv_piece_rows > 0 ? h->mv_piece_rows : 16, h->nx));
      mj.piece = sgk::PieceGeom{W, (h->nx + W - 1) / W, TY, (h->nx + TY - 1) / TY, h->mv_piece_waves};
    }
    h->mjobs.push_back(mj);
    const int base = (int)rws.size();
    for (int v : J.ptr) ptr.push_back(base + v);
    rws.insert(rws.end(), J.rows.begin(), J.rows.end());
    knd.insert(knd.end(), J.kind.begin(), J.kind.end());
    lk.insert(lk.end(), J.lk.begin(), J.lk.end());
    lcol.insert(lcol.end(), J.lcol.begin(), J.lcol.end());
    lw.insert(lw.end(), J.lw.begin(), J.lw.end());
  }
  hipStream_t s = h->stream;
  SG_HIP(hipMemcpyAsync(h->mj_ptr_d, ptr.data(), sizeof(int) * ptr.size(), hipMemcpyHostToDevice, s));
  SG_HIP(hipMemcpyAsync(h->mj_rows_d, rws.data(), sizeof(int) * rws.size(), hipMemcpyHostToDevice, s));
  SG_HIP(hipMemcpyAsync(h->mj_kind_d, knd.data(), sizeof(int) * knd.size(), hipMemcpyHostToDevice, s));
  SG_HIP(hipMemcpyAsync(h->mj_lk_d, lk.data(), sizeof(int) * lk.size(), hipMemcpyHostToDevice, s));
  SG_HIP(hipMemcpyAsync(h->mj_lcol_d, lcol.data(), sizeof(int) * lcol.size(), hipMemcpyHostToDevice, s));
  SG_HIP(hipMemcpyAsync(h->mj_lw_d, lw.data(), sizeof(double) * lw.size(), hipMemcpyHostToDevice, s));
  SG_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
  h->march_ok = true;
  h->mv_seg_per_xcd = piece ? 0 : seg_per_xcd;
  return SG_OK;
}

// Spectrum of D^-1 K_0 for the Q1 stencil: (8 - 2 c_i - 2 c_j - 4 c_i c_j) / 8, c_i = cos(i pi / n_e).
void cheb_interval(int n_e, double& lmin, double& lmax) {
  lmin = 1e300;
  lmax = -1e300;
  std::vector<double> c(n_e - 1);
  for (int i = 1; i < n_e; ++i) c[i - 1] = std::cos(i * M_PI / n_e);
  for (int i = 0; i < n_e - 1; ++i)
    for (int j = 0; j < n_e - 1; ++j) {
      const double l = (8.0 - 2.0 * c[i] - 2.0 * c[j] - 4.0 * c[i] * c[j]) / 8.0;
      lmin = std::min(lmin, l);
      lmax = std::max(lmax, l);
    }
}

template <typename T>
void fill_pcg_consts(const sg_ctx* h, sgk::PcgArgs<T>& a) {
  const double lmin = h->lmin, lmax = h->lmax;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double diag = h->theta0 * 8.0 / 3.0;
  a.c0 = (T)diag;
  a.c1 = (T)(-h->theta0 / 3.0);
  a.inv_diag = (T)(1.0 / diag);
  a.inv_theta = (T)(1.0 / theta);
  a.w8 = (T)0.125;
  for (int j = 0; j < sgk::kMaxCheb; ++j) {
    a.chebA[j] = T(0);
    a.chebB[j] = T(0);
  }
  if (delta > 0.0) {
    const double sigma1 = theta / delta;
    double rho = 1.0 / sigma1;
    for (int j = 1; j < h->opts.cheb_degree; ++j) {
      const double rn = 1.0 / (2.0 * sigma1 - rho);
      a.chebA[j] = (T)(rn * rho);
      a.chebB[j] = (T)(2.0 * rn / delta);
      rho = rn;
    }
  }
}

template void fill_pcg_consts<double>(const sg_ctx*, sgk::PcgArgs<double>&);
template void fill_pcg_consts<float>(const sg_ctx*, sgk::PcgArgs<float>&);

int effective_degree(const sg_ctx* h) { return h->lmax - h->lmin > 0.0 ? h->opts.cheb_degree : 1; }

int choose_tile(const sg_ctx* h, int degree) {
  // banded tiles (code 32) up to the precision's band degree limit; beyond it
  // the halo does not fit one wavefront (or the band its registers), so 16 x 16 tiles
  if (h->opts.tile == 16) return 16;
  return degree <= sgk::kBandMaxDegree ? 32 : 16;
}

int flush_inner(sg_ctx* h);

// State vectors and scratch of the inner solver: by default the handle's part
// of the workspace; sg_inner_solve_static passes its own.
struct PcgBufs {
  void *R0, *R1, *P0, *P1, *Q, *Z;
  sgk::PcgScratch sc;
  int maxcols;
};

PcgBufs handle_bufs(const sg_ctx* h) {
  return {h->pR0, h->pR1, h->pP0, h->pP1, h->pQ, h->pZ, h->pcgsc, h->pcg_maxcols};
}

// Batched inner PCG on `ncols` contiguous columns (inner precision T). warm:
// start from the contents of X where the options allow it, else from zero.
template <typename T>
int run_pcg(sg_ctx* h, const T* B, T* X, int ncols, int level_for_stats, std::vector<int>* iters_out = nullptr,
            bool warm = false, const PcgBufs* bufs = nullptr) {
  if (ncols <= 0) return SG_OK;
  const PcgBufs buf = bufs ? *bufs : handle_bufs(h);
  if (ncols > buf.maxcols) return fail(SG_EINVAL, "too many columns for the inner solver");
  sgk::PcgArgs<T> a{};
  const int degree = effective_degree(h);
  const int tile = choose_tile(h, degree);
  a.nx = h->nx;
  a.n = h->n;
  a.ncols = ncols;
  a.B = B;
  a.X = X;
  a.R0 = (T*)buf.R0;
  a.R1 = (T*)buf.R1;
  a.P0 = (T*)buf.P0;
  a.P1 = (T*)buf.P1;
  a.Q = (T*)buf.Q;
  a.Z = (T*)buf.Z;
  a.sc = buf.sc;
  const int prec = sizeof(T) == 4 ? 32 : 64;
  // automatic tiles: the band height by the rule for launches with few tiles
  a.rows = tile != 16 && h->opts.tile == 0 ? sgk::pcg_band_rows(h->nx, degree, prec, ncols, h->num_cu)
                                            : sgk::band_rows(prec, degree);
  sgk::pcg_tiling(h->nx, degree, tile, a.rows, a.ntx, a.ntiles);
  a.degree = degree;
  a.maxit = h->opts.inner_maxit;
  a.rtol = h->opts.inner_rtol > 0.0 ? h->opts.inner_rtol : 0.0;
  a.warm = warm && h->opts.warm_start && tile != 16;
  fill_pcg_consts<T>(h, a);
  a.no_coop = h->capturing ? 1 : 0;
  // room for this launch's read-back, else settle the earlier ones first (not
  // possible inside a graph capture: the action is then too large to capture)
  if ((int)h->pending.size() >= sg_ctx::kMaxPending || (int)h->pending.size() * 2 + 2 > h->nev ||
      h->iters_used + ncols > h->iters_cap) {
    if (h->capturing) return fail(SG_EINVAL, "preconditioner action too large for graph capture");
    int rc = flush_inner(h);
    if (rc) return rc;
  }
  const int k = (int)h->pending.size();
  hipEvent_t e0 = h->evpool[2 * k], e1 = h->evpool[2 * k + 1];
  // events recorded by graph nodes cannot be timed: a captured action is timed as a whole
  const bool timed = !h->capturing;
  if (timed) SG_HIP(hipEventRecord(e0, h->stream));
  SG_HIP(sgk::launch_pcg<T>(a, tile, h->pcg_max_blocks, h->stream));
  if (timed) SG_HIP(hipEventRecord(e1, h->stream));
  sg_ctx::PendingLaunch L{ncols, level_for_stats, tile, a.warm, (int)sizeof(T), h->iters_used, timed};
  SG_HIP(hipMemcpyAsync(h->iters_host + L.slot, buf.sc.iters, sizeof(int) * ncols, hipMemcpyDeviceToHost,
                        h->stream));
  SG_HIP(hipMemcpyAsync(h->status_host + k, buf.sc.status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  h->pending.push_back(L);
  h->iters_used += ncols;
  if ((h->defer > 0 || h->capturing) && !iters_out) return SG_OK;
  if (iters_out) iters_out->assign(ncols, 0);
  const long slot = L.slot;
  int rc = flush_inner(h);
  if (rc) return rc;
  if (iters_out)
    for (int c = 0; c < ncols; ++c) (*iters_out)[c] = h->iters_host[slot + c];
  return SG_OK;
}

// Settles every inner launch still pending: waits for the stream, then checks
// each launch's status word and adds its iteration counts, algorithmic bytes
// and event time to the handle's statistics.
int flush_inner(sg_ctx* h) {
  if (h->pending.empty()) return SG_OK;
  SG_HIP(hipStreamSynchronize(h->stream));
  int bad = 0;
  for (size_t k = 0; k < h->pending.size(); ++k) {
    const sg_ctx::PendingLaunch& L = h->pending[k];
    if (h->status_host[k] != 0) bad = 1;
    if (L.timed) {
      float ms = 0.f;
      SG_HIP(hipEventElapsedTime(&ms, h->evpool[2 * k], h->evpool[2 * k + 1]));
      h->inner_ms_acc += ms;
    }
    h->inner_launch_acc += 1;
    int mx = 0;
    for (int c = 0; c < L.ncols; ++c) {
      const int v = h->iters_host[L.slot + c];
      h->inner_it_acc += v;
      // phase A reads z, p and x and writes p and x (and q with 16 x 16 tiles); phase B
      // reads r and p (q) and writes r and z; the start reads b and writes z and x (warm:
      // reads b and x, writes z and r); a column that stops after at least one iteration
      // reads x and p and writes x once more
      const double per_it = L.tile == 16 ? 10.0 : 9.0;
      h->inner_bytes_acc += (per_it * v + (v > 0 ? 6.0 : 3.0) + (L.warm ? 1.0 : 0.0)) * (double)h->n * L.wsize;
      mx = std::max(mx, v);
    }
    if (L.level >= 0 && L.level < sgk::kMaxLevels) h->inner_it_max[L.level] = std::max(h->inner_it_max[L.level], mx);
  }
  h->pending.clear();
  h->iters_used = 0;
  if (bad) return fail(SG_EDEVICE, "inner solver: a bounded column wait expired");
  return SG_OK;
}

// Defers the read-back of inner launches for the lifetime of the guard (one
// preconditioner action); the caller settles them with flush_inner.
struct DeferInner {
  sg_ctx* h;
  explicit DeferInner(sg_ctx* hh) : h(hh) { ++h->defer; }
  ~DeferInner() { --h->defer; }
};

template <typename T>
sgk::ChaosLists<T> lists(const sg_ctx* h);
template <>
sgk::ChaosLists<double> lists<double>(const sg_ctx* h) {
  return {h->lo_ptr_d, h->lo_ent_d, h->lo_g64, h->up_ptr_d, h->up_ent_d, h->up_g64};
}
template <>
sgk::ChaosLists<float> lists<float>(const sg_ctx* h) {
  return {h->lo_ptr_d, h->lo_ent_d, h->lo_g32, h->up_ptr_d, h->up_ent_d, h->up_g32};
}
template <typename T>
sgk::StripTables<T> strip_tables(const sg_ctx* h);
template <>
sgk::StripTables<double> strip_tables<double>(const sg_ctx* h) {
  return {h->st_lo_d, h->st_up_d, h->st_glo64, h->st_gup64, h->M, h->mv_blocks_per_band,
          h->en_ptr_d, h->en_k_d, h->en_lo_d, h->en_up_d, h->en_glo64, h->en_gup64, h->mv_variant};
}
template <>
sgk::StripTables<float> strip_tables<float>(const sg_ctx* h) {
  return {h->st_lo_d, h->st_up_d, h->st_glo32, h->st_gup32, h->M, h->mv_blocks_per_band,
          h->en_ptr_d, h->en_k_d, h->en_lo_d, h->en_up_d, h->en_glo32, h->en_gup32, h->mv_variant};
}

template <typename T>
const T* coefs(const sg_ctx* h);
template <>
const double* coefs<double>(const sg_ctx* h) { return h->a64; }
template <>
const float* coefs<float>(const sg_ctx* h) { return h->a32; }

// R[level l-1] -= B_l V[level l] (dir 0) or R[level l] -= C_l V[level l-1] (dir 1).
template <typename T>
void coupling(sg_ctx* h, int l, int dir, T* R, const T* V) {
  sgk::SgOpArgs<T> a{};
  a.n_e = h->n_e;
  a.nx = h->nx;
  a.n = h->n;
  const int rl = dir == 0 ? l - 1 : l;
  a.row0 = h->off[rl];
  a.nrows = h->off[rl + 1] - h->off[rl];
  a.use_lower = dir == 1;
  a.use_upper = dir == 0;
  a.diag = T(0);
  a.rcoef = T(1);
  a.sgn = T(-1);
  a.in = V;
  a.rsrc = R;
  a.out = R;
  a.a = coefs<T>(h);
  a.lists = lists<T>(h);
  a.active = h->mask;
  sgk::launch_sgop<T>(a, strip_tables<T>(h), h->march_ok ? &h->mjobs[1 + 2 * (l - 1) + dir] : nullptr, h->stream);
}

template void coupling<double>(sg_ctx*, int, int, double*, const double*);
template void coupling<float>(sg_ctx*, int, int, float*, const float*);

long coupling_blocks(const sg_ctx* h, int l, int dir) {
  const int rl = dir == 0 ? l - 1 : l;
  const std::vector<int>& ptr = dir == 0 ? h->up_ptr : h->lo_ptr;
  return ptr[h->off[rl + 1]] - ptr[h->off[rl]];
}

// Algorithm 1 in inner precision T over the levels 0..ptop: rw holds a copy of
// the residual, Zb receives M_P r (ptop = p) or M_{P-1} r of the reduced system
// (ptop = p - 1; only the columns of degree <= ptop are read and written).
template <typename T>
int hsc_core(sg_ctx* h, T* rw, T* Zb, long* nbmv, long* nbs, int ptop) {
  const long n = h->n;
  for (int l = ptop; l >= 1; --l) {
    const int lo = h->off[l], hi = h->off[l + 1];
    int rc = run_pcg<T>(h, rw + lo * n, Zb + lo * n, hi - lo, l);  // y_l = D_l^-1 r_l^l
    if (rc) return rc;
    coupling<T>(h, l, 0, rw, Zb);  // g_{l-1} = r_l^{l-1} - B_l y_l
    *nbs += hi - lo;
    *nbmv += coupling_blocks(h, l, 0);
  }
  int rc = run_pcg<T>(h, rw, Zb, 1, 0);  // A_0 u_0 = g_0
  if (rc) return rc;
  *nbs += 1;
  for (int l = 1; l <= ptop; ++l) {
    const int lo = h->off[l], hi = h->off[l + 1];
    coupling<T>(h, l, 1, rw, Zb);  // w = r_l^l - C_l u_{l-1}
    *nbmv += coupling_blocks(h, l, 1);
    // u_l^l = D_l^-1 w, from y_l of the down sweep when warm starts are on
    rc = run_pcg<T>(h, rw + lo * n, Zb + lo * n, hi - lo, l, nullptr, true);
    if (rc) return rc;
    *nbs += hi - lo;
  }
  return SG_OK;
}

// Block symmetric Gauss-Seidel action in inner precision T from a zero initial
// guess: rw holds a copy of the residual, Zb receives M_bGS r. Forward sweep
// l = 0..p, backward sweep l = p-1..0; rw keeps r_l - C_l z'_{l-1} from the
// forward sweep, so the backward sweep only subtracts B_{l+1} z_{l+1}.
template <typename T>
int bgs_core(sg_ctx* h, T* rw, T* Zb, long* nbmv, long* nbs) {
  const long n = h->n;
  int rc = run_pcg<T>(h, rw, Zb, 1, 0);  // z'_0 = K_0^-1 r_0
  if (rc) return rc;
  *nbs += 1;
  for (int l = 1; l <= h->p; ++l) {
    const int lo = h->off[l], hi = h->off[l + 1];
    coupling<T>(h, l, 1, rw, Zb);  // r_l - C_l z'_{l-1}
    *nbmv += coupling_blocks(h, l, 1);
    rc = run_pcg<T>(h, rw + lo * n, Zb + lo * n, hi - lo, l);  // z'_l
    if (rc) return rc;
    *nbs += hi - lo;
  }
  for (int l = h->p - 1; l >= 0; --l) {
    const int lo = h->off[l], hi = h->off[l + 1];
    coupling<T>(h, l + 1, 0, rw, Zb);  // ... - B_{l+1} z_{l+1}
    *nbmv += coupling_blocks(h, l + 1, 0);
    // z_l, from z'_l of the forward sweep when warm starts are on
    rc = run_pcg<T>(h, rw + lo * n, Zb + lo * n, hi - lo, l, nullptr, true);
    if (rc) return rc;
    *nbs += hi - lo;
  }
  return SG_OK;
}

int apply_bgs_body(sg_ctx* h, const double* R, double* Z, long* nbmv, long* nbs) {
  const long N = h->n * (long)h->P;
  if (h->opts.inner_precision == 64) {
    double* rw = (double*)h->rw;
    sgk::launch_copy_d2d(rw, R, N, h->stream);
    return bgs_core<double>(h, rw, Z, nbmv, nbs);
  }
  float* rw = (float*)h->rw;
  float* zw = (float*)h->zw;
  sgk::launch_copy_d2f(rw, R, N, h->stream);
  int rc = bgs_core<float>(h, rw, zw, nbmv, nbs);
  if (rc) return rc;
  sgk::launch_copy_f2d(Z, zw, N, h->stream);
  return SG_OK;
}

int apply_hsc_body(sg_ctx* h, const double* R, double* Z, long* nbmv, long* nbs) {
  const long N = h->n * (long)h->P;
  if (h->opts.inner_precision == 64) {
    double* rw = (double*)h->rw;
    sgk::launch_copy_d2d(rw, R, N, h->stream);
    return hsc_core<double>(h, rw, Z, nbmv, nbs, h->p);
  }
  float* rw = (float*)h->rw;
  float* zw = (float*)h->zw;
  sgk::launch_copy_d2f(rw, R, N, h->stream);
  int rc = hsc_core<float>(h, rw, zw, nbmv, nbs, h->p);
  if (rc) return rc;
  sgk::launch_copy_f2d(Z, zw, N, h->stream);
  return SG_OK;
}

int apply_mean_body(sg_ctx* h, const double* R, double* Z, long* nbs) {
  const long N = h->n * (long)h->P;
  *nbs += h->P;
  if (h->opts.inner_precision == 64) return run_pcg<double>(h, R, Z, h->P, -1);
  float* rw = (float*)h->rw;
  float* zw = (float*)h->zw;
  sgk::launch_copy_d2f(rw, R, N, h->stream);
  int rc = run_pcg<float>(h, rw, zw, h->P, -1);
  if (rc) return rc;
  sgk::launch_copy_f2d(Z, zw, N, h->stream);
  return SG_OK;
}

// One preconditioner action with the inner launches' read-back settled once at its end.
int apply_bgs(sg_ctx* h, const double* R, double* Z, long* nbmv, long* nbs) {
  int rc;
  {
    DeferInner d(h);
    rc = apply_bgs_body(h, R, Z, nbmv, nbs);
  }
  const int rf = flush_inner(h);
  return rc ? rc : rf;
}

int apply_hsc(sg_ctx* h, const double* R, double* Z, long* nbmv, long* nbs) {
  int rc;
  {
    DeferInner d(h);
    rc = apply_hsc_body(h, R, Z, nbmv, nbs);
  }
  const int rf = flush_inner(h);
  return rc ? rc : rf;
}

int apply_mean(sg_ctx* h, const double* R, double* Z, long* nbs) {
  int rc;
  {
    DeferInner d(h);
    rc = apply_mean_body(h, R, Z, nbs);
  }
  const int rf = flush_inner(h);
  return rc ? rc : rf;
}

// Drops the captured preconditioner action (options or schedules changed).
void drop_pc_graph(sg_ctx* h) {
  if (h->pc_exec) (void)hipGraphExecDestroy(h->pc_exec);
  if (h->pc_graph) (void)hipGraphDestroy(h->pc_graph);
  h->pc_exec = nullptr;
  h->pc_graph = nullptr;
  h->pc_kind = -1;
  h->pc_pending.clear();
}

// One preconditioner action of kind pc replayed from a HIP graph: captured on
// the first call (or when the kind or the buffers change), then launched; the
// read-back records of the captured inner launches are settled after every
// replay exactly as after an eager action.
int apply_graph(sg_ctx* h, int pc, const double* R, double* Z, long* nbmv, long* nbs) {
  if (!h->stream) return fail(SG_EINVAL, "use_graph needs a stream other than the default stream");
  if (!h->pc_exec || h->pc_kind != pc || h->pc_R != R || h->pc_Z != Z) {
    drop_pc_graph(h);
    int rc = flush_inner(h);
    if (rc) return rc;
    long bm = 0, bs = 0;
    SG_HIP(hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
    h->capturing = true;
    if (pc == SG_PC_HSC) rc = apply_hsc_body(h, R, Z, &bm, &bs);
    else if (pc == SG_PC_BGS) rc = apply_bgs_body(h, R, Z, &bm, &bs);
    else rc = apply_mean_body(h, R, Z, &bs);
    h->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->stream, &g);
    std::vector<sg_ctx::PendingLaunch> recs = h->pending;
    const long used = h->iters_used;
    h->pending.clear();  // nothing of the capture has run
    h->iters_used = 0;
    if (rc || e != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      if (rc) return rc;
      return fail(SG_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(SG_EDEVICE, std::string("graph instantiation: ") + hipGetErrorString(ei));
    }
    h->pc_graph = g;
    h->pc_exec = x;
    h->pc_kind = pc;
    h->pc_R = R;
    h->pc_Z = Z;
    h->pc_pending = recs;
    h->pc_iters_used = used;
    h->pc_nbmv = bm;
    h->pc_nbs = bs;
  }
  SG_HIP(hipEventRecord(h->ev0, h->stream));
  SG_HIP(hipGraphLaunch(h->pc_exec, h->stream));
  SG_HIP(hipEventRecord(h->ev1, h->stream));
  h->pending = h->pc_pending;
  h->iters_used = h->pc_iters_used;
  if (nbmv) *nbmv += h->pc_nbmv;
  if (nbs) *nbs += h->pc_nbs;
  const int rc = flush_inner(h);  // synchronises the stream
  if (rc) return rc;
  float ms = 0.f;
  SG_HIP(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  h->inner_ms_acc += ms;  // the whole replayed action (its inner launches are not timed one by one)
  return SG_OK;
}

void matvec(sg_ctx* h, const double* U, double* Y) {
  sgk::SgOpArgs<double> a{};
  a.n_e = h->n_e;
  a.nx = h->nx;
  a.n = h->n;
  a.row0 = 0;
  a.nrows = h->P;
  a.use_lower = 1;
  a.use_upper = 1;
  a.diag = h->theta0;
  a.rcoef = 0.0;
  a.sgn = 1.0;
  a.in = U;
  a.rsrc = nullptr;
  a.out = Y;
  a.a = h->a64;
  a.lists = lists<double>(h);
  a.active = h->mask;
  if (h->mv_stage > 0) {
    sgk::launch_stage(a, h->stage, h->stream);
    return;
  }
  sgk::launch_sgop<double>(a, strip_tables<double>(h), h->march_ok ? &h->mjobs[0] : nullptr, h->stream);
}

int read_out(sg_ctx* h, int count) {
  if ((int)h->host_out.size() < count) h->host_out.resize(count);
  SG_HIP(hipMemcpyAsync(h->host_out.data(), h->red_out, sizeof(double) * count, hipMemcpyDeviceToHost, h->stream));
  SG_HIP(hipStreamSynchronize(h->stream));
  return SG_OK;
}

int dots_n(sg_ctx* h, long N, int nd, const double* a0, const double* b0, const double* a1 = nullptr,
           const double* b1 = nullptr, const double* a2 = nullptr, const double* b2 = nullptr) {
  const double* A[3] = {a0, a1, a2};
  const double* B[3] = {b0, b1, b2};
  sgk::launch_dots(A, B, nd, N, h->red_part, h->red_out, h->stream);
  return read_out(h, nd);
}

int dots(sg_ctx* h, int nd, const double* a0, const double* b0, const double* a1, const double* b1,
         const double* a2, const double* b2) {
  return dots_n(h, h->n * (long)h->P, nd, a0, b0, a1, b1, a2, b2);
}

double lanczos_kappa(const std::vector<double>& al, const std::vector<double>& be) {
  const int m = (int)al.size();
  if (m == 0) return 1.0;
  // symmetric tridiagonal eigenvalues by bisection (Sturm sequences)
  std::vector<double> d(m), e(m, 0.0);
  d[0] = 1.0 / al[0];
  for (int i = 1; i < m; ++i) {
    const double b = std::fabs(be[i - 1]);
    d[i] = 1.0 / al[i] + b / al[i - 1];
    e[i] = std::sqrt(b) / al[i - 1];
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = d[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < m; ++i) {
      if (q == 0.0) q = 1e-300;
      q = d[i] - x - e[i] * e[i] / q;
      if (q < 0) ++c;
    }
    return c;
  };
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    const double r = std::fabs(e[i]) + (i + 1 < m ? std::fabs(e[i + 1]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  auto kth = [&](int k) {  // k-th smallest eigenvalue, 0-based
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (a + b);
      if (count_below(mid) > k) b = mid; else a = mid;
    }
    return 0.5 * (a + b);
  };
  const double emin = kth(0), emax = kth(m - 1);
  return emax / emin;
}

struct Timer {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

// Outcome of a flexible CG run.
struct FcgRun {
  int status = SG_NOT_CONVERGED;
  int its = 0;
  double fn2 = 0.0, relres = 0.0;
  double ms_pc = 0.0, ms_mv = 0.0;
  std::vector<double> alphas, betas;
};

// Flexible CG with one stored direction on vectors of length N (prefixes of
// the handle's n x P vectors): op(x, y) sets y = A x, prec(r, z) sets z = M r.
// The vectors r, z, p and q of the handle hold the iteration.
int fcg_core(sg_ctx* h, long N, const double* F, double* U, double rtol, int maxit, int use_x0,
             const std::function<int(const double*, double*)>& op,
             const std::function<int(const double*, double*)>& prec, FcgRun& out) {
  int rc = dots_n(h, N, 1, F, F);
  if (rc) return rc;
  const double fn2 = h->host_out[0];
  out.fn2 = fn2;
  if (!std::isfinite(fn2)) return fail(SG_EINVAL, "right-hand side is not finite");
  double* r = h->r;
  double* z = h->z;
  double* p = h->pv;
  double* q = h->q;
  if (use_x0) {
    rc = op(U, h->tmp);
    if (rc) return rc;
    sgk::launch_sub(r, F, h->tmp, N, h->stream);
  } else {
    sgk::launch_fill(U, 0.0, N, h->stream);
    sgk::launch_copy_d2d(r, F, N, h->stream);
  }
  if (fn2 == 0.0) {
    sgk::launch_fill(U, 0.0, N, h->stream);
    out.status = SG_OK;
    return SG_OK;
  }
  rc = dots_n(h, N, 1, r, r);
  if (rc) return rc;
  out.relres = std::sqrt(h->host_out[0] / fn2);
  if (out.relres <= rtol) out.status = SG_OK;
  double pq_prev = 0.0;
  for (int it = 0; it < maxit && out.status == SG_NOT_CONVERGED; ++it) {
    Timer tp;
    rc = prec(r, z);
    if (rc) return rc;
    if (it == 0) {
      sgk::launch_copy_d2d(p, z, N, h->stream);
    } else {
      rc = dots_n(h, N, 1, z, q);
      if (rc) return rc;
      const double beta = -h->host_out[0] / pq_prev;
      out.betas.push_back(beta);
      sgk::launch_xpby(p, z, beta, N, h->stream);
    }
    SG_HIP(hipStreamSynchronize(h->stream));
    out.ms_pc += tp.ms();
    Timer tm;
    rc = op(p, q);
    if (rc) return rc;
    SG_HIP(hipStreamSynchronize(h->stream));
    out.ms_mv += tm.ms();
    rc = dots_n(h, N, 2, p, q, p, r);
    if (rc) return rc;
    const double pq = h->host_out[0], pr = h->host_out[1];
    if (!(pq > 0.0) || !std::isfinite(pq) || !std::isfinite(pr)) {
      out.status = SG_BREAKDOWN;
      break;
    }
    const double alpha = pr / pq;
    out.alphas.push_back(alpha);
    sgk::launch_fcg_update(U, r, p, q, alpha, N, h->red_part, h->red_out, h->stream);
    rc = read_out(h, 1);
    if (rc) return rc;
    pq_prev = pq;
    out.its = it + 1;
    out.relres = std::sqrt(h->host_out[0] / fn2);
    if (!std::isfinite(out.relres)) {
      out.status = SG_BREAKDOWN;
      break;
    }
    if (out.relres <= rtol) out.status = SG_OK;
  }
  return SG_OK;
}

void reset_inner_stats(sg_ctx* h) {
  h->inner_it_acc = 0;
  h->inner_ms_acc = 0.0;
  h->inner_bytes_acc = 0.0;
  h->inner_launch_acc = 0;
  for (int l = 0; l < sgk::kMaxLevels; ++l) h->inner_it_max[l] = 0;
}

// Relative true residual ||F - A U|| / ||F|| of the full system (uses tmp).
int full_true_relres(sg_ctx* h, const double* F, const double* U, double fn2, double* out) {
  const long N = h->n * (long)h->P;
  *out = 0.0;
  if (!(fn2 > 0.0)) return SG_OK;
  matvec(h, U, h->tmp);
  sgk::launch_sub(h->tmp, F, h->tmp, N, h->stream);
  int rc = dots(h, 1, h->tmp, h->tmp);
  if (rc) return rc;
  *out = std::sqrt(h->host_out[0] / fn2);
  return SG_OK;
}

int finish_stats(sg_ctx* h, const FcgRun& run, double true_rel, long nbmv, long nbs, const Timer& total,
                 sg_stats* st) {
  sg_stats S{};
  S.outer_it = run.its;
  S.status = run.status;
  S.inner_it_total = h->inner_it_acc;
  S.n_blockmv = nbmv;
  S.n_blocksolve = nbs;
  for (int l = 0; l < 16; ++l) S.inner_it_max[l] = h->inner_it_max[l];
  S.relres = run.relres;
  S.true_relres = true_rel;
  S.kappa_est = lanczos_kappa(run.alphas, run.betas);
  S.ms_inner = h->inner_ms_acc;
  S.inner_bytes = h->inner_bytes_acc;
  S.inner_launches = h->inner_launch_acc;
  S.ms_precond = run.ms_pc;
  S.ms_matvec = run.ms_mv;
  S.ms = total.ms();
  if (st) *st = S;
  if (run.status == SG_NOT_CONVERGED) g_last_error = "outer iteration did not converge";
  if (run.status == SG_BREAKDOWN) g_last_error = "breakdown: non-positive or non-finite curvature";
  return run.status;
}

// Flexible CG on the full system; preconditioner kind pc.
int fcg(sg_ctx* h, const double* F, double* U, double rtol, int maxit, int use_x0, int pc, sg_stats* st) {
  Timer total;
  const long N = h->n * (long)h->P;
  reset_inner_stats(h);
  long nbmv = 0, nbs = 0;
  auto op = [&](const double* x, double* y) {
    matvec(h, x, y);
    return SG_OK;
  };
  auto prec = [&](const double* r, double* z) {
    if (h->opts.use_graph && pc != SG_PC_NONE) return apply_graph(h, pc, r, z, &nbmv, &nbs);
    if (pc == SG_PC_HSC) return apply_hsc(h, r, z, &nbmv, &nbs);
    if (pc == SG_PC_BGS) return apply_bgs(h, r, z, &nbmv, &nbs);
    if (pc == SG_PC_MEAN) return apply_mean(h, r, z, &nbs);
    sgk::launch_copy_d2d(z, r, N, h->stream);
    return (int)SG_OK;
  };
  FcgRun run;
  int rc = fcg_core(h, N, F, U, rtol, maxit, use_x0, op, prec, run);
  if (rc) return rc;
  double true_rel = 0.0;
  rc = full_true_relres(h, F, U, run.fn2, &true_rel);
  if (rc) return rc;
  return finish_stats(h, run, true_rel, nbmv, nbs, total, st);
}

// Flexible CG on the Schur complement of the top degree (Section 5): the
// reduced unknown and right-hand side are the first off[p] columns; D_p^-1 of
// the operator, of the right-hand side and of the recovery runs the inner PCG
// (FP64) to op_rtol.
int solve_reduced(sg_ctx* h, const double* F, double* U, double rtol, int maxit, double op_rtol, sg_stats* st) {
  Timer total;
  const long n = h->n;
  const int p = h->p;
  const int lo = h->off[p], ntop = h->off[p + 1] - h->off[p];
  const long NP = n * (long)h->P, Nr = n * (long)lo;
  reset_inner_stats(h);
  long nbmv = 0, nbs = 0;
  const double pc_rtol = h->opts.inner_rtol;
  auto top_solve = [&](const double* B, double* X) {  // X_top = D_p^-1 B_top (tight)
    h->opts.inner_rtol = op_rtol;
    const int rc = run_pcg<double>(h, B + lo * n, X + lo * n, ntop, p);
    h->opts.inner_rtol = pc_rtol;
    nbs += ntop;
    return rc;
  };
  double* g = h->rhs;
  double* w = h->lam;
  // g = f_low - B_p D_p^-1 f_top
  int rc = top_solve(F, w);
  if (rc) return rc;
  sgk::launch_copy_d2d(g, F, Nr, h->stream);
  coupling<double>(h, p, 0, g, w);
  nbmv += coupling_blocks(h, p, 0);
  // the iteration vectors are prefixes; their top columns stay zero
  sgk::launch_fill(h->pv, 0.0, NP, h->stream);
  sgk::launch_fill(U, 0.0, NP, h->stream);
  // S x = A_low x - B_p D_p^-1 C_p x: the full product of [x; 0] gives A_low x on
  // the low columns and C_p x on the top ones
  auto op = [&](const double* x, double* y) {
    matvec(h, x, y);
    int rc2 = top_solve(y, w);
    if (rc2) return rc2;
    coupling<double>(h, p, 0, y, w);
    nbmv += coupling_blocks(h, p, 0);
    return (int)SG_OK;
  };
  auto prec = [&](const double* r, double* z) {
    if (h->opts.precond == SG_PC_MEAN) {
      nbs += lo;
      return run_pcg<double>(h, r, z, lo, -1);
    }
    sgk::launch_copy_d2d((double*)h->rw, r, Nr, h->stream);
    int rc2;
    {
      DeferInner d(h);
      rc2 = hsc_core<double>(h, (double*)h->rw, z, &nbmv, &nbs, p - 1);
    }
    const int rf = flush_inner(h);
    return rc2 ? rc2 : rf;
  };
  FcgRun run;
  rc = fcg_core(h, Nr, g, U, rtol, maxit, 0, op, prec, run);
  if (rc) return rc;
  // recovery: u_top = D_p^-1 (f_top - C_p u_low)
  sgk::launch_copy_d2d(w + lo * n, F + lo * n, n * (long)ntop, h->stream);
  coupling<double>(h, p, 1, w, U);
  nbmv += coupling_blocks(h, p, 1);
  rc = top_solve(w, U);
  if (rc) return rc;
  double fn2 = 0.0, true_rel = 0.0;
  rc = dots(h, 1, F, F);
  if (rc) return rc;
  fn2 = h->host_out[0];
  rc = full_true_relres(h, F, U, fn2, &true_rel);
  if (rc) return rc;
  return finish_stats(h, run, true_rel, nbmv, nbs, total, st);
}

// Bytes of scratch the inner solver needs for ncols columns outside the
// handle's workspace: the inner-precision copies of B and X (FP32 only), the
// six state vectors, the per-tile partials (sized for the finest tiling) and
// the per-column counters; each piece 256-byte aligned.
size_t inner_scratch_bytes(const sg_ctx* h, int ncols) {
  const size_t w = h->opts.inner_precision == 32 ? 4 : 8;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t vec = al(w * (size_t)h->n * ncols);
  const size_t ntiles = (size_t)((h->nx + 15) / 16) * ((h->nx + 15) / 16);
  size_t total = 6 * vec;
  if (w == 4) total += 2 * vec;
  total += al(sizeof(double) * sgk::kPcgPartials * ncols * ntiles);
  total += al(sizeof(unsigned) * ncols) + al(sizeof(int) * ncols) + al(sizeof(int));
  return total;
}

// sg_inner_solve with every buffer beyond B and X inside `scratch` (device,
// 256-byte aligned, at least inner_scratch_bytes(h, ncols) long).
int inner_solve_in(sg_ctx* h, const double* B, double* X, int ncols, int32_t* iters, char* scratch) {
  const size_t w = h->opts.inner_precision == 32 ? 4 : 8;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t vec = al(w * (size_t)h->n * ncols);
  const size_t ntiles = (size_t)((h->nx + 15) / 16) * ((h->nx + 15) / 16);
  char* p = scratch;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += al(bytes);
    return q;
  };
  void* rw = w == 4 ? take(vec) : nullptr;
  void* zw = w == 4 ? take(vec) : nullptr;
  PcgBufs buf{};
  buf.R0 = take(vec);
  buf.R1 = take(vec);
  buf.P0 = take(vec);
  buf.P1 = take(vec);
  buf.Q = take(vec);
  buf.Z = take(vec);
  buf.sc.part = (double*)take(sizeof(double) * sgk::kPcgPartials * ncols * ntiles);
  buf.sc.arrivals = (unsigned*)take(sizeof(unsigned) * ncols);
  buf.sc.iters = (int*)take(sizeof(int) * ncols);
  buf.sc.status = (int*)take(sizeof(int));
  buf.maxcols = ncols;
  std::vector<int> it;
  const long N = h->n * (long)ncols;
  int rc;
  if (w == 8) {
    rc = run_pcg<double>(h, B, X, ncols, -1, &it, false, &buf);
  } else {
    sgk::launch_copy_d2f((float*)rw, B, N, h->stream);
    rc = run_pcg<float>(h, (const float*)rw, (float*)zw, ncols, -1, &it, false, &buf);
    if (!rc) sgk::launch_copy_f2d(X, (const float*)zw, N, h->stream);
  }
  if (rc) return rc;
  SG_HIP(hipStreamSynchronize(h->stream));
  if (iters)
    for (int c = 0; c < ncols; ++c) iters[c] = it[c];
  return SG_OK;
}

// Schedule parameter of the SG operator variant in use (as in sg_tune_report).
int mv_param(const sg_ctx* h) {
  if (h->mv_variant == 3) return (h->mv_piece_rows > 0 ? h->mv_piece_rows : 16) * 100 + h->mv_piece_waves;
  if (h->mv_variant == 2) return h->mv_seg_per_xcd;
  return h->mv_blocks_per_band;
}

// Schedule autotuner (sg_autotune).
int autotune(sg_ctx* h, int flags, sg_tune_report* out) {
  drop_pc_graph(h);  // a captured action holds the old schedules
  sg_tune_report R{};
  const long N = h->n * (long)h->P;
  hipStream_t s = h->stream;
  auto event_ms = [&](const std::function<void()>& body, int reps, double* med) -> int {
    std::vector<float> t;
    for (int r = 0; r < reps; ++r) {
      SG_HIP(hipEventRecord(h->ev0, s));
      body();
      SG_HIP(hipEventRecord(h->ev1, s));
      SG_HIP(hipEventSynchronize(h->ev1));
      float ms = 0.f;
      SG_HIP(hipEventElapsedTime(&ms, h->ev0, h->ev1));
      t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    *med = t[t.size() / 2];
    return SG_OK;
  };
  if (flags & 1) {
    set_stage_rows(h, 0);  // the candidates below run the full operator through their own kernels
    sgk::launch_fill(h->pv, 1.0, N, s);
    struct Cand {
      int variant, param;
    };
    std::vector<Cand> cands;
    const bool wide = h->n_e % 64 == 0 && h->n_e >= 64 && h->n_e <= 512;
    // piece kernel: node rows per piece (param = rows * 100 + wave cap per CU)
    if (h->M <= sgk::kPieceMaxM)
      for (int ty : {8, 16, 32})
        for (int waves : {0, 4})  // all resident waves, or 4 per CU (fewer pieces at once per XCD)
          if (ty <= std::max(8, h->nx)) cands.push_back({3, ty * 100 + waves});
    if (sgk::march_supported(h->n_e, h->M))
      for (int spx : {0, 1, 2, 4}) cands.push_back({2, spx});
    if (wide) {
      for (int bpb : {32, 64, 128}) cands.push_back({1, bpb});
      if (h->M <= 12)
        for (int bpb : {64, 128}) cands.push_back({0, bpb});
    }
    auto apply = [&](const Cand& c) -> int {
      h->mv_variant = c.variant;
      h->mv_blocks_per_band = c.variant == 0 || c.variant == 1 ? c.param : 0;
      if (c.variant == 3) {
        h->mv_piece_rows = c.param / 100;
        h->mv_piece_waves = c.param % 100;
      }
      return build_march_jobs(h, c.variant == 2 ? c.param : 0);
    };
    double best = 1e300;
    Cand pick{h->mv_variant, mv_param(h)};
    for (const Cand& c : cands) {
      int rc = apply(c);
      if (rc) return rc;
      matvec(h, h->pv, h->q);
      matvec(h, h->pv, h->q);
      double med = 0.0;
      rc = event_ms([&] { matvec(h, h->pv, h->q); }, 5, &med);
      if (rc) return rc;
      ++R.candidates;
      if (med < best) {
        best = med;
        pick = c;
      }
    }
    int rc = apply(pick);
    if (rc) return rc;
    R.mv_ms = cands.empty() ? 0.0 : best;
    // the full operator may then take the row-staged kernel (the couplings keep the pick)
    int best_rows = 0;
    if (h->stage_ok)
      for (int rows : {4, 6, 8, 10, 12, 16}) {
        if (rows > std::max(4, h->nx)) continue;
        set_stage_rows(h, rows);
        matvec(h, h->pv, h->q);
        matvec(h, h->pv, h->q);
        double med = 0.0;
        rc = event_ms([&] { matvec(h, h->pv, h->q); }, 5, &med);
        if (rc) return rc;
        ++R.candidates;
        if (med < best) {
          best = med;
          best_rows = rows;
        }
      }
    set_stage_rows(h, best_rows);
    R.mv_ms = best < 1e300 ? best : 0.0;
  }
  R.mv_variant = h->mv_stage > 0 ? 4 : h->mv_variant;
  R.mv_param = h->mv_stage > 0 ? h->mv_stage : mv_param(h);
  const int degree = effective_degree(h);
  if (flags & 2) {
    const int lev = h->p;
    const int ncols = h->off[lev + 1] - h->off[lev];
    sgk::launch_fill(h->pv, 1.0, N, s);
    if (h->opts.inner_precision == 32) sgk::launch_copy_d2f((float*)h->rw, h->pv, N, s);
    else sgk::launch_copy_d2d((double*)h->rw, h->pv, N, s);
    // banded candidate: the automatic choice (0, which also shortens the bands of
    // small launches) unless banded tiles were asked for explicitly
    const int band = h->opts.tile == 32 ? 32 : 0;
    std::vector<int> tiles = degree <= sgk::kBandMaxDegree ? std::vector<int>{band, 16}
                                                                                       : std::vector<int>{16};
    // automatic grid, half the compute units, whole columns per block (large launches)
    std::vector<int> blocks = {0, std::max(1, h->num_cu / 2), -1};
    double best = 1e300;
    int bt = choose_tile(h, degree), bb = h->pcg_max_blocks;
    for (int t : tiles)
      for (int mb : blocks) {
        h->opts.tile = t;
        h->pcg_max_blocks = mb;
        int rc = h->opts.inner_precision == 32 ? run_pcg<float>(h, (const float*)h->rw, (float*)h->zw, ncols, -1)
                                               : run_pcg<double>(h, (const double*)h->rw, h->z, ncols, -1);
        if (rc) return rc;
        h->inner_ms_acc = 0.0;
        rc = h->opts.inner_precision == 32 ? run_pcg<float>(h, (const float*)h->rw, (float*)h->zw, ncols, -1)
                                           : run_pcg<double>(h, (const double*)h->rw, h->z, ncols, -1);
        if (rc) return rc;
        ++R.candidates;
        if (h->inner_ms_acc < best) {
          best = h->inner_ms_acc;
          bt = t;
          bb = mb;
        }
      }
    h->opts.tile = bt;
    h->pcg_max_blocks = bb;
    R.pcg_ms = best;
    h->inner_it_acc = 0;
    h->inner_ms_acc = 0.0;
    h->inner_bytes_acc = 0.0;
    h->inner_launch_acc = 0;
  }
  R.pcg_tile = choose_tile(h, degree);
  R.pcg_max_blocks = h->pcg_max_blocks;
  if (out) *out = R;
  return SG_OK;
}

// Frees a handle's host-side resources: events, pinned read-back buffers, the context.
void release_ctx(sg_ctx* h) {
  drop_pc_graph(h);
  (void)hipEventDestroy(h->ev0);
  (void)hipEventDestroy(h->ev1);
  for (int i = 0; i < h->nev; ++i) (void)hipEventDestroy(h->evpool[i]);
  if (h->iters_host) (void)hipHostFree(h->iters_host);
  if (h->status_host) (void)hipHostFree(h->status_host);
  delete h;
}

}  // namespace sgh

using namespace sgh;

extern "C" {

int sg_workspace_bytes(const sg_problem* prob, const sg_opts* opts, size_t* bytes) {
  int rc = validate(prob, opts);
  if (rc) return rc;
  if (!bytes) return fail(SG_EINVAL, "null bytes");
  Plan pl;
  make_plan(prob, opts, pl);
  *bytes = pl.total;
  return SG_OK;
}

int sg_setup(const sg_problem* pr, const sg_opts* op, void* workspace, size_t workspace_bytes, void* stream,
             sg_handle* out) {
  int rc = validate(pr, op);
  if (rc) return rc;
  if (!out || !workspace) return fail(SG_EINVAL, "null workspace or handle pointer");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(SG_EINVAL, "workspace must be 256-byte aligned");
  for (int k = 0; k < pr->M; ++k)
    if (!std::isfinite(pr->s[k])) return fail(SG_EINVAL, "s is not finite");
  Plan pl;
  make_plan(pr, op, pl);
  if (workspace_bytes < pl.total) return fail(SG_ENOMEM, "workspace too small");
  sg_ctx* h = new (std::nothrow) sg_ctx();
  if (!h) return fail(SG_ENOMEM, "host allocation failed");
  h->n_e = pr->n_e;
  h->M = pr->M;
  h->p = pr->p;
  h->family = pr->family;
  h->P = pl.P;
  h->nx = pl.nx;
  h->n = pl.n;
  h->theta0 = pr->theta0;
  h->sigma = pr->sigma;
  h->s.assign(pr->s, pr->s + pr->M);
  h->opts = *op;
  h->stream = (hipStream_t)stream;
  h->ws = (char*)workspace;
  h->ws_bytes = workspace_bytes;
  multi_indices(h->M, h->p, h->alpha, h->off);
  cheb_interval(h->n_e, h->lmin, h->lmax);
  h->mv_blocks_per_band = 0;
  if (const char* env = std::getenv("SGPC_MV_BLOCKS_PER_BAND")) h->mv_blocks_per_band = std::atoi(env);
  h->mv_variant = pr->M <= sgk::kPieceMaxM ? 3 : 2;
  if (const char* env = std::getenv("SGPC_MV_VARIANT")) h->mv_variant = std::atoi(env);
  if (const char* env = std::getenv("SGPC_MV_PIECE_ROWS")) h->mv_piece_rows = std::atoi(env);
  h->pcg_max_blocks = 0;
  if (const char* env = std::getenv("SGPC_PCG_MAX_BLOCKS")) h->pcg_max_blocks = std::atoi(env);
  const int M = h->M, P = h->P;
  const long ne2 = (long)h->n_e * h->n_e;
  // element coefficients
  std::vector<double> a64((size_t)M * ne2), c64((size_t)M * ne2);
  std::vector<float> a32((size_t)M * ne2);
  for (int k = 0; k < M; ++k)
    for (long e = 0; e < ne2; ++e) {
      const double ph = pr->phi[(long)k * ne2 + e];
      if (!std::isfinite(ph)) {
        delete h;
        return fail(SG_EINVAL, "phi is not finite");
      }
      c64[(size_t)k * ne2 + e] = pr->sigma * ph;
      a64[(size_t)k * ne2 + e] = pr->sigma * pr->s[k] * ph;
      a32[(size_t)k * ne2 + e] = (float)a64[(size_t)k * ne2 + e];
    }
  // chaos neighbour lists
  std::map<std::vector<int>, int> index;
  for (int a = 0; a < P; ++a)
    index[std::vector<int>(h->alpha.begin() + (long)a * M, h->alpha.begin() + (long)(a + 1) * M)] = a;
  std::vector<int> lo_ptr(P + 1, 0), up_ptr(P + 1, 0), lo_ent, up_ent;
  std::vector<double> lo_g, up_g;
  std::vector<std::vector<std::pair<int, int>>> pairs(M);  // per k: (a, b)
  std::vector<std::vector<double>> pairg(M);
  // (G_k)_{a, a+e_k} = E[xi psi_n psi_{n+1}] with n = a_k: sqrt(n + 1) for the
  // normalised Hermite basis, (n + 1) / sqrt((2n + 1)(2n + 3)) for the
  // normalised Legendre basis (three-term recurrences of the two families)
  const bool leg = h->family == SG_FAMILY_LEGENDRE;
  auto up_weight = [&](int n) {
    return leg ? (n + 1.0) / std::sqrt((2.0 * n + 1.0) * (2.0 * n + 3.0)) : std::sqrt(n + 1.0);
  };
  for (int a = 0; a < P; ++a) {
    std::vector<int> al(h->alpha.begin() + (long)a * M, h->alpha.begin() + (long)(a + 1) * M);
    int deg = 0;
    for (int v : al) deg += v;
    for (int k = 0; k < M; ++k) {
      if (al[k] > 0) {
        std::vector<int> b = al;
        b[k] -= 1;
        const int bi = index.at(b);
        lo_ent.push_back(bi | ((k + 1) << 20));
        lo_g.push_back(up_weight(al[k] - 1));
        pairs[k].push_back({a, bi});
        pairg[k].push_back(up_weight(al[k] - 1));
      }
    }
    lo_ptr[a + 1] = (int)lo_ent.size();
    for (int k = 0; k < M; ++k) {
      if (deg < h->p) {
        std::vector<int> b = al;
        b[k] += 1;
        const int bi = index.at(b);
        up_ent.push_back(bi | ((k + 1) << 20));
        up_g.push_back(up_weight(al[k]));
        pairs[k].push_back({a, bi});
        pairg[k].push_back(up_weight(al[k]));
      }
    }
    up_ptr[a + 1] = (int)up_ent.size();
  }
  std::vector<float> lo_g32(lo_g.begin(), lo_g.end()), up_g32(up_g.begin(), up_g.end());
  // dense [P][M] neighbour tables for the strip kernel
  const size_t PMd = std::max<size_t>(1, (size_t)P * M);
  std::vector<int> st_lo(PMd, -1), st_up(PMd, -1);
  std::vector<double> st_glo(PMd, 0.0), st_gup(PMd, 0.0);
  for (int a = 0; a < P; ++a) {
    for (int e = lo_ptr[a]; e < lo_ptr[a + 1]; ++e) {
      const int k = (lo_ent[e] >> 20) - 1;
      st_lo[(size_t)a * M + k] = lo_ent[e] & 0xFFFFF;
      st_glo[(size_t)a * M + k] = lo_g[e];
    }
    for (int e = up_ptr[a]; e < up_ptr[a + 1]; ++e) {
      const int k = (up_ent[e] >> 20) - 1;
      st_up[(size_t)a * M + k] = up_ent[e] & 0xFFFFF;
      st_gup[(size_t)a * M + k] = up_g[e];
    }
  }
  std::vector<float> st_glo32(st_glo.begin(), st_glo.end()), st_gup32(st_gup.begin(), st_gup.end());
  // compact entry lists: one entry per KL term with at least one Galerkin neighbour
  std::vector<int> en_ptr(P + 1, 0), en_k, en_lo, en_up;
  std::vector<double> en_glo, en_gup;
  for (int a = 0; a < P; ++a) {
    for (int k = 0; k < M; ++k) {
      const int lo = st_lo[(size_t)a * M + k], upi = st_up[(size_t)a * M + k];
      if (lo < 0 && upi < 0) continue;
      en_k.push_back(k);
      en_lo.push_back(lo >= 0 ? lo : a);
      en_up.push_back(upi >= 0 ? upi : a);
      en_glo.push_back(lo >= 0 ? st_glo[(size_t)a * M + k] : 0.0);
      en_gup.push_back(upi >= 0 ? st_gup[(size_t)a * M + k] : 0.0);
    }
    en_ptr[a + 1] = (int)en_k.size();
  }
  std::vector<float> en_glo32(en_glo.begin(), en_glo.end()), en_gup32(en_gup.begin(), en_gup.end());
  std::vector<int> pair_ptr(M + 1, 0), pair_a, pair_b;
  std::vector<double> pair_g;
  for (int k = 0; k < M; ++k) {
    for (size_t i = 0; i < pairs[k].size(); ++i) {
      pair_a.push_back(pairs[k][i].first);
      pair_b.push_back(pairs[k][i].second);
      pair_g.push_back(pairg[k][i]);
    }
    pair_ptr[k + 1] = (int)pair_a.size();
  }
  // the host tables above need no device; the first HIP call comes here
  int dev = 0;
  h->num_cu = 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    delete h;
    return fail(SG_EDEVICE, "no HIP device");
  }
  h->lo_ptr = lo_ptr;
  h->up_ptr = up_ptr;
  char* w = h->ws;
  h->a64 = (double*)(w + pl.o_a64);
  h->a32 = (float*)(w + pl.o_a32);
  h->c64 = (double*)(w + pl.o_c64);
  h->lo_ptr_d = (int*)(w + pl.o_lo_ptr);
  h->lo_ent_d = (int*)(w + pl.o_lo_ent);
  h->lo_g64 = (double*)(w + pl.o_lo_g64);
  h->lo_g32 = (float*)(w + pl.o_lo_g32);
  h->up_ptr_d = (int*)(w + pl.o_up_ptr);
  h->up_ent_d = (int*)(w + pl.o_up_ent);
  h->up_g64 = (double*)(w + pl.o_up_g64);
  h->up_g32 = (float*)(w + pl.o_up_g32);
  h->st_lo_d = (int*)(w + pl.o_st_lo);
  h->st_up_d = (int*)(w + pl.o_st_up);
  h->st_glo64 = (double*)(w + pl.o_st_glo64);
  h->st_gup64 = (double*)(w + pl.o_st_gup64);
  h->st_glo32 = (float*)(w + pl.o_st_glo32);
  h->st_gup32 = (float*)(w + pl.o_st_gup32);
  h->en_ptr_d = (int*)(w + pl.o_en_ptr);
  h->en_k_d = (int*)(w + pl.o_en_k);
  h->en_lo_d = (int*)(w + pl.o_en_lo);
  h->en_up_d = (int*)(w + pl.o_en_up);
  h->en_glo64 = (double*)(w + pl.o_en_glo64);
  h->en_gup64 = (double*)(w + pl.o_en_gup64);
  h->en_glo32 = (float*)(w + pl.o_en_glo32);
  h->en_gup32 = (float*)(w + pl.o_en_gup32);
  h->pair_ptr_d = (int*)(w + pl.o_pair_ptr);
  h->pair_a_d = (int*)(w + pl.o_pair_a);
  h->pair_b_d = (int*)(w + pl.o_pair_b);
  h->pair_g_d = (double*)(w + pl.o_pair_g);
  double** vecs[7] = {&h->r, &h->z, &h->pv, &h->q, &h->lam, &h->tmp, &h->rhs};
  for (int i = 0; i < 7; ++i) *vecs[i] = (double*)(w + pl.o_vec[i]);
  h->rw = w + pl.o_rw;
  h->zw = op->inner_precision == 32 ? (void*)(w + pl.o_zw) : nullptr;
  void** pcgv[6] = {&h->pR0, &h->pR1, &h->pP0, &h->pP1, &h->pQ, &h->pZ};
  for (int i = 0; i < 6; ++i) *pcgv[i] = w + pl.o_pcg[i];
  h->pcg_maxcols = pl.maxcols;
  h->pcgsc.part = (double*)(w + pl.o_part);
  h->pcgsc.arrivals = (unsigned*)(w + pl.o_arr);
  h->pcgsc.iters = (int*)(w + pl.o_iters);
  h->pcgsc.status = (int*)(w + pl.o_status);
  h->red_part = (double*)(w + pl.o_red_part);
  h->red_out = (double*)(w + pl.o_red_out);
  h->host_out.assign(std::max(64, M + 1), 0.0);
  hipStream_t s = h->stream;
  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up(h->a64, a64.data(), sizeof(double) * a64.size());
  if (e == hipSuccess) e = up(h->a32, a32.data(), sizeof(float) * a32.size());
  if (e == hipSuccess) e = up(h->c64, c64.data(), sizeof(double) * c64.size());
  if (e == hipSuccess) e = up(h->lo_ptr_d, lo_ptr.data(), sizeof(int) * lo_ptr.size());
  if (e == hipSuccess) e = up(h->lo_ent_d, lo_ent.data(), sizeof(int) * lo_ent.size());
  if (e == hipSuccess) e = up(h->lo_g64, lo_g.data(), sizeof(double) * lo_g.size());
  if (e == hipSuccess) e = up(h->lo_g32, lo_g32.data(), sizeof(float) * lo_g32.size());
  if (e == hipSuccess) e = up(h->up_ptr_d, up_ptr.data(), sizeof(int) * up_ptr.size());
  if (e == hipSuccess) e = up(h->up_ent_d, up_ent.data(), sizeof(int) * up_ent.size());
  if (e == hipSuccess) e = up(h->up_g64, up_g.data(), sizeof(double) * up_g.size());
  if (e == hipSuccess) e = up(h->up_g32, up_g32.data(), sizeof(float) * up_g32.size());
  if (e == hipSuccess) e = up(h->st_lo_d, st_lo.data(), sizeof(int) * st_lo.size());
  if (e == hipSuccess) e = up(h->st_up_d, st_up.data(), sizeof(int) * st_up.size());
  if (e == hipSuccess) e = up(h->st_glo64, st_glo.data(), sizeof(double) * st_glo.size());
  if (e == hipSuccess) e = up(h->st_gup64, st_gup.data(), sizeof(double) * st_gup.size());
  if (e == hipSuccess) e = up(h->st_glo32, st_glo32.data(), sizeof(float) * st_glo32.size());
  if (e == hipSuccess) e = up(h->st_gup32, st_gup32.data(), sizeof(float) * st_gup32.size());
  if (e == hipSuccess) e = up(h->en_ptr_d, en_ptr.data(), sizeof(int) * en_ptr.size());
  if (e == hipSuccess) e = up(h->en_k_d, en_k.data(), sizeof(int) * en_k.size());
  if (e == hipSuccess) e = up(h->en_lo_d, en_lo.data(), sizeof(int) * en_lo.size());
  if (e == hipSuccess) e = up(h->en_up_d, en_up.data(), sizeof(int) * en_up.size());
  if (e == hipSuccess) e = up(h->en_glo64, en_glo.data(), sizeof(double) * en_glo.size());
  if (e == hipSuccess) e = up(h->en_gup64, en_gup.data(), sizeof(double) * en_gup.size());
  if (e == hipSuccess) e = up(h->en_glo32, en_glo32.data(), sizeof(float) * en_glo32.size());
  if (e == hipSuccess) e = up(h->en_gup32, en_gup32.data(), sizeof(float) * en_gup32.size());
  if (e == hipSuccess) e = up(h->pair_ptr_d, pair_ptr.data(), sizeof(int) * pair_ptr.size());
  if (e == hipSuccess) e = up(h->pair_a_d, pair_a.data(), sizeof(int) * pair_a.size());
  if (e == hipSuccess) e = up(h->pair_b_d, pair_b.data(), sizeof(int) * pair_b.size());
  if (e == hipSuccess) e = up(h->pair_g_d, pair_g.data(), sizeof(double) * pair_g.size());
  h->st_lo_h = st_lo;
  h->st_up_h = st_up;
  h->st_glo_h = st_glo;
  h->mj_ptr_d = (int*)(w + pl.o_mj_ptr);
  h->mj_rows_d = (int*)(w + pl.o_mj_rows);
  h->mj_kind_d = (int*)(w + pl.o_mj_kind);
  h->mj_lk_d = (int*)(w + pl.o_mj_lk);
  h->mj_lcol_d = (int*)(w + pl.o_mj_lcol);
  h->mj_lw_d = (double*)(w + pl.o_mj_lw);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && build_march_jobs(h, 0) != SG_OK) e = hipErrorUnknown;
  if (e == hipSuccess &&
      build_stage_tables(h, (sgk::StageTerm*)(w + pl.o_stg_terms), (sgk::StageSlot*)(w + pl.o_stg_slots),
                         (int*)(w + pl.o_stg_wslot)) != SG_OK)
    e = hipErrorUnknown;
  if (e == hipSuccess) {
    // the full operator takes the row-staged kernel where it fits and its pieces
    // of 10 node rows keep at least half of the compute units busy (one block per
    // CU); the autotuner chooses among 4..16 rows or the other kernels
    const long pieces10 = (long)((h->nx + sgk::kStageOut - 1) / sgk::kStageOut) * ((h->nx + 9) / 10);
    int rows = 2 * pieces10 >= h->num_cu ? 10 : 0;
    if (const char* env = std::getenv("SGPC_MV_STAGE")) rows = std::atoi(env);
    set_stage_rows(h, rows);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete h;
    return fail(SG_EDEVICE, std::string("upload failed: ") + hipGetErrorString(e));
  }
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) {
    delete h;
    return fail(SG_EDEVICE, "event creation failed");
  }
  // read-back of deferred inner launches: an action launches at most 2p + 1
  // solves over at most 2P + 1 columns (more only force an earlier flush)
  h->iters_cap = 2L * P + 64;
  bool ok = hipHostMalloc((void**)&h->iters_host, sizeof(int) * h->iters_cap, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&h->status_host, sizeof(int) * sg_ctx::kMaxPending, hipHostMallocDefault) ==
                hipSuccess;
  for (int i = 0; ok && i < 2 * sg_ctx::kMaxPending; ++i) {
    ok = hipEventCreate(&h->evpool[i]) == hipSuccess;
    if (ok) h->nev = i + 1;
  }
  if (!ok) {
    release_ctx(h);
    return fail(SG_EDEVICE, "event or pinned buffer creation failed");
  }
  // this device's static scratch (used only by sg_inner_solve_static); a
  // failure here is reported by that call, which retries the lookup
  if (static_scratch_address(&h->static_scratch) != SG_OK) h->static_scratch = nullptr;
  *out = h;
  return SG_OK;
}

int sg_sizes(sg_handle h, int64_t* n, int32_t* P, int32_t* level_off, int32_t* alpha) {
  if (!h) return fail(SG_EINVAL, "null handle");
  if (n) *n = h->n;
  if (P) *P = h->P;
  if (level_off)
    for (int l = 0; l <= h->p + 1; ++l) level_off[l] = h->off[l];
  if (alpha)
    for (size_t i = 0; i < h->alpha.size(); ++i) alpha[i] = h->alpha[i];
  return SG_OK;
}

int sg_set_opts(sg_handle h, const sg_opts* opts) {
  if (!h || !opts) return fail(SG_EINVAL, "null handle or options");
  sg_problem dummy{};
  dummy.n_e = h->n_e;
  dummy.M = 0;
  dummy.p = h->p;
  dummy.theta0 = h->theta0;
  int rc = validate(&dummy, opts);
  if (rc) return rc;
  if (opts->inner_precision != h->opts.inner_precision)
    return fail(SG_EINVAL, "inner precision is fixed at setup");
  h->opts = *opts;
  drop_pc_graph(h);  // a captured action holds the old options
  return SG_OK;
}

int sg_matvec(sg_handle h, const double* U, double* Y) {
  if (!h || !U || !Y) return fail(SG_EINVAL, "null argument");
  if (U == Y) return fail(SG_EINVAL, "U and Y must be distinct");
  matvec(h, U, Y);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

int sg_apply_hsc(sg_handle h, const double* R, double* Z) {
  if (!h || !R || !Z) return fail(SG_EINVAL, "null argument");
  if (R == Z) return fail(SG_EINVAL, "R and Z must be distinct");
  long a = 0, b = 0;
  for (int l = 0; l < sgk::kMaxLevels; ++l) h->inner_it_max[l] = 0;
  int rc = apply_hsc(h, R, Z, &a, &b);
  if (rc) return rc;
  SG_HIP(hipGetLastError());
  return SG_OK;
}

int sg_apply_bgs(sg_handle h, const double* R, double* Z) {
  if (!h || !R || !Z) return fail(SG_EINVAL, "null argument");
  if (R == Z) return fail(SG_EINVAL, "R and Z must be distinct");
  long a = 0, b = 0;
  int rc = apply_bgs(h, R, Z, &a, &b);
  if (rc) return rc;
  SG_HIP(hipGetLastError());
  return SG_OK;
}

int sg_apply_mean(sg_handle h, const double* R, double* Z) {
  if (!h || !R || !Z) return fail(SG_EINVAL, "null argument");
  if (R == Z) return fail(SG_EINVAL, "R and Z must be distinct");
  long b = 0;
  int rc = apply_mean(h, R, Z, &b);
  if (rc) return rc;
  SG_HIP(hipGetLastError());
  return SG_OK;
}

int sg_inner_solve(sg_handle h, const double* B, double* X, int32_t ncols, int32_t* iters) {
  if (!h || !B || !X) return fail(SG_EINVAL, "null argument");
  if ((const double*)X == B) return fail(SG_EINVAL, "B and X must be distinct");
  if (ncols < 0 || ncols > h->P) return fail(SG_EINVAL, "ncols must be in 0..P");
  if (ncols == 0) return SG_OK;
  std::vector<int> it;
  const long N = h->n * (long)ncols;
  int rc;
  if (h->opts.inner_precision == 64) {
    rc = run_pcg<double>(h, B, X, ncols, -1, &it);
  } else {
    float* rw = (float*)h->rw;
    float* zw = (float*)h->zw;
    sgk::launch_copy_d2f(rw, B, N, h->stream);
    rc = run_pcg<float>(h, rw, zw, ncols, -1, &it);
    if (!rc) sgk::launch_copy_f2d(X, zw, N, h->stream);
  }
  if (rc) return rc;
  SG_HIP(hipStreamSynchronize(h->stream));
  if (iters)
    for (int c = 0; c < ncols; ++c) iters[c] = it[c];
  return SG_OK;
}

int sg_coupling(sg_handle h, int32_t level, int32_t dir, double* R, const double* V) {
  if (!h || !R || !V) return fail(SG_EINVAL, "null argument");
  if (level < 1 || level > h->p) return fail(SG_EINVAL, "level must be in 1..p");
  if (dir != 0 && dir != 1) return fail(SG_EINVAL, "dir must be 0 or 1");
  if ((const double*)R == V) return fail(SG_EINVAL, "R and V must be distinct");
  coupling<double>(h, level, dir, R, V);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

int sg_solve(sg_handle h, const double* F, double* U, double rtol, int32_t maxit, int32_t use_x0, sg_stats* stats) {
  if (!h || !F || !U) return fail(SG_EINVAL, "null argument");
  if (F == U) return fail(SG_EINVAL, "F and U must be distinct");
  if (!(rtol >= 0.0) || maxit < 0) return fail(SG_EINVAL, "rtol must be >= 0 and maxit >= 0");
  return fcg(h, F, U, rtol, maxit, use_x0, h->opts.precond, stats);
}

int sg_solve_reduced(sg_handle h, const double* F, double* U, double rtol, int32_t maxit, double op_rtol,
                     sg_stats* stats) {
  if (!h || !F || !U) return fail(SG_EINVAL, "null argument");
  if (F == U) return fail(SG_EINVAL, "F and U must be distinct");
  if (!(rtol >= 0.0) || maxit < 0) return fail(SG_EINVAL, "rtol must be >= 0 and maxit >= 0");
  if (!(op_rtol > 0.0 && op_rtol < 1.0)) return fail(SG_EINVAL, "op_rtol must be in (0, 1)");
  if (h->p < 1) return fail(SG_EINVAL, "the reduction needs chaos degree p >= 1");
  if (h->opts.inner_precision != 64) return fail(SG_EINVAL, "the reduced solve needs FP64 inner solves");
  if (h->opts.precond != SG_PC_HSC && h->opts.precond != SG_PC_MEAN)
    return fail(SG_EINVAL, "the reduced solve takes the HSC or the mean-based preconditioner");
  return solve_reduced(h, F, U, rtol, maxit, op_rtol, stats);
}

int sg_qoi(sg_handle h, const double* U, const double* w_mean, const double* w_var, double* Q) {
  if (!h || !U || !w_mean || !w_var || !Q) return fail(SG_EINVAL, "null argument");
  sgk::launch_qoi(U, w_mean, w_var, h->n, h->P, h->red_part, h->red_out, h->stream);
  int rc = read_out(h, 1);
  if (rc) return rc;
  *Q = h->host_out[0];
  return SG_OK;
}

int sg_adjoint_grad(sg_handle h, const double* U, const double* w_mean, const double* w_var, double rtol,
                    int32_t maxit, double* Q, double* grad, double* Lambda, sg_stats* stats) {
  if (!h || !U || !w_mean || !w_var || !Q || !grad) return fail(SG_EINVAL, "null argument");
  if ((const double*)Lambda == U) return fail(SG_EINVAL, "Lambda must differ from U");
  if (!(rtol >= 0.0) || maxit < 0) return fail(SG_EINVAL, "rtol must be >= 0 and maxit >= 0");
  int rc = sg_qoi(h, U, w_mean, w_var, Q);
  if (rc) return rc;
  sgk::launch_qoi_grad(U, w_mean, w_var, h->n, h->P, h->rhs, h->stream);
  double* lam = Lambda ? Lambda : h->lam;
  const int status = fcg(h, h->rhs, lam, rtol, maxit, 0, h->opts.precond, stats);
  if (status < 0) return status;
  sgk::ContractArgs c{};
  c.n_e = h->n_e;
  c.nx = h->nx;
  c.n = h->n;
  c.M = h->M;
  c.P = h->P;
  c.Lam = lam;
  c.U = U;
  c.c = h->c64;
  c.pair_ptr = h->pair_ptr_d;
  c.pair_a = h->pair_a_d;
  c.pair_b = h->pair_b_d;
  c.pair_g = h->pair_g_d;
  c.partials = h->red_part;
  c.out = h->red_out;
  sgk::launch_contract(c, h->stream);
  rc = read_out(h, h->M + 1);
  if (rc) return rc;
  for (int k = 0; k <= h->M; ++k) grad[k] = h->host_out[k];
  return status;
}

int sg_autotune(sg_handle h, int32_t flags, sg_tune_report* report) {
  if (!h) return fail(SG_EINVAL, "null handle");
  if (flags & ~3) return fail(SG_EINVAL, "unknown autotune flags");
  return autotune(h, flags, report);
}

void sg_destroy(sg_handle h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  release_ctx(h);
}

const char* sg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
