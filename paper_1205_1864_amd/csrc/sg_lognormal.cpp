// Lognormal-coefficient SG operator (Section 6, second set of experiments;
// Tables 6-9): k(x, xi) = exp(g(x, xi)) with the Gaussian field
// g = mu_g + sum_k g_k(x) xi_k, expanded in the normalised Hermite chaos to
// total degree 2p. The global matrix A = sum_i G_i (x) K_i,
// (G_i)_ab = E[psi_i psi_a psi_b], is block dense; this file sets up the block
// coefficient fields c_ab = sum_i (G_i)_ab k_i on the device and applies A.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "sg_host.h"
#include "sg_internal.h"

namespace sgk {
void launch_logn_blocks(const long* ptr, const int* term, const double* g, const double* kc, int ne2, int nslots,
                        double* C, hipStream_t s);
void launch_logn_matvec(const int* rptr, const int* rcol, const int* rslot, const double* C, const double* U,
                        int n_e, long n, int P, double* Y, hipStream_t s);
void launch_logn_apply(const int* rptr, const int* rcol, const int* rslot, const double* C, const double* X,
                       int n_e, long n, int row0, int nrows, int col0, int col1, int mode, const double* R, double* Y,
                       hipStream_t s);
void launch_logn_invdiag(const int* rptr, const int* rcol, const int* rslot, const double* C, int n_e, long n, int P,
                         double* Dinv, hipStream_t s);
void launch_logn_dot(const double* x, const double* y, long len, double* part, int nblocks, hipStream_t s);
void launch_logn_axpby(long len, double a, const double* x, double b, double* y, int mode, const double* d,
                       long dn, hipStream_t s);
void launch_logn_mean_apply(const double* c, const double* X, int n_e, long n, int ncols, double* Y, hipStream_t s);
void launch_logn_cg_update(long len, double alpha, const double* p, const double* q, double* x, double* r,
                           const double* d, long dn, double* z, double* part, int nblocks, hipStream_t s);
}  // namespace sgk

namespace sgh {
double lanczos_kappa(const std::vector<double>& al, const std::vector<double>& be);
}  // namespace sgh

constexpr int kLognDotBlocks = 256;

struct sg_logn_ctx {
  int n_e = 0, M = 0, p = 0, P = 0, nslots = 0;
  long n = 0;
  hipStream_t stream = nullptr;
  double* C = nullptr;  // block coefficient fields, nslots x n_e^2
  int *rptr = nullptr, *rcol = nullptr, *rslot = nullptr;
  std::vector<int> off;  // level offsets of the chaos columns, p + 2 entries
  // solver vectors (n x P each): outer FCG r, z, p, q; preconditioner copy of
  // r and a level temporary; level-solve r, z, p, q; inverse diagonal of A
  double *R = nullptr, *Z = nullptr, *Pv = nullptr, *Q = nullptr, *Rh = nullptr, *W = nullptr;
  double *cr = nullptr, *cz = nullptr, *cp = nullptr, *cq = nullptr, *Dinv = nullptr, *part = nullptr;
  double* XF = nullptr;  // forward-sweep values of block Gauss-Seidel
  std::vector<double> host_part;
};

namespace {

using sgh::fail;

// Multi-indices of total degree <= p, graded, descending lexicographic within
// a degree (the order of the chaos columns).
std::vector<std::vector<int>> graded(int M, int p) {
  std::vector<std::vector<int>> out;
  for (int d = 0; d <= p; ++d) {
    std::vector<std::vector<int>> lvl;
    std::vector<int> pre;
    struct Rec {
      std::vector<std::vector<int>>& lv;
      int M;
      void go(std::vector<int>& pre, int rem) {
        if ((int)pre.size() == M) {
          if (rem == 0) lv.push_back(pre);
          return;
        }
        for (int v = rem; v >= 0; --v) {
          pre.push_back(v);
          go(pre, rem - v);
          pre.pop_back();
        }
      }
    } rec{lvl, M};
    if (M == 0) {
      if (d == 0) lvl.push_back({});
    } else {
      rec.go(pre, d);
    }
    out.insert(out.end(), lvl.begin(), lvl.end());
  }
  return out;
}

double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

// E[psi_a psi_b psi_c] for the normalised 1D Hermite basis: with s = (a+b+c)/2
// an integer not below a, b, c, sqrt(a! b! c!) / ((s-a)! (s-b)! (s-c)!); else 0.
double triple(int a, int b, int c) {
  const int two_s = a + b + c;
  if (two_s & 1) return 0.0;
  const int s = two_s / 2;
  if (s < a || s < b || s < c) return 0.0;
  return std::sqrt(factorial(a) * factorial(b) * factorial(c)) / (factorial(s - a) * factorial(s - b) * factorial(s - c));
}

struct Plan {
  int P = 0, T = 0, nslots = 0;
  size_t o_C = 0, o_kc = 0, o_ptr = 0, o_term = 0, o_g = 0, o_rptr = 0, o_rcol = 0, o_rslot = 0, total = 0;
  size_t o_vec = 0, o_part = 0;
  // host tables
  std::vector<std::vector<int>> alpha, coef;
  std::vector<long> ptr;
  std::vector<int> term, rptr, rcol, rslot;
  std::vector<double> g;
};

size_t take(size_t& total, size_t bytes) {
  const size_t o = total;
  total += (bytes + 255) / 256 * 256;
  return o;
}

int validate(const sg_problem* pr) {
  if (!pr) return fail(SG_EINVAL, "null problem");
  if (pr->n_e < 3 || pr->n_e > 4096) return fail(SG_EINVAL, "n_e must be in 3..4096");
  if (pr->M < 0 || pr->M > 16 || pr->p < 0 || pr->p > 8) return fail(SG_EINVAL, "need 0 <= M <= 16, 0 <= p <= 8");
  if (pr->family != SG_FAMILY_HERMITE) return fail(SG_EINVAL, "the lognormal operator uses the Hermite family");
  if (!(pr->theta0 > 0.0) || !(pr->sigma >= 0.0) || !std::isfinite(pr->theta0) || !std::isfinite(pr->sigma))
    return fail(SG_EINVAL, "theta0 (mean) must be > 0 and sigma (CoV) >= 0");
  if (pr->M > 0 && (!pr->s || !pr->phi)) return fail(SG_EINVAL, "null KL arrays");
  return SG_OK;
}

// Chaos tables and the (block, term) lists: block (a, b) is stored if some
// coefficient term i with |i| <= 2p couples a and b.
int plan(const sg_problem* pr, Plan& pl) {
  const int M = pr->M, p = pr->p, ne2 = pr->n_e * pr->n_e;
  // sizes before any table is built: P = C(M+p, p) chaos functions, T = C(M+2p, 2p) coefficient terms
  auto binom = [](int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
  };
  const double P_est = binom(M + p, p), T_est = binom(M + 2 * p, 2 * p);
  if (P_est * P_est > double(1L << 22)) return fail(SG_EINVAL, "too many chaos blocks (P^2 > 2^22)");
  if (T_est > double(1 << 20) || T_est * ne2 > 2.5e8)
    return fail(SG_EINVAL, "too many coefficient terms (C(M+2p, 2p) > 2^20 or times n_e^2 > 2.5e8)");
  pl.alpha = graded(M, p);
  pl.coef = graded(M, 2 * p);
  pl.P = (int)pl.alpha.size();
  pl.T = (int)pl.coef.size();
  if ((long)pl.P * pl.P > (1L << 22)) return fail(SG_EINVAL, "too many chaos blocks (P^2 > 2^22)");
  std::unordered_map<unsigned long long, int> index;
  const unsigned base = 2u * (unsigned)p + 1u;
  if (M * std::log2((double)base) >= 63.0) return fail(SG_EINVAL, "M and p too large for the coefficient index");
  auto key = [&](const std::vector<int>& v) {
    unsigned long long k = 0;
    for (int d = 0; d < M; ++d) k = k * base + (unsigned)v[d];
    return k;
  };
  for (int t = 0; t < pl.T; ++t) index[key(pl.coef[t])] = t;
  pl.ptr.assign(1, 0);
  pl.rptr.assign(1, 0);
  std::vector<int> cur(M);
  for (int a = 0; a < pl.P; ++a) {
    for (int b = 0; b < pl.P; ++b) {
      const std::vector<int>&A = pl.alpha[a], &B = pl.alpha[b];
      const long before = (long)pl.term.size();
      // per dimension i_d runs over |a_d - b_d|, +2, ..., a_d + b_d
      std::vector<int> lo(M), hi(M);
      for (int d = 0; d < M; ++d) {
        lo[d] = std::abs(A[d] - B[d]);
        hi[d] = A[d] + B[d];
      }
      for (int d = 0; d < M; ++d) cur[d] = lo[d];
      if (M == 0) {
        pl.term.push_back(0);
        pl.g.push_back(1.0);
      } else {
        while (true) {
          int deg = 0;
          for (int d = 0; d < M; ++d) deg += cur[d];
          if (deg <= 2 * p) {
            double gv = 1.0;
            for (int d = 0; d < M && gv != 0.0; ++d) gv *= triple(cur[d], A[d], B[d]);
            if (gv != 0.0) {
              pl.term.push_back(index.at(key(cur)));
              pl.g.push_back(gv);
            }
          }
          int d = M - 1;
          while (d >= 0 && cur[d] + 2 > hi[d]) {
            cur[d] = lo[d];
            --d;
          }
          if (d < 0) break;
          cur[d] += 2;
        }
      }
      if (pl.term.size() > (size_t(1) << 28)) return fail(SG_EINVAL, "too many (block, term) couplings (> 2^28)");
      if ((long)pl.term.size() > before) {
        pl.ptr.push_back((long)pl.term.size());
        pl.rcol.push_back(b);
        pl.rslot.push_back(pl.nslots++);
      }
    }
    pl.rptr.push_back((int)pl.rcol.size());
  }
  if (pl.rcol.empty() || pl.rcol[0] != 0) return fail(SG_EINVAL, "internal: block (0, 0) is not the first slot");
  size_t tot = 0;
  pl.o_C = take(tot, sizeof(double) * (size_t)pl.nslots * ne2);
  pl.o_kc = take(tot, sizeof(double) * (size_t)pl.T * ne2);
  pl.o_ptr = take(tot, sizeof(long) * pl.ptr.size());
  pl.o_term = take(tot, sizeof(int) * std::max<size_t>(1, pl.term.size()));
  pl.o_g = take(tot, sizeof(double) * std::max<size_t>(1, pl.g.size()));
  pl.o_rptr = take(tot, sizeof(int) * pl.rptr.size());
  pl.o_rcol = take(tot, sizeof(int) * std::max<size_t>(1, pl.rcol.size()));
  pl.o_rslot = take(tot, sizeof(int) * std::max<size_t>(1, pl.rslot.size()));
  const size_t nP = (size_t)(pr->n_e - 1) * (pr->n_e - 1) * pl.P;
  pl.o_vec = take(tot, sizeof(double) * nP * 12);
  pl.o_part = take(tot, sizeof(double) * 2 * kLognDotBlocks);  // two partial sets
  pl.total = tot;
  return SG_OK;
}

// Deterministic FP64 dot product: device partials, host sum in index order.
int dotp(sg_logn_ctx* h, const double* x, const double* y, long len, double& out) {
  sgk::launch_logn_dot(x, y, len, h->part, kLognDotBlocks, h->stream);
  SG_HIP(hipMemcpyAsync(h->host_part.data(), h->part, sizeof(double) * kLognDotBlocks, hipMemcpyDeviceToHost,
                        h->stream));
  SG_HIP(hipStreamSynchronize(h->stream));
  double s = 0.0;
  for (int i = 0; i < kLognDotBlocks; ++i) s += h->host_part[i];
  out = s;
  return SG_OK;
}

// Block solve by Jacobi-preconditioned CG from X = 0 to ||r|| <= rtol ||B||
// or maxit iterations, on the n x nr system of
//   kind 0: the diagonal sub-block of A over chaos columns lo..lo+nr-1 (a
//           level block D_l of Section 6, where the level blocks couple, or one
//           block A_aa);
//   kind 1: I (x) K(k_0) over nr columns (the mean-based preconditioner).
// B and X: n x nr device blocks.
int range_solve(sg_logn_ctx* h, int kind, int lo, int nr, const double* B, double* X, double rtol, int maxit,
                long& its) {
  const long len = h->n * (long)nr;
  hipStream_t s = h->stream;
  const double* dinv = kind == 0 ? h->Dinv + (long)lo * h->n : h->Dinv;  // column 0: K(k_0)
  const long dn = kind == 0 ? len : h->n;
  double bb = 0.0, rz = 0.0, pq = 0.0, rr = 0.0, rzn = 0.0;
  int rc = dotp(h, B, B, len, bb);
  if (rc) return rc;
  sgk::launch_logn_axpby(len, 0.0, B, 0.0, X, 0, nullptr, 0, s);  // X = 0
  if (bb == 0.0) return SG_OK;
  sgk::launch_logn_axpby(len, 1.0, B, 0.0, h->cr, 0, nullptr, 0, s);    // r = B
  sgk::launch_logn_axpby(len, 0.0, h->cr, 0.0, h->cz, 1, dinv, dn, s);   // z = D^-1 r
  sgk::launch_logn_axpby(len, 1.0, h->cz, 0.0, h->cp, 0, nullptr, 0, s);  // p = z
  if ((rc = dotp(h, h->cr, h->cz, len, rz))) return rc;
  for (int it = 0; it < maxit; ++it) {
    if (kind == 0)
      sgk::launch_logn_apply(h->rptr, h->rcol, h->rslot, h->C, h->cp, h->n_e, h->n, lo, nr, lo, lo + nr, 0, nullptr,
                             h->cq, s);
    else
      sgk::launch_logn_mean_apply(h->C, h->cp, h->n_e, h->n, nr, h->cq, s);  // block (0, 0) is slot 0
    if ((rc = dotp(h, h->cp, h->cq, len, pq))) return rc;
    if (!(pq > 0.0) || !std::isfinite(pq)) break;
    const double alpha = rz / pq;
    // x += alpha p, r -= alpha q, z = D^-1 r and the partials of r.r and r.z in one pass
    sgk::launch_logn_cg_update(len, alpha, h->cp, h->cq, X, h->cr, dinv, dn, h->cz, h->part, kLognDotBlocks, s);
    SG_HIP(hipMemcpyAsync(h->host_part.data(), h->part, sizeof(double) * 2 * kLognDotBlocks, hipMemcpyDeviceToHost,
                          s));
    SG_HIP(hipStreamSynchronize(s));
    rr = 0.0;
    rzn = 0.0;
    for (int i = 0; i < kLognDotBlocks; ++i) rr += h->host_part[i];
    for (int i = 0; i < kLognDotBlocks; ++i) rzn += h->host_part[kLognDotBlocks + i];
    ++its;
    if (rr <= rtol * rtol * bb) break;
    const double beta = rzn / rz;
    rz = rzn;
    sgk::launch_logn_axpby(len, 1.0, h->cz, beta, h->cp, 0, nullptr, 0, s);
  }
  return SG_OK;
}

int level_solve(sg_logn_ctx* h, int l, const double* B, double* X, double rtol, int maxit, long& its) {
  return range_solve(h, 0, h->off[l], h->off[l + 1] - h->off[l], B, X, rtol, maxit, its);
}

// Block symmetric Gauss-Seidel over the chaos blocks (Section 6) from zero:
// forward a = 0..P-1: xf_a = A_aa^-1 (r_a - sum_{b<a} A_ab xf_b); backward
// a = P-1..0: x_a = A_aa^-1 (r_a - sum_{b<a} A_ab xf_b - sum_{b>a} A_ab x_b).
int bgs_apply(sg_logn_ctx* h, const double* R, double* Z, double rtol, int maxit, long& its) {
  hipStream_t s = h->stream;
  const long n = h->n;
  int rc;
  for (int a = 0; a < h->P; ++a) {
    sgk::launch_logn_apply(h->rptr, h->rcol, h->rslot, h->C, h->XF, h->n_e, n, a, 1, 0, a, 1, R + a * n, h->W, s);
    if ((rc = range_solve(h, 0, a, 1, h->W, h->XF + a * n, rtol, maxit, its))) return rc;
  }
  for (int a = h->P - 1; a >= 0; --a) {
    sgk::launch_logn_apply(h->rptr, h->rcol, h->rslot, h->C, h->XF, h->n_e, n, a, 1, 0, a, 1, R + a * n, h->W, s);
    sgk::launch_logn_apply(h->rptr, h->rcol, h->rslot, h->C, Z + (a + 1) * n, h->n_e, n, a, 1, a + 1, h->P, 1, h->W,
                           h->W, s);
    if ((rc = range_solve(h, 0, a, 1, h->W, Z + a * n, rtol, maxit, its))) return rc;
  }
  return SG_OK;
}

// One action of Algorithm 1 with the full level blocks: down sweep
// y_l = D_l^-1 r_l, r_{<l} -= B_l y_l (l = p..1); u_0 = D_0^-1 r_0; up sweep
// u_l = D_l^-1 (r_l - C_l u_{<l}) (l = 1..p). Z receives u.
int hsc_apply(sg_logn_ctx* h, const double* R, double* Z, double rtol, int maxit, long& its) {
  const long nP = h->n * (long)h->P;
  hipStream_t s = h->stream;
  sgk::launch_logn_axpby(nP, 1.0, R, 0.0, h->Rh, 0, nullptr, 0, s);
  int rc;
  for (int l = h->p; l >= 1; --l) {
    const int lo = h->off[l], hi = h->off[l + 1];
    if ((rc = level_solve(h, l, h->Rh + (long)lo * h->n, Z + (long)lo * h->n, rtol, maxit, its))) return rc;
    sgk::launch_logn_apply(h->rptr, h->rcol, h->rslot, h->C, Z + (long)lo * h->n, h->n_e, h->n, 0, lo, lo, hi, 1,
                           h->Rh, h->Rh, s);
  }
  if ((rc = level_solve(h, 0, h->Rh, Z, rtol, maxit, its))) return rc;
  for (int l = 1; l <= h->p; ++l) {
    const int lo = h->off[l], hi = h->off[l + 1];
    sgk::launch_logn_apply(h->rptr, h->rcol, h->rslot, h->C, Z, h->n_e, h->n, lo, hi - lo, 0, lo, 1,
                           h->Rh + (long)lo * h->n, h->W, s);
    if ((rc = level_solve(h, l, h->W, Z + (long)lo * h->n, rtol, maxit, its))) return rc;
  }
  return SG_OK;
}

}  // namespace

extern "C" {

int sg_logn_workspace_bytes(const sg_problem* prob, size_t* bytes) {
  int rc = validate(prob);
  if (rc) return rc;
  if (!bytes) return fail(SG_EINVAL, "null output");
  Plan pl;
  rc = plan(prob, pl);
  if (rc) return rc;
  *bytes = pl.total;
  return SG_OK;
}

int sg_logn_setup(const sg_problem* pr, void* workspace, size_t workspace_bytes, void* stream, sg_logn_handle* out) {
  int rc = validate(pr);
  if (rc) return rc;
  if (!out || !workspace) return fail(SG_EINVAL, "null workspace or output handle");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255u) != 0) return fail(SG_EINVAL, "workspace must be 256-byte aligned");
  Plan pl;
  rc = plan(pr, pl);
  if (rc) return rc;
  if (workspace_bytes < pl.total) return fail(SG_ENOMEM, "workspace too small");
  const int n_e = pr->n_e, M = pr->M, ne2 = n_e * n_e;
  // Chaos coefficients of exp(g) (Section 6; the Gaussian field carries the KL
  // data and the lognormal mean and CoV fix its mean and variance):
  // k_i(e) = exp(mu_g + sum_k g_k(e)^2 / 2) prod_k g_k(e)^{i_k} / sqrt(i_k!).
  const double sg2 = std::log(1.0 + pr->sigma * pr->sigma);
  const double mu_g = std::log(pr->theta0) - 0.5 * sg2;
  const double sgm = std::sqrt(sg2);
  std::vector<double> gk((size_t)M * ne2), base(ne2);
  for (int e = 0; e < ne2; ++e) {
    double q = 0.0;
    for (int k = 0; k < M; ++k) {
      const double v = sgm * pr->s[k] * pr->phi[(size_t)k * ne2 + e];
      gk[(size_t)k * ne2 + e] = v;
      q += v * v;
    }
    base[e] = std::exp(mu_g + 0.5 * q);
  }
  std::vector<double> kc((size_t)pl.T * ne2);
  for (int t = 0; t < pl.T; ++t) {
    double norm = 1.0;
    for (int k = 0; k < M; ++k) norm *= std::sqrt(factorial(pl.coef[t][k]));
    for (int e = 0; e < ne2; ++e) {
      double v = base[e];
      for (int k = 0; k < M; ++k)
        for (int j = 0; j < pl.coef[t][k]; ++j) v *= gk[(size_t)k * ne2 + e];
      kc[(size_t)t * ne2 + e] = v / norm;
    }
  }
  auto* h = new (std::nothrow) sg_logn_ctx();
  if (!h) return fail(SG_ENOMEM, "host allocation failed");
  h->n_e = n_e;
  h->M = M;
  h->p = pr->p;
  h->P = pl.P;
  h->n = (long)(n_e - 1) * (n_e - 1);
  h->nslots = pl.nslots;
  h->stream = (hipStream_t)stream;
  char* w = (char*)workspace;
  h->C = (double*)(w + pl.o_C);
  h->rptr = (int*)(w + pl.o_rptr);
  h->rcol = (int*)(w + pl.o_rcol);
  h->rslot = (int*)(w + pl.o_rslot);
  {
    const size_t nP = (size_t)h->n * pl.P;
    double* v = (double*)(w + pl.o_vec);
    double** vecs[12] = {&h->R,  &h->Z,  &h->Pv, &h->Q,  &h->Rh,   &h->W,
                         &h->cr, &h->cz, &h->cp, &h->cq, &h->Dinv, &h->XF};
    for (int i = 0; i < 12; ++i) *vecs[i] = v + i * nP;
    h->part = (double*)(w + pl.o_part);
    h->host_part.assign(2 * kLognDotBlocks, 0.0);
    h->off.assign(1, 0);
    for (int d = 0; d <= pr->p; ++d) {
      int cnt = 0;
      for (const auto& al : pl.alpha) {
        int deg = 0;
        for (int v2 : al) deg += v2;
        if (deg == d) ++cnt;
      }
      h->off.push_back(h->off.back() + cnt);
    }
  }
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, h->stream) : hipSuccess;
  };
  hipError_t e = up(pl.o_kc, kc.data(), sizeof(double) * kc.size());
  if (e == hipSuccess) e = up(pl.o_ptr, pl.ptr.data(), sizeof(long) * pl.ptr.size());
  if (e == hipSuccess) e = up(pl.o_term, pl.term.data(), sizeof(int) * pl.term.size());
  if (e == hipSuccess) e = up(pl.o_g, pl.g.data(), sizeof(double) * pl.g.size());
  if (e == hipSuccess) e = up(pl.o_rptr, pl.rptr.data(), sizeof(int) * pl.rptr.size());
  if (e == hipSuccess) e = up(pl.o_rcol, pl.rcol.data(), sizeof(int) * pl.rcol.size());
  if (e == hipSuccess) e = up(pl.o_rslot, pl.rslot.data(), sizeof(int) * pl.rslot.size());
  if (e == hipSuccess) {
    sgk::launch_logn_blocks((const long*)(w + pl.o_ptr), (const int*)(w + pl.o_term), (const double*)(w + pl.o_g),
                            (const double*)(w + pl.o_kc), ne2, pl.nslots, h->C, h->stream);
    sgk::launch_logn_invdiag(h->rptr, h->rcol, h->rslot, h->C, n_e, h->n, pl.P, h->Dinv, h->stream);
    e = hipGetLastError();
  }
  // the host tables are freed on return: wait for the copies
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    delete h;
    return fail(SG_EDEVICE, std::string("lognormal setup: ") + hipGetErrorString(e));
  }
  *out = h;
  return SG_OK;
}

int sg_logn_sizes(sg_logn_handle h, int64_t* n, int32_t* P, int32_t* nblocks) {
  if (!h) return fail(SG_EINVAL, "null handle");
  if (n) *n = h->n;
  if (P) *P = h->P;
  if (nblocks) *nblocks = h->nslots;
  return SG_OK;
}

int sg_logn_matvec(sg_logn_handle h, const double* U, double* Y) {
  if (!h || !U || !Y) return fail(SG_EINVAL, "null argument");
  if (U == Y) return fail(SG_EINVAL, "U and Y must be distinct");
  sgk::launch_logn_matvec(h->rptr, h->rcol, h->rslot, h->C, U, h->n_e, h->n, h->P, Y, h->stream);
  SG_HIP(hipGetLastError());
  return SG_OK;
}

int sg_logn_solve(sg_logn_handle h, int32_t precond, const double* F, double* U, double rtol, int32_t maxit,
                  double inner_rtol, int32_t inner_maxit, int32_t* outer_it, int64_t* inner_it, double* relres,
                  double* kappa) {
  if (!h || !F || !U) return fail(SG_EINVAL, "null argument");
  if (precond != SG_PC_HSC && precond != SG_PC_MEAN && precond != SG_PC_BGS)
    return fail(SG_EINVAL, "precond must be SG_PC_HSC, SG_PC_MEAN or SG_PC_BGS");
  if (F == U) return fail(SG_EINVAL, "F and U must be distinct");
  if (!(rtol >= 0.0) || maxit < 0 || !(inner_rtol > 0.0 && inner_rtol < 1.0) || inner_maxit < 1)
    return fail(SG_EINVAL, "need rtol >= 0, maxit >= 0, 0 < inner_rtol < 1, inner_maxit >= 1");
  const long nP = h->n * (long)h->P;
  hipStream_t s = h->stream;
  // flexible CG (Section 5) on A with Algorithm 1 as the preconditioner
  sgk::launch_logn_axpby(nP, 0.0, F, 0.0, U, 0, nullptr, 0, s);  // U = 0
  sgk::launch_logn_axpby(nP, 1.0, F, 0.0, h->R, 0, nullptr, 0, s);
  double ff = 0.0, rr = 0.0;
  int rc = dotp(h, F, F, nP, ff);
  if (rc) return rc;
  if (!std::isfinite(ff)) return fail(SG_EINVAL, "right-hand side is not finite");
  std::vector<double> al, be;
  long its_in = 0;
  int it = 0, status = SG_NOT_CONVERGED;
  double rel = ff > 0.0 ? 1.0 : 0.0, pq_prev = 0.0;
  if (ff == 0.0 || rel <= rtol) status = SG_OK;
  for (; status == SG_NOT_CONVERGED && it < maxit; ++it) {
    if (precond == SG_PC_HSC)
      rc = hsc_apply(h, h->R, h->Z, inner_rtol, inner_maxit, its_in);
    else if (precond == SG_PC_BGS)
      rc = bgs_apply(h, h->R, h->Z, inner_rtol, inner_maxit, its_in);
    else  // each column its own K(k_0) solve, so every column meets the inner tolerance
      for (int a = 0; a < h->P && !rc; ++a)
        rc = range_solve(h, 1, 0, 1, h->R + a * h->n, h->Z + a * h->n, inner_rtol, inner_maxit, its_in);
    if (rc) return rc;
    if (it == 0) {
      sgk::launch_logn_axpby(nP, 1.0, h->Z, 0.0, h->Pv, 0, nullptr, 0, s);
    } else {
      double zq = 0.0;
      if ((rc = dotp(h, h->Z, h->Q, nP, zq))) return rc;
      const double beta = -zq / pq_prev;
      be.push_back(beta);
      sgk::launch_logn_axpby(nP, 1.0, h->Z, beta, h->Pv, 0, nullptr, 0, s);
    }
    sgk::launch_logn_matvec(h->rptr, h->rcol, h->rslot, h->C, h->Pv, h->n_e, h->n, h->P, h->Q, s);
    double pq = 0.0, pr = 0.0;
    if ((rc = dotp(h, h->Pv, h->Q, nP, pq))) return rc;
    if (!(pq > 0.0) || !std::isfinite(pq)) {
      status = SG_BREAKDOWN;
      break;
    }
    if ((rc = dotp(h, h->Pv, h->R, nP, pr))) return rc;
    const double alpha = pr / pq;
    al.push_back(alpha);
    sgk::launch_logn_axpby(nP, alpha, h->Pv, 1.0, U, 0, nullptr, 0, s);
    sgk::launch_logn_axpby(nP, -alpha, h->Q, 1.0, h->R, 0, nullptr, 0, s);
    pq_prev = pq;
    if ((rc = dotp(h, h->R, h->R, nP, rr))) return rc;
    rel = std::sqrt(rr / ff);
    if (!std::isfinite(rel)) {
      status = SG_BREAKDOWN;
      ++it;
      break;
    }
    if (rel <= rtol) {
      status = SG_OK;
      ++it;
      break;
    }
  }
  SG_HIP(hipStreamSynchronize(s));
  if (outer_it) *outer_it = it;
  if (inner_it) *inner_it = its_in;
  if (relres) *relres = rel;
  if (kappa) *kappa = al.empty() ? 1.0 : sgh::lanczos_kappa(al, be);
  if (status == SG_NOT_CONVERGED) return fail(SG_NOT_CONVERGED, "outer iteration did not converge");
  if (status == SG_BREAKDOWN) return fail(SG_BREAKDOWN, "breakdown: non-positive or non-finite curvature");
  return SG_OK;
}

void sg_logn_destroy(sg_logn_handle h) { delete h; }

}  // extern "C"
