// Host-side checks of the library's C interface for a build with
// AddressSanitizer on a machine without a GPU: workspace queries, argument
// validation, and the host table building of sg_setup, sg_batch_setup and
// sg_logn_setup, which run before the first HIP call and must then fail
// cleanly with SG_EDEVICE. Exits 77 (skipped) when a HIP device is present,
// since the setup calls below hand the library a host buffer as workspace.
#include <hip/hip_runtime_api.h>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include "sg.h"

namespace {

int failures = 0, checks = 0;

void expect(bool ok, const char* what, int rc) {
  ++checks;
  if (!ok) {
    ++failures;
    std::fprintf(stderr, "FAIL %s (rc %d: %s)\n", what, rc, sg_last_error());
  }
}

struct Problem {
  std::vector<double> s, phi;
  sg_problem p{};
  Problem(int n_e, int M, int deg, int family, double theta0 = 1.0, double sigma = 0.2) {
    s.resize(M);
    phi.resize((size_t)M * n_e * n_e);
    for (int k = 0; k < M; ++k) {
      s[k] = 1.0 / (k + 1.0);
      for (int e = 0; e < n_e * n_e; ++e)
        phi[(size_t)k * n_e * n_e + e] = std::sin(0.37 * (k + 1) * (e % n_e) + 0.11 * (e / n_e));
    }
    p.n_e = n_e;
    p.M = M;
    p.p = deg;
    p.family = family;
    p.theta0 = theta0;
    p.sigma = sigma;
    p.s = M ? s.data() : nullptr;
    p.phi = M ? phi.data() : nullptr;
  }
};

sg_opts options(int prec = 64, int degree = 8, int tile = 0) {
  sg_opts o{};
  o.inner_precision = prec;
  o.cheb_degree = degree;
  o.inner_maxit = 100;
  o.precond = SG_PC_HSC;
  o.tile = tile;
  o.warm_start = 0;
  o.inner_rtol = 1e-4;
  return o;
}

void* host_workspace(size_t bytes) { return std::aligned_alloc(256, (bytes + 255) / 256 * 256); }

}  // namespace

int main() {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
    std::printf("SKIP: a HIP device is present\n");
    return 77;
  }
  char msg[160];
  // workspace queries over the option space
  for (int family : {SG_FAMILY_HERMITE, SG_FAMILY_LEGENDRE})
    for (int n_e : {3, 4, 17, 64})
      for (int M : {0, 1, 2, 4, 10})
        for (int deg : {0, 1, 3, 4}) {
          Problem pr(n_e, M, deg, family);
          for (int prec : {32, 64})
            for (int degree : {1, 8, 16})
              for (int tile : {0, 16, 32}) {
                sg_opts o = options(prec, degree, tile);
                size_t nb = 0;
                const int rc = sg_workspace_bytes(&pr.p, &o, &nb);
                std::snprintf(msg, sizeof msg, "workspace n_e=%d M=%d p=%d prec=%d d=%d tile=%d", n_e, M, deg, prec,
                              degree, tile);
                expect(rc == SG_OK && nb > 0, msg, rc);
              }
        }
  // rejected arguments
  {
    Problem pr(16, 4, 2, SG_FAMILY_HERMITE);
    sg_opts o = options();
    size_t nb = 0;
    expect(sg_workspace_bytes(nullptr, &o, &nb) == SG_EINVAL, "null problem", 0);
    expect(sg_workspace_bytes(&pr.p, nullptr, &nb) == SG_EINVAL, "null options", 0);
    expect(sg_workspace_bytes(&pr.p, &o, nullptr) == SG_EINVAL, "null output", 0);
    struct Bad {
      const char* what;
      void (*edit)(sg_problem&, sg_opts&);
    } bad[] = {
        {"n_e = 2", [](sg_problem& p, sg_opts&) { p.n_e = 2; }},
        {"M < 0", [](sg_problem& p, sg_opts&) { p.M = -1; }},
        {"p < 0", [](sg_problem& p, sg_opts&) { p.p = -1; }},
        {"family 7", [](sg_problem& p, sg_opts&) { p.family = 7; }},
        {"theta0 <= 0", [](sg_problem& p, sg_opts&) { p.theta0 = 0.0; }},
        {"sigma < 0", [](sg_problem& p, sg_opts&) { p.sigma = -0.1; }},
        {"P > 2^20", [](sg_problem& p, sg_opts&) { p.M = 40, p.p = 8; }},
        {"precision 48", [](sg_problem&, sg_opts& o) { o.inner_precision = 48; }},
        {"degree 0", [](sg_problem&, sg_opts& o) { o.cheb_degree = 0; }},
        {"degree 17", [](sg_problem&, sg_opts& o) { o.cheb_degree = 17; }},
        {"warm_start 2", [](sg_problem&, sg_opts& o) { o.warm_start = 2; }},
        {"null KL arrays", [](sg_problem& p, sg_opts&) { p.phi = nullptr; }},
        {"inner_maxit 0", [](sg_problem&, sg_opts& o) { o.inner_maxit = 0; }},
        {"precond 9", [](sg_problem&, sg_opts& o) { o.precond = 9; }},
        {"tile 8", [](sg_problem&, sg_opts& o) { o.tile = 8; }},
        {"inner_rtol NaN", [](sg_problem&, sg_opts& o) { o.inner_rtol = NAN; }},
        {"use_graph 2", [](sg_problem&, sg_opts& o) { o.use_graph = 2; }},
        {"reserved 1", [](sg_problem&, sg_opts& o) { o.reserved = 1; }},
    };
    for (const Bad& b : bad) {
      sg_problem p = pr.p;
      sg_opts oo = o;
      b.edit(p, oo);
      const int rc = sg_workspace_bytes(&p, &oo, &nb);
      expect(rc == SG_EINVAL && std::strlen(sg_last_error()) > 0, b.what, rc);
    }
  }
  // sg_setup: host tables, then SG_EDEVICE at the first HIP call
  for (int family : {SG_FAMILY_HERMITE, SG_FAMILY_LEGENDRE})
    for (auto shape : std::vector<std::vector<int>>{{3, 0, 0}, {4, 1, 1}, {16, 4, 2}, {16, 10, 3}, {33, 6, 4}}) {
      Problem pr(shape[0], shape[1], shape[2], family);
      sg_opts o = options(family == SG_FAMILY_HERMITE ? 64 : 32);
      size_t nb = 0;
      int rc = sg_workspace_bytes(&pr.p, &o, &nb);
      expect(rc == SG_OK, "setup workspace", rc);
      void* ws = host_workspace(nb);
      sg_handle h = nullptr;
      rc = sg_setup(&pr.p, &o, ws, nb, nullptr, &h);
      std::snprintf(msg, sizeof msg, "setup without device n_e=%d M=%d p=%d", shape[0], shape[1], shape[2]);
      expect(rc == SG_EDEVICE && h == nullptr, msg, rc);
      rc = sg_setup(&pr.p, &o, (char*)ws + 8, nb - 8, nullptr, &h);
      expect(rc == SG_EINVAL, "misaligned workspace", rc);
      rc = sg_setup(&pr.p, &o, ws, nb - 1, nullptr, &h);
      expect(rc == SG_ENOMEM, "workspace too small", rc);
      rc = sg_setup(&pr.p, &o, nullptr, nb, nullptr, &h);
      expect(rc == SG_EINVAL, "null workspace", rc);
      if (pr.p.M > 0) {
        pr.phi[pr.phi.size() / 2] = NAN;
        rc = sg_setup(&pr.p, &o, ws, nb, nullptr, &h);
        expect(rc == SG_EINVAL, "phi not finite", rc);
        pr.s[0] = INFINITY;
        rc = sg_setup(&pr.p, &o, ws, nb, nullptr, &h);
        expect(rc == SG_EINVAL, "s not finite", rc);
      }
      std::free(ws);
    }
  // batch: per-problem workspace plan, then SG_EDEVICE from the first member
  {
    Problem a(8, 2, 2, SG_FAMILY_HERMITE), b(16, 4, 3, SG_FAMILY_HERMITE), c(12, 3, 1, SG_FAMILY_HERMITE);
    sg_problem probs[3] = {a.p, b.p, c.p};
    sg_opts o = options(32, 8, 32);
    size_t nb = 0;
    int rc = sg_batch_workspace_bytes(3, probs, &o, &nb);
    expect(rc == SG_OK && nb > 0, "batch workspace", rc);
    expect(sg_batch_workspace_bytes(0, probs, &o, &nb) == SG_EINVAL, "batch of zero problems", 0);
    expect(sg_batch_workspace_bytes(3, nullptr, &o, &nb) == SG_EINVAL, "batch null problems", 0);
    void* ws = host_workspace(nb);
    sg_batch bh = nullptr;
    rc = sg_batch_setup(3, probs, &o, ws, nb, nullptr, &bh);
    expect(rc == SG_EDEVICE && bh == nullptr, "batch setup without device", rc);
    rc = sg_batch_setup(3, probs, &o, ws, nb - 1, nullptr, &bh);
    expect(rc == SG_ENOMEM, "batch workspace too small", rc);
    std::free(ws);
  }
  // lognormal coefficient: triple-product tables in the workspace query and setup
  for (int n_e : {4, 10, 30})
    for (int M : {0, 1, 2, 4})
      for (int deg : {1, 2, 4}) {
        Problem pr(n_e, M, deg, SG_FAMILY_HERMITE, 1.0, 1.0);
        size_t nb = 0;
        int rc = sg_logn_workspace_bytes(&pr.p, &nb);
        std::snprintf(msg, sizeof msg, "lognormal workspace n_e=%d M=%d p=%d", n_e, M, deg);
        expect(rc == SG_OK && nb > 0, msg, rc);
        if (rc != SG_OK) continue;
        void* ws = host_workspace(nb);
        sg_logn_handle h = nullptr;
        rc = sg_logn_setup(&pr.p, ws, nb, nullptr, &h);
        std::snprintf(msg, sizeof msg, "lognormal setup without device n_e=%d M=%d p=%d", n_e, M, deg);
        expect(rc == SG_EDEVICE && h == nullptr, msg, rc);
        std::free(ws);
      }
  {
    Problem pr(10, 2, 2, SG_FAMILY_HERMITE, 1.0, 1.0);
    size_t nb = 0;
    sg_problem p = pr.p;
    p.sigma = -0.5;
    expect(sg_logn_workspace_bytes(&p, &nb) == SG_EINVAL, "lognormal CoV < 0", 0);
    p = pr.p;
    p.theta0 = 0.0;
    expect(sg_logn_workspace_bytes(&p, &nb) == SG_EINVAL, "lognormal mean 0", 0);
    p = pr.p;
    p.family = SG_FAMILY_LEGENDRE;
    expect(sg_logn_workspace_bytes(&p, &nb) == SG_EINVAL, "lognormal Legendre", 0);
    expect(sg_logn_workspace_bytes(&pr.p, nullptr) == SG_EINVAL, "lognormal null output", 0);
  }
  sg_destroy(nullptr);
  sg_batch_destroy(nullptr);
  sg_logn_destroy(nullptr);
  std::printf("%d checks, %d failures\n", checks, failures);
  return failures ? 1 : 0;
}
