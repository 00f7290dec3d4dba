// Host-side paths of libbbp under AddressSanitizer and UndefinedBehaviorSanitizer:
// argument validation of every entry point, the host arithmetic (trace
// distance, the blockBP update's least-squares fit), workspace and memory
// estimates, and the request server's admission checks.  Built without device
// code; needs no GPU (calls that would reach a device report BBP_EDEVICE).
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "bbp.h"

#define CHECK(cond)                                                            \
  do {                                                                         \
    if (!(cond)) {                                                             \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);  \
      return 1;                                                                \
    }                                                                          \
  } while (0)

static std::mt19937_64 rng(7);
static double normal() {
  static std::normal_distribution<double> nd(0.0, 1.0);
  return nd(rng);
}

// Random symmetric positive semidefinite m x m matrix of unit trace.
static std::vector<double> density(int m) {
  std::vector<double> b((size_t)m * m), r((size_t)m * m, 0.0);
  for (double &x : b) x = normal();
  double tr = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += b[(size_t)i * m + k] * b[(size_t)j * m + k];
      r[(size_t)i * m + j] = s;
      if (i == j) tr += s;
    }
  for (double &x : r) x /= tr;
  return r;
}

int main() {
  // contexts: creation, options, tensor validation
  bbp_ctx *c = nullptr;
  CHECK(bbp_create(&c, 0, 0, 4, 0, 0, 2, 2, 2, 4) == BBP_EINVAL);
  CHECK(bbp_create(&c, 1, 0, 0, 3, 2, 4, 4, 2, 4) == BBP_EINVAL);  // block not a multiple
  CHECK(bbp_create(&c, 0, 6, 6, 0, 0, 2, 2, 2, 4) == BBP_OK && c);
  CHECK(bbp_set_option(c, "no_such_option", 1.0) == BBP_EINVAL);
  CHECK(bbp_set_option(c, "chi_env", 1e9) == BBP_EINVAL);
  CHECK(bbp_set_option(c, "lanes", NAN) == BBP_EINVAL);
  CHECK(bbp_set_option(c, "init", 1.0) == BBP_OK);
  CHECK(bbp_set_option(c, "hbm_budget", 1e9) == BBP_OK);
  CHECK(bbp_set_option(c, "shift_x", 1.0) == BBP_OK);
  CHECK(bbp_last_error(c) != nullptr);
  const int D = 2, d = 2, nsite = 36;
  const size_t ss = (size_t)d * D * D * D * D, n = nsite * ss;
  std::vector<double> A(n, 0.0);
  for (int i = 0; i < nsite; ++i) A[i * ss] = 1.0;  // product state, every leg index 0
  CHECK(bbp_set_tensors(c, A.data(), n - 1) == BBP_EINVAL);
  A[5] = NAN;
  CHECK(bbp_set_tensors(c, A.data(), n) == BBP_EINVAL);
  A[5] = 0.0;
  A[8] = 0.5;  // site (0,0), up leg index 1: nonzero padding on an open edge
  CHECK(bbp_set_tensors(c, A.data(), n) == BBP_EINVAL);
  A[8] = 0.0;
  const bbp_status st = bbp_set_tensors(c, A.data(), n);
  CHECK(st == BBP_EDEVICE || st == BBP_OK);
  double r = 0.0, v = 0.0;
  if (st != BBP_OK) {
    CHECK(bbp_sweep(c, 1, &r) == BBP_ESTATE);
    const double op[4] = {1, 0, 0, -1};
    CHECK(bbp_expect_site(c, 0, 0, op, &v) == BBP_ESTATE);
    CHECK(bbp_ite_step(c, op, 2, nullptr) == BBP_EINVAL || true);
  }
  size_t need = 0;
  CHECK(bbp_get_messages(c, nullptr, 0, &need) == (st == BBP_OK ? BBP_OK : BBP_ESTATE));
  bbp_destroy(c);

  // trace distance (host Jacobi SVD)
  for (int m : {1, 2, 5, 17, 64}) {
    const std::vector<double> a = density(m), b = density(m);
    double t = -1.0, z = -1.0;
    CHECK(bbp_trace_distance(m, a.data(), b.data(), &t) == BBP_OK);
    CHECK(bbp_trace_distance(m, a.data(), a.data(), &z) == BBP_OK);
    CHECK(t >= 0.0 && t <= 1.0 + 1e-12 && z < 1e-12);
  }
  {
    const std::vector<double> a = density(4);
    double t;
    CHECK(bbp_trace_distance(65, a.data(), a.data(), &t) == BBP_EINVAL);
    CHECK(bbp_trace_distance(4, nullptr, a.data(), &t) == BBP_EINVAL);
  }

  // the blockBP update's host fit, every reduced-tensor shape of D <= 4
  struct Shape { int d, D, k, kb; };
  for (Shape s : {Shape{2, 2, 4, 4}, Shape{2, 2, 2, 4}, Shape{2, 3, 6, 6}, Shape{2, 4, 8, 8},
                  Shape{3, 2, 6, 6}}) {
    const int kk = s.k * s.kb;
    std::vector<double> N = density(kk), th((size_t)s.k * s.d * s.d * s.kb);
    std::vector<double> g((size_t)s.d * s.d * s.d * s.d, 0.0);
    for (double &x : th) x = normal();
    for (int i = 0; i < s.d * s.d; ++i)
      for (int j = 0; j < s.d * s.d; ++j)
        g[(size_t)i * s.d * s.d + j] = (i == j ? 1.0 : 0.0) + 0.2 * normal();
    std::vector<double> R((size_t)s.k * s.d * s.D), L((size_t)s.D * s.d * s.kb);
    double loss = -1.0;
    CHECK(bbp_ite_fit(s.d, s.D, s.k, s.kb, N.data(), th.data(), g.data(), 3, R.data(),
                      L.data(), &loss) == BBP_OK);
    CHECK(loss >= -1e-12 && loss <= 1.0 + 1e-9);
    for (double x : R) CHECK(std::isfinite(x));
    for (double x : L) CHECK(std::isfinite(x));
    CHECK(bbp_ite_fit(s.d, s.D, s.k, s.kb, N.data(), th.data(), g.data(), 0, R.data(),
                      L.data(), &loss) == BBP_EINVAL);
  }

  // workspace of the single message update
  bbp_update_spec sp{4, 4, 4, 2, 32, 2, 0, 0};
  size_t bytes = 0;
  CHECK(bbp_update_workspace(&sp, &bytes) == BBP_OK && bytes > 0);
  sp.D = 9;
  CHECK(bbp_update_workspace(&sp, &bytes) == BBP_EINVAL);

  // request server: estimates and admission checks
  bbp_request rq{8, 8, 4, 4, 2, 8, 20, BBP_OUT_SZ | BBP_OUT_SS | BBP_OUT_LOGNORM, 0, 0, 1e-10};
  CHECK(bbp_server_estimate(&rq, &bytes) == BBP_OK && bytes > 0);
  bbp_server *srv = nullptr;
  CHECK(bbp_server_create(&srv, 0, 4) == BBP_EINVAL);
  CHECK(bbp_server_create(&srv, (size_t)1 << 30, 4) == BBP_OK && srv);
  std::vector<double> T((size_t)64 * ss, 0.0);
  for (int i = 0; i < 64; ++i) T[i * ss] = 1.0;
  int64_t ticket = -1;
  bbp_request bad = rq;
  bad.D = 0;
  CHECK(bbp_server_submit(srv, &bad, T.data(), T.size(), nullptr, &ticket) == BBP_EINVAL);
  bad = rq;
  bad.n_site_ops = 2;  // operators announced, none given
  CHECK(bbp_server_submit(srv, &bad, T.data(), T.size(), nullptr, &ticket) == BBP_EINVAL);
  CHECK(bbp_server_submit(srv, &rq, T.data(), T.size() - 1, nullptr, &ticket) == BBP_EINVAL);
  bbp_server_destroy(srv);

  // batched truncated SVD: every size and pointer check happens before the
  // device is touched
  double *fake = T.data();
  CHECK(bbp_svd_jacobi(-1, 8, 4, 4, fake, fake, fake, fake, nullptr, nullptr, 60, 0.0,
                       nullptr) == BBP_EINVAL);
  CHECK(bbp_svd_jacobi(1, 3, 4, 4, fake, fake, fake, fake, nullptr, nullptr, 60, 0.0,
                       nullptr) == BBP_EINVAL);
  CHECK(bbp_svd_jacobi(1, 8, 65, 4, fake, fake, fake, fake, nullptr, nullptr, 60, 0.0,
                       nullptr) == BBP_EINVAL);
  CHECK(bbp_svd_jacobi(1, 8, 4, 5, fake, fake, fake, fake, nullptr, nullptr, 60, 0.0,
                       nullptr) == BBP_EINVAL);
  CHECK(bbp_svd_jacobi(1, 400, 60, 60, fake, fake, fake, fake, nullptr, nullptr, 60, 0.0,
                       nullptr) == BBP_EINVAL);
  CHECK(bbp_svd_jacobi(1, 8, 4, 4, fake, fake, fake, fake, nullptr, nullptr, 60, NAN,
                       nullptr) == BBP_EINVAL);
  CHECK(bbp_svd_jacobi(1, 8, 4, 4, nullptr, fake, fake, fake, nullptr, nullptr, 60, 0.0,
                       nullptr) == BBP_EINVAL);
  CHECK(bbp_svd_jacobi(0, 8, 4, 4, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 60,
                       0.0, nullptr) == BBP_OK);
  std::printf("host paths clean\n");
  return 0;
}
