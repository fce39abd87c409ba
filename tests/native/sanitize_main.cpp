// Host build of the library's CPU-side code under AddressSanitizer and
// UndefinedBehaviorSanitizer: the convection-diffusion generator and the CSR
// transpose (gen.cpp), the red-black preconditioner tables (rbhost.h), the
// small dense routines (small.h) and the tolerance controller
// (controller.h), each exercised on the shapes the library meets.  Any
// sanitizer report aborts the program; a logic check failing returns 1.
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "../../include/lradi.h"
#include "../../paper_2312_02891_amd/csrc/controller.h"
#include "../../paper_2312_02891_amd/csrc/rbhost.h"
#include "../../paper_2312_02891_amd/csrc/small.h"

namespace lradi {
void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vfprintf(stderr, fmt, ap);
  va_end(ap);
  fputc('\n', stderr);
}
void csr_transpose(int n, const int32_t* rp, const int32_t* ci, const double* v, std::vector<int32_t>& trp,
                   std::vector<int32_t>& tci, std::vector<double>& tv);
}  // namespace lradi

static int fails = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

static void check_generator_and_tables(int dim, int N, const double* omega) {
  int64_t n = 0, nnz = 0;
  CHECK(lradi_convdiff_size(dim, N, &n, &nnz) == LRADI_OK);
  std::vector<int32_t> rp(n + 1), ci(nnz);
  std::vector<double> v(nnz);
  CHECK(lradi_gen_convdiff(dim, N, omega, rp.data(), ci.data(), v.data()) == LRADI_OK);
  CHECK(rp[0] == 0 && rp[n] == nnz);
  std::vector<int32_t> trp, tci;
  std::vector<double> tv;
  lradi::csr_transpose((int)n, rp.data(), ci.data(), v.data(), trp, tci, tv);
  CHECK((int64_t)tci.size() == nnz && trp[n] == nnz);
  for (int tiles : {0, 1, 7, 64}) {
    lradi::RbHost h;
    CHECK(lradi::rb_host_build((int)n, rp.data(), ci.data(), v.data(), trp.data(), tci.data(), tv.data(),
                               tiles, h));
    CHECK(h.nred >= 1 && h.nred <= n && (int64_t)h.rows.size() == n);
  }
}

int main() {
  const double w2[2] = {12.0, -7.0}, w3[3] = {6.0, -3.0, 2.0};
  check_generator_and_tables(2, 1, w2);
  check_generator_and_tables(2, 37, w2);
  check_generator_and_tables(3, 2, w3);
  check_generator_and_tables(3, 13, w3);
  // invalid arguments come back as errors, not memory errors
  int64_t n = 0, nnz = 0;
  CHECK(lradi_convdiff_size(4, 10, &n, &nnz) != LRADI_OK);
  CHECK(lradi_convdiff_size(2, 0, &n, &nnz) != LRADI_OK);

  std::mt19937_64 rng(7);
  std::normal_distribution<double> nd;
  for (int r = 1; r <= 8; ++r) {
    // SPD Gram of r random columns, then the small routines on it
    std::vector<double> X(3 * r * r), G(r * r, 0.0), S(r * r), Si(r * r), A(r * r), Q(r * r);
    for (double& x : X) x = nd(rng);
    for (int a = 0; a < r; ++a)
      for (int b = 0; b < r; ++b)
        for (int i = 0; i < 3 * r; ++i) G[a * r + b] += X[i * r + a] * X[i * r + b];
    CHECK(lradi::chol_upper_reg(G.data(), S.data(), r, 1e-14) >= 0);
    lradi::tri_inv_upper(S.data(), Si.data(), r);
    A = G;
    lradi::jacobi_eig(A.data(), Q.data(), r);
    const double l1 = lradi::lambda_max_sym(G.data(), r);
    const double l2 = lradi::lambda_max_sym_ms<16>(G.data(), r);
    const double l3 = lradi::lambda_max_sym_ms<64>(G.data(), r);
    CHECK(std::fabs(l1 - l2) <= 1e-12 * l1 && std::fabs(l1 - l3) <= 1e-12 * l1);
    const double lp = lradi::lambda_max_prod(G.data(), G.data(), r);
    CHECK(std::fabs(lp - l1 * l1) <= 1e-10 * l1 * l1);
    std::vector<double> M(2 * r * r), H(4 * r * r);
    for (double& x : M) x = nd(rng);
    lradi::householder_2nxn(M.data(), H.data(), r);
  }
  // controller: every selection on random inputs, including spent budgets
  for (int it = 0; it < 2000; ++it) {
    lradi::CtlParams p{};
    p.eps = std::pow(10.0, -12.0 + 10.0 * (it % 97) / 97.0);
    p.delta_min = 5e-10;
    p.delta_max = 0.1;
    p.xi = 1.0;
    p.delta_fixed = 5e-10;
    p.rho = 1e-12;
    p.kmax = 50;
    p.selection = it % 6;
    p.backlook = it % 2;
    p.paper_abs = (it / 2) % 2;
    p.balance = (it / 4) % 2;
    const double nw = std::pow(10.0, nd(rng) * 3), nt = std::pow(10.0, nd(rng) * 3);
    double u = std::fabs(nd(rng)) * p.eps, v = std::fabs(nd(rng)) * p.eps, dA = 0, dB = 0;
    lradi::ctl_tolerances(p, 1 + it % 50, nw, nt, u, v, &dA, &dB);
    CHECK(dA > 0.0 && dB > 0.0 && std::isfinite(dA) && std::isfinite(dB));
    lradi::ctl_update_gap(&u, &v, -3.0, 2.0, 0.5, dA, dB);
    CHECK(std::isfinite(u) && std::isfinite(v));
  }
  std::printf("sanitized host checks: %d failures\n", fails);
  return fails == 0 ? 0 : 1;
}
