// Host numerics of the fit run under AddressSanitizer and UndefinedBehaviorSanitizer (built with
// g++ by tests/test_sanitize.py, no device code).  Each check states a property the result
// must have; the program exits 1 on the first violation, and the sanitizers abort on any
// memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "host_math.h"

using namespace ddc;

static int fails = 0;
#define CHECK(c, ...)                      \
  do {                                     \
    if (!(c)) {                            \
      std::printf("FAIL %s: ", #c);        \
      std::printf(__VA_ARGS__);            \
      std::printf("\n");                   \
      ++fails;                             \
    }                                      \
  } while (0)

static double unif(uint64_t &s) {
  s = splitmix64(s);
  return (double)(s >> 11) * (1.0 / 9007199254740992.0);
}

int main() {
  uint64_t st = 12345;
  // symmetric eigendecomposition: A v_i = lam_i v_i, rows orthonormal, lam descending
  for (int n : {1, 2, 3, 7, 32, 65}) {
    std::vector<double> A((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = unif(st) - 0.5;
    std::vector<double> lam, V;
    CHECK(sym_eig_desc(A, n, lam, V), "n=%d", n);
    CHECK((int)lam.size() == n && (int)V.size() == n * n, "n=%d sizes", n);
    double worst = 0.0, orth = 0.0;
    for (int i = 0; i < n; ++i) {
      if (i) CHECK(lam[i - 1] >= lam[i], "n=%d order at %d", n, i);
      for (int r = 0; r < n; ++r) {
        double av = 0.0;
        for (int c = 0; c < n; ++c) av += A[(size_t)r * n + c] * V[(size_t)i * n + c];
        worst = std::fmax(worst, std::fabs(av - lam[i] * V[(size_t)i * n + r]));
      }
      for (int j = 0; j < n; ++j) {
        double dot = 0.0;
        for (int c = 0; c < n; ++c) dot += V[(size_t)i * n + c] * V[(size_t)j * n + c];
        orth = std::fmax(orth, std::fabs(dot - (i == j ? 1.0 : 0.0)));
      }
    }
    CHECK(worst < 1e-10 && orth < 1e-10, "n=%d residual %g orthogonality %g", n, worst, orth);
  }
  // Haar rotation: orthogonal
  for (int D : {1, 5, 40}) {
    std::vector<double> R;
    haar_rotation(D, 7, R);
    double orth = 0.0;
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        double dot = 0.0;
        for (int c = 0; c < D; ++c) dot += R[(size_t)i * D + c] * R[(size_t)j * D + c];
        orth = std::fmax(orth, std::fabs(dot - (i == j ? 1.0 : 0.0)));
      }
    CHECK(orth < 1e-12, "D=%d orthogonality %g", D, orth);
  }
  // logistic regression: label 1 iff e > tau (noisy), so w1 > 0 > w2 and the boundary m = -w1/w2 > 0
  {
    const int n = 4000;
    std::vector<double> F(2 * n), y(n);
    for (int i = 0; i < n; ++i) {
      const double e = unif(st) * 10.0, tau = unif(st) * 10.0;
      F[2 * i] = e;
      F[2 * i + 1] = tau;
      y[i] = (e + 0.3 * (unif(st) - 0.5) > tau) ? 1.0 : 0.0;
    }
    double b, w1, w2;
    logistic_fit(F, y, b, w1, w2);
    CHECK(std::isfinite(b) && w1 > 0 && w2 < 0, "b=%g w1=%g w2=%g", b, w1, w2);
    CHECK(std::fabs(-w1 / w2 - 1.0) < 0.1, "m=%g", -w1 / w2);
    std::vector<double> F3(3 * n), w;
    for (int i = 0; i < n; ++i) {
      F3[3 * i] = F[2 * i];
      F3[3 * i + 1] = unif(st);
      F3[3 * i + 2] = F[2 * i + 1];
    }
    logistic_fit_p(F3, 3, y, b, w);
    CHECK(w.size() == 3 && w[0] > 0 && w[2] < 0, "p=3 weights");
  }
  // beta(alpha): non-decreasing in alpha, -inf at alpha = 0
  {
    const int64_t n0 = 500;
    const int stn = 3;
    std::vector<double> G((size_t)n0 * stn);
    for (auto &g : G) g = unif(st) * 4.0 - 1.0;
    for (int mode : {0, 1}) {
      std::vector<double> prev = beta_for_alpha(G, n0, stn, 0.0, mode);
      for (double v : prev) CHECK(std::isinf(v) && v < 0, "alpha=0 mode %d", mode);
      for (double a : {0.001, 0.01, 0.05, 0.2, 0.5, 0.9}) {
        std::vector<double> bb = beta_for_alpha(G, n0, stn, a, mode);
        CHECK((int)bb.size() == stn, "size");
        for (int s = 0; s < stn; ++s) CHECK(bb[s] >= prev[s], "mode %d alpha %g stage %d", mode, a, s);
        prev = bb;
      }
    }
  }
  // selection by counter keys: m distinct ascending indices
  for (int64_t n : {1, 10, 1000}) {
    for (int64_t m : {0, 1, 5, 2000}) {
      auto sel = select_by_key(n, m, 99, TAG_PCA);
      CHECK((int64_t)sel.size() == std::min(n, m), "n=%lld m=%lld", (long long)n, (long long)m);
      for (size_t i = 1; i < sel.size(); ++i) CHECK(sel[i - 1] < sel[i], "ascending");
      for (auto v : sel) CHECK(v >= 0 && v < n, "range");
    }
  }
  // OPQ allocation: a permutation of the axes, ascending within each subspace
  {
    std::vector<double> lam(64);
    for (int i = 0; i < 64; ++i) lam[i] = 1.0 / (1 + i);
    auto perm = opq_allocation(lam, 8);
    std::vector<int> seen(64, 0);
    for (auto p : perm) {
      CHECK(p >= 0 && p < 64, "axis");
      if (p >= 0 && p < 64) seen[p]++;
    }
    for (int i = 0; i < 64; ++i) CHECK(seen[i] == 1, "axis %d taken %d times", i, seen[i]);
    for (int j = 0; j < 8; ++j)
      for (int t = 1; t < 8; ++t) CHECK(perm[j * 8 + t - 1] < perm[j * 8 + t], "subspace %d order", j);
  }
  std::printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
  return fails ? 1 : 0;
}
