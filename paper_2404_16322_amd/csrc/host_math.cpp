// Host numerics of the fit.  See host_math.h.
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <stdexcept>

namespace ddc {

uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t ctr_key(uint64_t seed, uint64_t tag, uint64_t i) { return splitmix64(splitmix64(seed + tag) + i); }

std::vector<int64_t> select_by_key(int64_t n, int64_t m, uint64_t seed, uint64_t tag) {
  std::vector<int64_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  if (m >= n) return idx;
  const uint64_t base = splitmix64(seed + tag);
  std::vector<uint64_t> key(n);
  for (int64_t i = 0; i < n; ++i) key[i] = splitmix64(base + (uint64_t)i);
  auto less = [&](int64_t a, int64_t b) { return key[a] < key[b] || (key[a] == key[b] && a < b); };
  std::nth_element(idx.begin(), idx.begin() + m, idx.end(), less);
  idx.resize(m);
  std::sort(idx.begin(), idx.end());
  return idx;
}

// ---------------------------------------------------------------------------------------
// Symmetric eigenproblem.  Householder: for column k, reflect the sub-column x = A[k+1:, k]
// onto alpha e_1 with H = I - 2 v v^T (v = x - alpha e_1 normalised); A <- H A H updates the
// trailing block as A' -= 2 (v w^T + w v^T), w = A'v - (v^T A' v) v.  Accumulated
// Q = H_0 H_1 ... gives A = Q T Q^T.  Then the tridiagonal T is diagonalised by implicit
// QL sweeps (Givens rotations chasing the bulge from the bottom), each rotation also
// applied to the columns of Q.
// ---------------------------------------------------------------------------------------
static void tridiagonalise(std::vector<double> &A, int n, std::vector<double> &Q,
                           std::vector<double> &d, std::vector<double> &e) {
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), p(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the sub-column
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) {
      const double x = A[(size_t)(k + 1 + i) * n + k];
      nrm += x * x;
    }
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const double x0 = A[(size_t)(k + 1) * n + k];
    const double alpha = x0 > 0 ? -nrm : nrm;
    for (int i = 0; i < m; ++i) v[i] = A[(size_t)(k + 1 + i) * n + k];
    v[0] -= alpha;
    double vn = 0.0;
    for (int i = 0; i < m; ++i) vn += v[i] * v[i];
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = 0; i < m; ++i) v[i] /= vn;
    // p = A' v on the trailing block (rows/cols k+1..n-1)
    for (int i = 0; i < m; ++i) {
      const double *row = &A[(size_t)(k + 1 + i) * n + k + 1];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = s;
    }
    double K = 0.0;
    for (int i = 0; i < m; ++i) K += v[i] * p[i];
    for (int i = 0; i < m; ++i) w[i] = p[i] - K * v[i];
    for (int i = 0; i < m; ++i) {
      double *row = &A[(size_t)(k + 1 + i) * n + k + 1];
      const double vi = v[i], wi = w[i];
      for (int j = 0; j < m; ++j) row[j] -= 2.0 * (vi * w[j] + wi * v[j]);
    }
    A[(size_t)(k + 1) * n + k] = alpha;
    A[(size_t)k * n + k + 1] = alpha;
    for (int i = 1; i < m; ++i) {
      A[(size_t)(k + 1 + i) * n + k] = 0.0;
      A[(size_t)k * n + k + 1 + i] = 0.0;
    }
    // Q[:, k+1:] <- Q[:, k+1:] (I - 2 v v^T)
    for (int r = 0; r < n; ++r) {
      double *row = &Q[(size_t)r * n + k + 1];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      s *= 2.0;
      for (int j = 0; j < m; ++j) row[j] -= s * v[j];
    }
  }
  d.resize(n);
  e.assign(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];  // e[i] couples i, i+1
}

static bool tridiag_ql(std::vector<double> &d, std::vector<double> &e, int n, std::vector<double> &Q) {
  // Q is row-major n x n; rotations act on its columns.  Work on the transpose for locality.
  std::vector<double> Qt((size_t)n * n);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) Qt[(size_t)c * n + r] = Q[(size_t)r * n + c];
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    for (;;) {
      int m = l;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      if (++iter > 60) return false;
      // shift from the leading 2x2 block of the unreduced segment
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        const double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        double *ci = &Qt[(size_t)i * n];
        double *cj = &Qt[(size_t)(i + 1) * n];
        for (int k = 0; k < n; ++k) {
          const double fk = cj[k];
          cj[k] = s * ci[k] + c * fk;
          ci[k] = c * ci[k] - s * fk;
        }
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) Q[(size_t)r * n + c] = Qt[(size_t)c * n + r];
  return true;
}

bool sym_eig_desc(const std::vector<double> &Ain, int n, std::vector<double> &lam,
                  std::vector<double> &vecs) {
  std::vector<double> A = Ain, Q, d, e;
  tridiagonalise(A, n, Q, d, e);
  if (!tridiag_ql(d, e, n, Q)) return false;
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] > d[b]; });
  lam.resize(n);
  vecs.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    const int c = order[i];
    lam[i] = d[c];
    int arg = 0;
    double best = -1.0;
    for (int j = 0; j < n; ++j) {
      const double a = std::fabs(Q[(size_t)j * n + c]);
      if (a > best) { best = a; arg = j; }
    }
    const double sgn = Q[(size_t)arg * n + c] < 0 ? -1.0 : 1.0;
    for (int j = 0; j < n; ++j) vecs[(size_t)i * n + j] = sgn * Q[(size_t)j * n + c];
  }
  return true;
}

// ---------------------------------------------------------------------------------------
void logistic_fit_p(const std::vector<double> &F, int p, const std::vector<double> &y, double &b,
                    std::vector<double> &wout) {
  if (p < 1 || p > 3) throw std::invalid_argument("logistic_fit_p: 1..3 features");
  const size_t n = y.size();
  const int q = p + 1;   // intercept + features
  double mean[3] = {0, 0, 0}, sd[3] = {0, 0, 0};
  for (size_t i = 0; i < n; ++i)
    for (int j = 0; j < p; ++j) mean[j] += F[p * i + j];
  for (int j = 0; j < p; ++j) mean[j] /= n;
  for (size_t i = 0; i < n; ++i)
    for (int j = 0; j < p; ++j) sd[j] += (F[p * i + j] - mean[j]) * (F[p * i + j] - mean[j]);
  for (int j = 0; j < p; ++j) {
    sd[j] = std::sqrt(sd[j] / n);
    if (sd[j] == 0) sd[j] = 1.0;
  }
  const double ridge = 1e-8;
  double w[4] = {0, 0, 0, 0};
  for (int it = 0; it < 100; ++it) {
    double g[4] = {0, 0, 0, 0}, H[4][4] = {{0}};
    for (size_t i = 0; i < n; ++i) {
      double z[4] = {1.0, 0, 0, 0};
      for (int j = 0; j < p; ++j) z[j + 1] = (F[p * i + j] - mean[j]) / sd[j];
      double t = w[0];
      for (int j = 1; j < q; ++j) t += w[j] * z[j];
      const double pr = 0.5 * (1.0 + std::tanh(0.5 * t));
      const double r = pr - y[i], wt = pr * (1.0 - pr);
      for (int a = 0; a < q; ++a) {
        g[a] += z[a] * r;
        for (int c = 0; c < q; ++c) H[a][c] += wt * z[a] * z[c];
      }
    }
    for (int a = 0; a < q; ++a) {
      g[a] /= n;
      for (int c = 0; c < q; ++c) H[a][c] /= n;
    }
    for (int a = 1; a < q; ++a) { g[a] += ridge * w[a]; H[a][a] += ridge; }
    // solve H x = g (Gaussian elimination with partial pivoting)
    double M[4][5];
    for (int a = 0; a < q; ++a) {
      for (int c = 0; c < q; ++c) M[a][c] = H[a][c];
      M[a][q] = g[a];
    }
    for (int col = 0; col < q; ++col) {
      int piv = col;
      for (int r = col + 1; r < q; ++r)
        if (std::fabs(M[r][col]) > std::fabs(M[piv][col])) piv = r;
      if (piv != col)
        for (int c = 0; c <= q; ++c) std::swap(M[col][c], M[piv][c]);
      const double dv = M[col][col] != 0 ? M[col][col] : 1e-300;
      for (int r = col + 1; r < q; ++r) {
        const double f = M[r][col] / dv;
        for (int c = col; c <= q; ++c) M[r][c] -= f * M[col][c];
      }
    }
    double x[4];
    for (int r = q - 1; r >= 0; --r) {
      double s2 = M[r][q];
      for (int c = r + 1; c < q; ++c) s2 -= M[r][c] * x[c];
      x[r] = s2 / (M[r][r] != 0 ? M[r][r] : 1e-300);
    }
    double mx = 0;
    for (int a = 0; a < q; ++a) {
      w[a] -= x[a];
      mx = std::max(mx, std::fabs(x[a]));
    }
    if (mx < 1e-12) break;
  }
  wout.assign(p, 0.0);
  b = w[0];
  for (int j = 0; j < p; ++j) {
    wout[j] = w[j + 1] / sd[j];
    b -= w[j + 1] * mean[j] / sd[j];
  }
}

void logistic_fit(const std::vector<double> &F, const std::vector<double> &y, double &b, double &w1,
                  double &w2) {
  std::vector<double> w;
  logistic_fit_p(F, 2, y, b, w);
  w1 = w[0];
  w2 = w[1];
}

std::vector<double> beta_for_alpha(const std::vector<double> &G, int64_t n0, int st, double alpha,
                                   int mode) {
  std::vector<double> beta(st, -std::numeric_limits<double>::infinity());
  if (alpha <= 0.0 || n0 == 0 || st == 0) return beta;
  std::vector<double> Gs((size_t)n0 * st);
  for (int s = 0; s < st; ++s) {
    std::vector<double> col(n0);
    for (int64_t j = 0; j < n0; ++j) col[j] = G[(size_t)j * st + s];
    std::sort(col.begin(), col.end());
    for (int64_t j = 0; j < n0; ++j) Gs[(size_t)j * st + s] = col[j];
  }
  int64_t k;
  if (mode == 1) {
    k = std::min<int64_t>((int64_t)std::floor(alpha * (double)n0 / st), n0 - 1);
  } else {
    auto frac = [&](int64_t kk) {
      int64_t cnt = 0;
      for (int64_t j = 0; j < n0; ++j) {
        for (int s = 0; s < st; ++s) {
          if (G[(size_t)j * st + s] < Gs[(size_t)kk * st + s]) { ++cnt; break; }
        }
      }
      return (double)cnt / (double)n0;
    };
    int64_t lo = 0, hi = n0 - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      if (frac(mid) <= alpha) lo = mid; else hi = mid - 1;
    }
    k = lo;
  }
  for (int s = 0; s < st; ++s) beta[s] = Gs[(size_t)k * st + s];
  return beta;
}

void haar_rotation(int D, uint64_t seed, std::vector<double> &R) {
  const int64_t cnt = (int64_t)D * D;
  std::vector<double> Z(cnt);
  const double two53 = 1.0 / 9007199254740992.0;   // 2^-53
  for (int64_t p = 0; 2 * p < cnt; ++p) {
    const double u1 = ((double)(ctr_key(seed, TAG_HAAR, 2 * p) >> 11) + 1.0) * two53;   // (0, 1]
    const double u2 = (double)(ctr_key(seed, TAG_HAAR, 2 * p + 1) >> 11) * two53;       // [0, 1)
    const double r = std::sqrt(-2.0 * std::log(u1));
    const double a = 2.0 * M_PI * u2;
    Z[2 * p] = r * std::cos(a);
    if (2 * p + 1 < cnt) Z[2 * p + 1] = r * std::sin(a);
  }
  // Householder QR: Z <- H_{D-1} ... H_0 Z (upper triangular), Q = H_0 ... H_{D-1}
  std::vector<double> Q((size_t)cnt, 0.0), v(D);
  for (int i = 0; i < D; ++i) Q[(size_t)i * D + i] = 1.0;
  for (int k = 0; k < D; ++k) {
    double nx = 0.0;
    for (int i = k; i < D; ++i) nx += Z[(size_t)i * D + k] * Z[(size_t)i * D + k];
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    const double x0 = Z[(size_t)k * D + k];
    const double alpha = x0 >= 0 ? -nx : nx;
    double vn = 0.0;
    for (int i = k; i < D; ++i) {
      v[i] = Z[(size_t)i * D + k] - (i == k ? alpha : 0.0);
      vn += v[i] * v[i];
    }
    if (vn == 0.0) continue;
    const double sc = 2.0 / vn;
    for (int j = k; j < D; ++j) {          // Z[k:, j] -= sc v (v . Z[k:, j])
      double d = 0.0;
      for (int i = k; i < D; ++i) d += v[i] * Z[(size_t)i * D + j];
      d *= sc;
      for (int i = k; i < D; ++i) Z[(size_t)i * D + j] -= d * v[i];
    }
    for (int i = 0; i < D; ++i) {          // Q[i, k:] -= sc (Q[i, k:] . v) v
      double d = 0.0;
      for (int j = k; j < D; ++j) d += Q[(size_t)i * D + j] * v[j];
      d *= sc;
      for (int j = k; j < D; ++j) Q[(size_t)i * D + j] -= d * v[j];
    }
  }
  R.assign((size_t)cnt, 0.0);
  for (int j = 0; j < D; ++j) {
    const double sg = Z[(size_t)j * D + j] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < D; ++i) R[(size_t)j * D + i] = sg * Q[(size_t)i * D + j];
  }
}

std::vector<int32_t> opq_allocation(const std::vector<double> &lam, int M) {
  const int D = (int)lam.size();
  if (M < 1 || D % M) throw std::invalid_argument("opq_allocation: M must divide D");
  const int dsub = D / M;
  double mx = 0;
  for (double v : lam) mx = std::max(mx, v);
  const double floor_v = mx > 0 ? mx * 1e-12 : 1e-300;
  std::vector<double> ll(D);
  double mean = 0;
  for (int i = 0; i < D; ++i) { ll[i] = std::log(std::max(lam[i], floor_v)); mean += ll[i]; }
  mean /= D;
  for (int i = 0; i < D; ++i) ll[i] -= mean;
  std::vector<int> order(D);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lam[a] > lam[b]; });
  std::vector<double> logp(M, 0.0);
  std::vector<std::vector<int32_t>> mem(M);
  for (int i : order) {
    int best = -1;
    for (int j = 0; j < M; ++j)
      if ((int)mem[j].size() < dsub && (best < 0 || logp[j] < logp[best])) best = j;
    mem[best].push_back(i);
    logp[best] += ll[i];
  }
  std::vector<int32_t> perm((size_t)D);
  for (int j = 0; j < M; ++j) {
    std::sort(mem[j].begin(), mem[j].end());
    for (int t = 0; t < dsub; ++t) perm[(size_t)j * dsub + t] = mem[j][t];
  }
  return perm;
}

}  // namespace ddc
