"""Host-side numerics of the library (C++, no GPU) against the oracle: compiled with g++
into a scratch shared object and called through a small C wrapper."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_16322_amd", "csrc")

WRAP = r'''
#include "host_math.h"
#include <cstring>
extern "C" {
void hm_haar(int D, unsigned long long seed, double *R) {
  std::vector<double> r; ddc::haar_rotation(D, seed, r); std::memcpy(R, r.data(), r.size() * 8);
}
int hm_eig(const double *A, int n, double *lam, double *vecs) {
  std::vector<double> a(A, A + (size_t)n * n), l, v;
  if (!ddc::sym_eig_desc(a, n, l, v)) return 0;
  std::memcpy(lam, l.data(), n * 8); std::memcpy(vecs, v.data(), (size_t)n * n * 8); return 1;
}
void hm_logit(const double *F, const double *y, long n, double *out) {
  std::vector<double> f(F, F + 2 * n), yy(y, y + n);
  ddc::logistic_fit(f, yy, out[0], out[1], out[2]);
}
void hm_logit3(const double *F, const double *y, long n, double *out) {
  std::vector<double> f(F, F + 3 * n), yy(y, y + n), w;
  ddc::logistic_fit_p(f, 3, yy, out[0], w); std::memcpy(out + 1, w.data(), 24);
}
void hm_opq(const double *lam, int D, int M, int *out) {
  auto p = ddc::opq_allocation(std::vector<double>(lam, lam + D), M); std::memcpy(out, p.data(), D * 4);
}
void hm_beta(const double *G, long n0, int st, double alpha, int mode, double *out) {
  std::vector<double> g(G, G + n0 * st);
  auto b = ddc::beta_for_alpha(g, n0, st, alpha, mode); std::memcpy(out, b.data(), st * 8);
}
long hm_select(long n, long m, unsigned long long seed, unsigned long long tag, long long *out) {
  auto s = ddc::select_by_key(n, m, seed, tag); std::memcpy(out, s.data(), s.size() * 8); return (long)s.size();
}
}
'''


@pytest.fixture(scope="module")
def hm(tmp_path_factory):
    d = tmp_path_factory.mktemp("hm")
    (d / "wrap.cpp").write_text(WRAP)
    so = d / "libhm.so"
    subprocess.run(["g++", "-std=c++17", "-O2", "-shared", "-fPIC", f"-I{CSRC}", str(d / "wrap.cpp"),
                    os.path.join(CSRC, "host_math.cpp"), "-o", str(so)], check=True)
    lib = C.CDLL(str(so))
    vp = C.c_void_p
    lib.hm_haar.argtypes = [C.c_int, C.c_ulonglong, vp]
    lib.hm_eig.argtypes = [vp, C.c_int, vp, vp]
    lib.hm_logit.argtypes = [vp, vp, C.c_long, vp]
    lib.hm_beta.argtypes = [vp, C.c_long, C.c_int, C.c_double, C.c_int, vp]
    lib.hm_logit3.argtypes = [vp, vp, C.c_long, vp]
    lib.hm_opq.argtypes = [vp, C.c_int, C.c_int, vp]
    lib.hm_select.argtypes = [C.c_long, C.c_long, C.c_ulonglong, C.c_ulonglong, vp]
    lib.hm_select.restype = C.c_long
    return lib


def test_haar_rotation_equals_oracle(hm):
    for D, seed in [(16, 7), (33, 1), (128, 7)]:
        R = np.zeros((D, D))
        hm.hm_haar(D, seed, R.ctypes.data)
        np.testing.assert_allclose(R, O.haar_rotation(D, seed), atol=1e-12, rtol=0)


def test_eigendecomposition_equals_oracle_pca(hm, small_workload):
    p = O.pca_fit(small_workload["base"])
    D = p["cov"].shape[0]
    lam, V = np.zeros(D), np.zeros((D, D))
    cov = np.ascontiguousarray(p["cov"])
    assert hm.hm_eig(cov.ctypes.data, D, lam.ctypes.data, V.ctypes.data) == 1
    np.testing.assert_allclose(lam, p["lam"], rtol=1e-10, atol=1e-12 * p["lam"][0])
    gaps = np.minimum(np.r_[np.inf, -np.diff(lam)], np.r_[-np.diff(lam), np.inf]) / lam[0]
    sep = gaps > 1e-6
    np.testing.assert_allclose(V[sep], p["R"][sep], atol=1e-8)


def test_logistic_fit_equals_oracle_irls(hm):
    rng = np.random.default_rng(2)
    n = 3000
    F = np.column_stack([rng.gamma(2.0, 50.0, n), rng.gamma(3.0, 40.0, n)])
    y = (rng.random(n) < 1 / (1 + np.exp(-(0.05 * F[:, 0] - 0.04 * F[:, 1] + 0.3)))).astype(np.float64)
    out = np.zeros(3)
    Fc = np.ascontiguousarray(F)
    hm.hm_logit(Fc.ctypes.data, y.ctypes.data, n, out.ctypes.data)
    b, w = O.irls_logistic(F, y)
    np.testing.assert_allclose(out, [b, w[0], w[1]], rtol=1e-7, atol=1e-10)


def test_beta_and_key_selection_equal_oracle(hm):
    rng = np.random.default_rng(3)
    G = rng.standard_normal((500, 4)) * 10
    for mode, name in [(0, "joint"), (1, "bonferroni")]:
        for a in [0.0, 0.01, 0.1, 0.5]:
            out = np.zeros(4)
            hm.hm_beta(np.ascontiguousarray(G).ctypes.data, 500, 4, a, mode, out.ctypes.data)
            np.testing.assert_array_equal(out, O.beta_for_alpha(G, a, name))
    out = np.zeros(100, np.int64)
    k = hm.hm_select(5000, 100, 11, O.TAG_CALIB, out.ctypes.data)
    assert k == 100 and out.tolist() == O.select_by_key(5000, 100, 11, O.TAG_CALIB).tolist()


def test_three_feature_logistic_fit_equals_oracle_irls(hm):
    rng = np.random.default_rng(4)
    n = 3000
    F = np.column_stack([rng.gamma(2.0, 50.0, n), rng.gamma(1.5, 5.0, n), rng.gamma(3.0, 40.0, n)])
    t = 0.05 * F[:, 0] + 0.1 * F[:, 1] - 0.04 * F[:, 2] + 0.3
    y = (rng.random(n) < 1 / (1 + np.exp(-t))).astype(np.float64)
    out = np.zeros(4)
    hm.hm_logit3(np.ascontiguousarray(F).ctypes.data, y.ctypes.data, n, out.ctypes.data)
    b, w = O.irls_logistic(F, y)
    np.testing.assert_allclose(out, [b, *w], rtol=1e-7, atol=1e-10)


def test_opq_allocation_equals_oracle(hm):
    for lam, M in [(1.0 / np.arange(1, 129), 32), (np.arange(1, 961) ** -1.2, 120),
                   (np.array([16.0, 8, 4, 2, 1, 1]), 3), (np.r_[np.ones(8), np.zeros(8)], 4)]:
        out = np.zeros(lam.size, np.int32)
        hm.hm_opq(np.ascontiguousarray(lam).ctypes.data, lam.size, M, out.ctypes.data)
        assert out.reshape(M, -1).tolist() == O.opq_allocation(lam, M).tolist()
