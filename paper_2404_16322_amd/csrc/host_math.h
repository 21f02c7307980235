// Host-side numerics of the fit: symmetric eigendecomposition for the PCA rotation,
// logistic-regression training and the target-recall bias adjustment of the correction.
#pragma once

#include <stdint.h>

#include <vector>

namespace ddc {

// SplitMix64 (Steele, Lea & Flood 2014): output for state x (state advanced by the golden gamma).
uint64_t splitmix64(uint64_t x);
// key(seed, tag, i) = splitmix64(splitmix64(seed + tag) + i)
uint64_t ctr_key(uint64_t seed, uint64_t tag, uint64_t i);
// Indices (ascending) of the m smallest keys among 0..n-1, ties by index; all if m >= n.
std::vector<int64_t> select_by_key(int64_t n, int64_t m, uint64_t seed, uint64_t tag);

enum : uint64_t { TAG_PCA = 1, TAG_KMEANS_INIT = 2, TAG_KMEANS_SAMPLE = 3, TAG_NEG = 4, TAG_CALIB = 5,
                  TAG_HAAR = 6, TAG_PQ_SAMPLE = 7 };

// OPQ eigenvalue allocation: the axes (eigenvalues lam, largest first) dealt to M subspaces of
// D/M axes, each to the non-full subspace with the smallest product of its eigenvalues over
// their geometric mean (lowest index on ties); perm[j * D/M + t] = axis t of subspace j,
// ascending within a subspace.
std::vector<int32_t> opq_allocation(const std::vector<double> &lam, int M);

// A Haar-distributed random rotation (Mezzadri 2007): Householder QR of a D x D matrix of
// standard normals (Box-Muller over pairs of counter keys, row-major), every column of Q
// signed so that the triangular factor's diagonal is positive; rows of `R` = columns of Q.
void haar_rotation(int D, uint64_t seed, std::vector<double> &R);

// Eigen-decomposition of the symmetric n x n matrix A (row-major, FP64): Householder
// reduction to tridiagonal form, then implicit QL iterations with Wilkinson-type shifts.
// Returns eigenvalues in `lam` and eigenvectors as the rows of `vecs` (vecs[i*n + j]),
// ordered by eigenvalue, largest first (index order on ties); every eigenvector is signed
// so that its largest-magnitude component (first one on ties) is positive.
bool sym_eig_desc(const std::vector<double> &A, int n, std::vector<double> &lam,
                  std::vector<double> &vecs);

// Logistic regression (cross-entropy, +ridge/2 |w|^2 without the intercept) of labels y on
// features F (n x 2, row-major), solved by Newton's method on standardised features.
// Returns b, w1, w2 in the original units.
void logistic_fit(const std::vector<double> &F, const std::vector<double> &y, double &b,
                  double &w1, double &w2);
// The same for p = 1..3 features (F: n x p, row-major): w[p] in the original units.
void logistic_fit_p(const std::vector<double> &F, int p, const std::vector<double> &y, double &b,
                    std::vector<double> &w);

// beta_s(alpha) from the label-0 residual matrix G (n0 x st, row-major); mode 0 = joint,
// 1 = per-stage alpha / st.  alpha <= 0 -> -inf.
std::vector<double> beta_for_alpha(const std::vector<double> &G, int64_t n0, int st, double alpha,
                                   int mode);

}  // namespace ddc
