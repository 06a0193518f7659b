// Host-side small dense linear algebra shared by the library's host code: a
// Hermitian eigensolver (the Rayleigh-Ritz step of the eigenmode solver,
// spectral norms of per-voxel blocks in canonicalisation) and the inverse of
// a small complex matrix.
#pragma once
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace usp_host {

// Eigen-decomposition of a Hermitian n x n matrix (row-major) by cyclic Jacobi
// sweeps: each step turns a_pq real by a phase on column/row q, then zeroes it
// with a real plane rotation.  w ascending, Z columns orthonormal eigenvectors.
inline int hermitian_jacobi(int n, std::vector<std::complex<double>> a, std::vector<double>& w,
                            std::vector<std::complex<double>>& Z) {
  typedef std::complex<double> zd;
  Z.assign((size_t)n * n, zd(0.0));
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  auto A = [&](int i, int j) -> zd& { return a[(size_t)i * n + j]; };
  double scale = 0.0;
  for (const zd& v : a) scale = std::max(scale, std::abs(v));
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off = std::max(off, std::abs(A(p, q)));
    if (!(off > 1e-15 * scale)) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double g = std::abs(A(p, q));
        if (!(g > 1e-300)) continue;
        // phase: column q times e, row q times conj(e), so that a_pq becomes |a_pq|
        const zd e = std::conj(A(p, q)) / g;
        for (int k = 0; k < n; ++k) A(k, q) *= e;
        for (int k = 0; k < n; ++k) A(q, k) *= std::conj(e);
        for (int k = 0; k < n; ++k) Z[(size_t)k * n + q] *= e;
        // real rotation on (p, q) zeroing the (now real) a_pq
        const double app = A(p, p).real(), aqq = A(q, q).real(), apq = A(p, q).real();
        const double th = (aqq - app) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const zd kp = A(k, p), kq = A(k, q);
          A(k, p) = c * kp - sn * kq;
          A(k, q) = sn * kp + c * kq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const zd pk = A(p, k), qk = A(q, k);
          A(p, k) = c * pk - sn * qk;
          A(q, k) = sn * pk + c * qk;
        }
        A(p, q) = A(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {
          const zd kp = Z[(size_t)k * n + p], kq = Z[(size_t)k * n + q];
          Z[(size_t)k * n + p] = c * kp - sn * kq;
          Z[(size_t)k * n + q] = sn * kp + c * kq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int i, int j) { return A(i, i).real() < A(j, j).real(); });
  std::vector<zd> Zs((size_t)n * n);
  w.resize(n);
  for (int jj = 0; jj < n; ++jj) {
    w[jj] = A(idx[jj], idx[jj]).real();
    for (int k = 0; k < n; ++k) Zs[(size_t)k * n + jj] = Z[(size_t)k * n + idx[jj]];
  }
  Z.swap(Zs);
  return 0;
}

// inverse of a d x d complex matrix (row-major, d <= 3) by Gauss-Jordan
// elimination with partial pivoting; false if singular
inline bool small_inverse(int d, const std::complex<double>* m, std::complex<double>* inv) {
  typedef std::complex<double> cd;
  cd a[3][6];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      a[i][j] = m[i * d + j];
      a[i][d + j] = (i == j) ? 1.0 : 0.0;
    }
  for (int c = 0; c < d; ++c) {
    int piv = c;
    for (int r = c + 1; r < d; ++r)
      if (std::abs(a[r][c]) > std::abs(a[piv][c])) piv = r;
    if (!(std::abs(a[piv][c]) > 0.0)) return false;
    if (piv != c)
      for (int j = 0; j < 2 * d; ++j) std::swap(a[c][j], a[piv][j]);
    const cd ip = 1.0 / a[c][c];
    for (int j = 0; j < 2 * d; ++j) a[c][j] *= ip;
    for (int r = 0; r < d; ++r) {
      if (r == c) continue;
      const cd f = a[r][c];
      if (f == cd(0.0)) continue;
      for (int j = 0; j < 2 * d; ++j) a[r][j] -= f * a[c][j];
    }
  }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) inv[i * d + j] = a[i][d + j];
  return true;
}

}  // namespace usp_host
