// Host-code workout for an AddressSanitizer / UndefinedBehaviorSanitizer build
// (tests/test_host_sanitizers.py builds it with g++ against the library's host
// sources): every host-only entry point on random and degenerate inputs, with
// a few consistency checks; any invalid access or undefined behaviour aborts.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "../../include/usp.h"
#include "../../paper_2207_14222_amd/csrc/hermitian.hpp"

static int failures = 0;
#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      std::printf("check failed line %d: %s\n", __LINE__, #c); \
      ++failures;                                             \
    }                                                         \
  } while (0)

static usp_symbol grid(int ndim, const int* shape, double h) {
  usp_symbol g{};
  g.ndim = ndim;
  for (int a = 0; a < ndim; ++a) {
    g.shape[a] = shape[a];
    g.spacing[a] = h;
  }
  return g;
}

int main() {
  std::mt19937_64 rng(1234);
  std::normal_distribution<double> N01(0.0, 1.0);
  // smallest circle: random, duplicated, collinear, tiny sets, both kinds
  for (int trial = 0; trial < 60; ++trial) {
    const int n = trial < 6 ? trial + 1 : 1 + (int)(rng() % 400);
    std::vector<double> p(2 * n);
    for (int i = 0; i < n; ++i) {
      if (trial % 7 == 3) {           // collinear
        const double t = N01(rng);
        p[2 * i] = 2.0 * t + 1.0;
        p[2 * i + 1] = -t;
      } else if (trial % 7 == 5) {    // many duplicates
        p[2 * i] = (double)(i % 3);
        p[2 * i + 1] = (double)(i % 2);
      } else {
        p[2 * i] = N01(rng) * 3.0;
        p[2 * i + 1] = N01(rng);
      }
    }
    for (int kind : {USP_BIAS_COMPLEX, USP_BIAS_REAL}) {
      double c[2], r;
      CHECK(usp_smallest_circle(p.data(), n, kind, c, &r) == 0);
      for (int i = 0; i < n; ++i)
        CHECK(std::hypot(p[2 * i] - c[0], p[2 * i + 1] - c[1]) <= r * (1 + 1e-9) + 1e-12);
    }
  }
  // Helmholtz / diffusion / Schrodinger canonical forms on small grids
  const int sh3[3] = {4, 8, 6};
  usp_symbol g3 = grid(3, sh3, 0.25), out{};
  const size_t n3 = 4 * 8 * 6;
  std::vector<double> k2(2 * n3), mu(n3);
  for (size_t i = 0; i < n3; ++i) {
    k2[2 * i] = 40.0 + 5.0 * N01(rng);
    k2[2 * i + 1] = std::fabs(N01(rng));
    mu[i] = 0.05 + 0.01 * std::fabs(N01(rng));
  }
  double c[2], b[2];
  CHECK(usp_canonical_helmholtz(k2.data(), n3, USP_BIAS_COMPLEX, nullptr, 0.95, &g3, &out, c, b) == 0);
  CHECK(usp_canonical_helmholtz(k2.data(), n3, USP_BIAS_REAL, nullptr, 0.95, &g3, &out, c, b) == 0);
  const double given[4] = {40.0, 0.5, 0.0, 10.0};
  CHECK(usp_canonical_helmholtz(k2.data(), n3, USP_BIAS_COMPLEX, given, 0.95, &g3, &out, c, b) == 0);
  CHECK(usp_canonical_diffusion(mu.data(), n3, 0.03, 0.01, 0.95, &g3, &out, c, b) == 0);
  CHECK(usp_canonical_schrodinger(mu.data(), n3, 2.0, 0.95, &g3, &out, c, b) == 0);
  std::vector<double> flat(n3, 1.0);
  CHECK(usp_canonical_schrodinger(flat.data(), n3, 2.0, 0.95, &g3, &out, c, b) != 0);
  // pantograph, several lengths and dilations (gather near both ends)
  for (int n : {8, 33, 256, 1000}) {
    for (double lam : {0.5, 0.9, 1.3}) {
      std::vector<double> a(2 * n), bb(2 * n), x0(2 * n, 0.0), B(2 * n), g0(2 * n), g1(2 * n), y(2 * n);
      std::vector<int32_t> idx(n);
      for (int i = 0; i < n; ++i) {
        a[2 * i] = 5.0 + N01(rng);
        a[2 * i + 1] = N01(rng);
        bb[2 * i] = -5.0;
        bb[2 * i + 1] = 0.0;
      }
      const double x0t0[2] = {1.0, 0.0};
      usp_symbol s{};
      CHECK(usp_canonical_pantograph(a.data(), bb.data(), n, lam, 1.0, 0.01, x0.data(), x0t0, 0.95, &s, B.data(),
                                     idx.data(), g0.data(), g1.data(), y.data(), c, b) == 0);
      for (int i = 0; i < n; ++i) CHECK(idx[i] >= 0 && idx[i] < n);
    }
  }
  // flux form, 2-D and 3-D, isotropic and anisotropic tensors
  for (int ndim : {2, 3}) {
    const int shape[3] = {4, 6, ndim == 3 ? 8 : 1};
    const size_t nv = (size_t)shape[0] * shape[1] * (ndim == 3 ? shape[2] : 1);
    std::vector<double> m(2 * nv), D(2 * ndim * ndim * nv, 0.0), src(2 * nv, 0.0);
    for (size_t v = 0; v < nv; ++v) {
      m[2 * v] = 0.1 + 0.05 * std::fabs(N01(rng));
      for (int i = 0; i < ndim; ++i) {
        D[2 * (v * ndim * ndim + i * ndim + i)] = 1.0 + std::fabs(N01(rng));
        if (i + 1 < ndim) {
          const double o = 0.2 * N01(rng);
          D[2 * (v * ndim * ndim + i * ndim + i + 1)] = o;
          D[2 * (v * ndim * ndim + (i + 1) * ndim + i)] = o;
        }
      }
      src[2 * v] = N01(rng);
    }
    usp_flux_symbol fs{};
    std::vector<double> bu(2 * nv), b2(2 * ndim * ndim * nv), yy(2 * (1 + ndim) * nv);
    CHECK(usp_canonical_flux(m.data(), D.data(), src.data(), ndim, shape, 0.3, 0.95, &fs, bu.data(), b2.data(),
                             yy.data()) == 0);
  }
  // Jacobi eigensolver: reconstruction of random Hermitian matrices
  for (int n : {1, 2, 5, 17, 40}) {
    std::vector<std::complex<double>> A((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j) {
        const std::complex<double> z(N01(rng), i == j ? 0.0 : N01(rng));
        A[(size_t)i * n + j] = z;
        A[(size_t)j * n + i] = std::conj(z);
      }
    std::vector<double> w;
    std::vector<std::complex<double>> Z;
    usp_host::hermitian_jacobi(n, A, w, Z);
    double err = 0.0, nrm = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        std::complex<double> s = 0.0;
        for (int k = 0; k < n; ++k) s += Z[(size_t)i * n + k] * w[k] * std::conj(Z[(size_t)j * n + k]);
        err += std::norm(s - A[(size_t)i * n + j]);
        nrm += std::norm(A[(size_t)i * n + j]);
      }
    CHECK(std::sqrt(err) <= 1e-10 * std::sqrt(nrm) + 1e-14);
  }
  std::printf("host sanitizer workout: %d failures\n", failures);
  return failures ? 1 : 0;
}
