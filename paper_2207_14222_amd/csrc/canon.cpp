// Host canonicalisation helpers (Sec. 2.2, 3.1): the smallest disc enclosing the
// diagonal entries of the raw V0 gives the bias (its centre) and, divided by
// 0.95, the scale |c|.
//
// Complex centre: Welzl's randomised incremental algorithm (expected linear
// time), run over the points in a seeded random order.  Real-axis centre:
// golden-section search of the convex function b -> max_j |z_j - b|.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <complex>
#include <cstdint>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "../../include/usp.h"
#include "hermitian.hpp"

namespace {

struct Pt {
  double x, y;
};
struct Circle {
  double x, y, r;
};

inline bool inside(const Circle& c, const Pt& p) {
  const double dx = p.x - c.x, dy = p.y - c.y;
  const double d = std::sqrt(dx * dx + dy * dy);
  return d <= c.r * (1.0 + 1e-12) + 1e-300;
}

Circle from2(const Pt& a, const Pt& b) {
  const double cx = 0.5 * (a.x + b.x), cy = 0.5 * (a.y + b.y);
  return {cx, cy, 0.5 * std::hypot(a.x - b.x, a.y - b.y)};
}

Circle from3(const Pt& a, const Pt& b, const Pt& c) {
  // circumcircle via the perpendicular-bisector linear system, relative to a
  const double bx = b.x - a.x, by = b.y - a.y, cx = c.x - a.x, cy = c.y - a.y;
  const double d = 2.0 * (bx * cy - by * cx);
  if (std::fabs(d) < 1e-300) {
    // collinear: the widest pair
    Circle c1 = from2(a, b), c2 = from2(a, c), c3 = from2(b, c);
    if (c1.r >= c2.r && c1.r >= c3.r) return c1;
    return c2.r >= c3.r ? c2 : c3;
  }
  const double b2 = bx * bx + by * by, c2 = cx * cx + cy * cy;
  const double ux = (cy * b2 - by * c2) / d, uy = (bx * c2 - cx * b2) / d;
  return {a.x + ux, a.y + uy, std::hypot(ux, uy)};
}

Circle welzl(std::vector<Pt>& p) {
  std::mt19937_64 rng(12345);
  std::shuffle(p.begin(), p.end(), rng);
  const size_t n = p.size();
  Circle c{p[0].x, p[0].y, 0.0};
  for (size_t i = 1; i < n; ++i) {
    if (inside(c, p[i])) continue;
    c = {p[i].x, p[i].y, 0.0};
    for (size_t j = 0; j < i; ++j) {
      if (inside(c, p[j])) continue;
      c = from2(p[i], p[j]);
      for (size_t k = 0; k < j; ++k) {
        if (inside(c, p[k])) continue;
        c = from3(p[i], p[j], p[k]);
      }
    }
  }
  return c;
}

double farthest(const std::vector<Pt>& p, double bx, double by) {
  double m = 0.0;
  for (const Pt& q : p) m = std::max(m, (q.x - bx) * (q.x - bx) + (q.y - by) * (q.y - by));
  return std::sqrt(m);
}

}  // namespace

extern "C" int usp_smallest_circle(const double* pts, size_t n, int kind, double* centre_out, double* radius_out) {
  if (!pts || !centre_out || !radius_out || n == 0) return USP_ERR_INVALID;
  // de-duplicate (media hold few distinct values)
  std::vector<Pt> p(n);
  for (size_t i = 0; i < n; ++i) p[i] = {pts[2 * i], pts[2 * i + 1]};
  std::sort(p.begin(), p.end(), [](const Pt& a, const Pt& b) { return a.x < b.x || (a.x == b.x && a.y < b.y); });
  p.erase(std::unique(p.begin(), p.end(), [](const Pt& a, const Pt& b) { return a.x == b.x && a.y == b.y; }),
          p.end());
  for (const Pt& q : p)
    if (!std::isfinite(q.x) || !std::isfinite(q.y)) return USP_ERR_NAN;
  if (kind == USP_BIAS_COMPLEX) {
    Circle c = welzl(p);
    centre_out[0] = c.x;
    centre_out[1] = c.y;
    *radius_out = farthest(p, c.x, c.y);
    return 0;
  }
  if (kind == USP_BIAS_REAL) {
    double lo = p.front().x, hi = p.back().x;
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    double a = hi - g * (hi - lo), b = lo + g * (hi - lo);
    double fa = farthest(p, a, 0.0), fb = farthest(p, b, 0.0);
    for (int it = 0; it < 200 && (hi - lo) > 1e-15 * (1.0 + std::fabs(lo) + std::fabs(hi)); ++it) {
      if (fa <= fb) {
        hi = b; b = a; fb = fa;
        a = hi - g * (hi - lo);
        fa = farthest(p, a, 0.0);
      } else {
        lo = a; a = b; fa = fb;
        b = lo + g * (hi - lo);
        fb = farthest(p, b, 0.0);
      }
    }
    const double bc = 0.5 * (lo + hi);
    centre_out[0] = bc;
    centre_out[1] = 0.0;
    *radius_out = farthest(p, bc, 0.0);
    return 0;
  }
  return USP_ERR_INVALID;
}

namespace {
int fill_grid(const usp_symbol* grid, usp_symbol* out) {
  if (!grid || !out) return USP_ERR_INVALID;
  *out = *grid;
  out->s[0] = out->s[1] = out->a0[0] = out->a0[1] = out->a1[0] = out->a1[1] = out->a2[0] = out->a2[1] = 0.0;
  out->nyquist_zero = 0;
  return 0;
}
void cdiv(double ar, double ai, double br, double bi, double* o) {
  const double d = br * br + bi * bi;
  o[0] = (ar * br + ai * bi) / d;
  o[1] = (ai * br - ar * bi) / d;
}
}  // namespace

// Helmholtz (Sec. 3.1): (laplacian + k^2) psi = -S.  kbar^2 = smallest-circle
// centre of {k^2} (or the best real centre), c = -R/(vnorm i) = i R / vnorm, so
// that max|v| = vnorm and A = (laplacian + k^2)/c is accretive.  With `given`
// (kbar^2 re, im, c re, im) both are taken from the caller.  Symbol:
// l(p) = (-|p|^2 + kbar^2)/c.
extern "C" int usp_canonical_helmholtz(const double* k2_host, size_t n, int bias_kind, const double* given,
                                       double vnorm, const usp_symbol* grid, usp_symbol* sym_out, double* c_out,
                                       double* bias_out) {
  if (!c_out || !bias_out || !(vnorm > 0.0 && vnorm < 1.0)) return USP_ERR_INVALID;
  int rc = fill_grid(grid, sym_out);
  if (rc) return rc;
  double centre[2], R = 0.0;
  if (given) {
    centre[0] = given[0];
    centre[1] = given[1];
    c_out[0] = given[2];
    c_out[1] = given[3];
  } else {
    if (!k2_host) return USP_ERR_INVALID;
    rc = usp_smallest_circle(k2_host, n, bias_kind, centre, &R);
    if (rc) return rc;
    if (!(R > 0.0)) return USP_ERR_INVALID;  // homogeneous medium: bias and c must be given
    c_out[0] = 0.0;
    c_out[1] = R / vnorm;
  }
  bias_out[0] = centre[0];
  bias_out[1] = centre[1];
  cdiv(1.0, 0.0, c_out[0], c_out[1], sym_out->s);
  sym_out->a0[0] = centre[0];
  sym_out->a0[1] = centre[1];
  sym_out->a2[0] = -1.0;
  return 0;
}

// Scalar frequency-domain diffusion with constant D (Sec. 3.2 with D constant,
// e^{-i omega t}): A0 = -D laplacian + mu_a - i omega/v.  mubar = centre of the
// smallest circle of the real mu_a values (their midrange), c = R/vnorm (real).
// Symbol: l(p) = (D |p|^2 + mubar - i omega/v)/c.
extern "C" int usp_canonical_diffusion(const double* mu_host, size_t n, double D, double omega_over_v, double vnorm,
                                       const usp_symbol* grid, usp_symbol* sym_out, double* c_out,
                                       double* bias_out) {
  if (!mu_host || !c_out || !bias_out || n == 0 || !(vnorm > 0.0 && vnorm < 1.0)) return USP_ERR_INVALID;
  int rc = fill_grid(grid, sym_out);
  if (rc) return rc;
  double lo = mu_host[0], hi = mu_host[0];
  for (size_t i = 1; i < n; ++i) {
    if (!std::isfinite(mu_host[i])) return USP_ERR_NAN;
    lo = std::min(lo, mu_host[i]);
    hi = std::max(hi, mu_host[i]);
  }
  const double pts[4] = {lo, 0.0, hi, 0.0};
  double centre[2], R;
  rc = usp_smallest_circle(pts, 2, USP_BIAS_COMPLEX, centre, &R);
  if (rc) return rc;
  if (!(R > 0.0)) return USP_ERR_INVALID;
  c_out[0] = R / vnorm;
  c_out[1] = 0.0;
  bias_out[0] = centre[0];
  bias_out[1] = 0.0;
  sym_out->s[0] = 1.0 / c_out[0];
  sym_out->a0[0] = centre[0];
  sym_out->a0[1] = -omega_over_v;
  sym_out->a2[0] = D;
  return 0;
}

// Schrodinger operator shifted by Abar (Sec. 4, Eq. schrodinger; unit mass,
// natural units): H + Abar = -1/2 laplacian + V + Abar is the constant-D
// diffusion operator with D = 1/2, mu = V + Abar, omega = 0.  The smallest
// circle of the real set {V + Abar} is centred at midrange(V) + Abar with the
// radius of {V}, so c = (max V - min V)/(2 vnorm), the symbol's a0 is
// midrange(V) + Abar, and B = 1 - (V - midrange(V))/c: the field bias returned
// in bias_out is midrange(V), for usp_canonical_fields on V itself.
extern "C" int usp_canonical_schrodinger(const double* V_host, size_t n, double shift, double vnorm,
                                         const usp_symbol* grid, usp_symbol* sym_out, double* c_out,
                                         double* bias_out) {
  if (!std::isfinite(shift)) return USP_ERR_INVALID;
  const int rc = usp_canonical_diffusion(V_host, n, 0.5, 0.0, vnorm, grid, sym_out, c_out, bias_out);
  if (rc) return rc;
  sym_out->a0[0] = bias_out[0] + shift;
  return 0;
}

// Pantograph (Sec. 3.3, Eq. pantograph-A) on t_j = t0 + j h, j < n:
//   A x = c^-1 [(d/dt + a) x + b x(lam t)],  y = c^-1 [b x0(lam t) + x0(t0) delta(t - t0)].
// abar = smallest-circle centre of {a_j}; the dilation x(lam t_j) is a
// linear-interpolation gather S (entries with lam t_j < t0 belong to the
// initial condition and are zero in S; the caller's x0(lam t_j) carries them).
// c = (sup|a - abar| + sup|b| ||S||_2)/vnorm (||S||_2 by power iteration on
// S^T S), so ||V|| <= vnorm.  Outputs (host arrays of n complex = 2n doubles):
// B = 1 - (a - abar)/c, the gather weights g0 = b w0 / c, g1 = b w1 / c with
// indices idx, and y.  Symbol: s = 1/c, a0 = abar, a1 = 1, Nyquist i p = 0.
extern "C" int usp_canonical_pantograph(const double* a, const double* b, int n, double lam, double t0, double h,
                                        const double* x0_lam_t, const double* x0_t0, double vnorm,
                                        usp_symbol* sym_out, double* B_out, int32_t* idx_out, double* g0_out,
                                        double* g1_out, double* y_out, double* c_out, double* bias_out) {
  if (!a || !b || !x0_lam_t || !x0_t0 || !sym_out || !B_out || !idx_out || !g0_out || !g1_out || !y_out || !c_out ||
      !bias_out || n < 2 || !(h > 0.0) || !(lam > 0.0) || !(vnorm > 0.0 && vnorm < 1.0))
    return USP_ERR_INVALID;
  double centre[2], Ra;
  int rc = usp_smallest_circle(a, (size_t)n, USP_BIAS_COMPLEX, centre, &Ra);
  if (rc) return rc;
  // interpolation gather
  std::vector<int> idx(n, 0);
  std::vector<double> w0(n, 0.0), w1(n, 0.0);
  for (int j = 0; j < n; ++j) {
    const double pos = (lam * (t0 + h * j) - t0) / h;
    if (pos < -1e-9 || pos > (n - 1) + 1e-9) continue;
    int i0 = (int)std::floor(pos + 1e-9);
    double f = pos - i0;
    if (std::fabs(f) < 1e-9) f = 0.0;
    if (i0 >= n - 1) {
      idx[j] = n - 2;
      w1[j] = 1.0;  // exactly the last sample
      continue;
    }
    idx[j] = i0;
    w0[j] = 1.0 - f;
    w1[j] = f;
  }
  // ||S||_2 = sqrt(lambda_max(S^T S)).  Each row of S touches two adjacent
  // columns, so S^T S is symmetric tridiagonal; its largest eigenvalue is found
  // by bisection on Sturm-sequence counts (to the last bit).
  std::vector<double> dg(n, 0.0), od(n, 0.0);
  for (int j = 0; j < n; ++j) {
    const int i = idx[j];
    dg[i] += w0[j] * w0[j];
    dg[i + 1] += w1[j] * w1[j];
    od[i] += w0[j] * w1[j];
  }
  auto count_below = [&](double x) {  // eigenvalues < x
    int cnt = 0;
    double q = dg[0] - x;
    if (q < 0) ++cnt;
    for (int i = 1; i < n; ++i) {
      if (q == 0.0) q = 1e-300;
      q = dg[i] - x - od[i - 1] * od[i - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  double hi = 0.0;
  for (int i = 0; i < n; ++i) hi = std::max(hi, dg[i] + std::fabs(od[i]) + (i ? std::fabs(od[i - 1]) : 0.0));
  double lo = 0.0;
  hi *= 1.0 + 1e-12;
  for (int it = 0; it < 200 && hi - lo > 1e-16 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= n) hi = mid;  // all eigenvalues below mid
    else lo = mid;
  }
  const double snorm = std::sqrt(0.5 * (lo + hi));
  double bmax = 0.0;
  for (int j = 0; j < n; ++j) bmax = std::max(bmax, std::hypot(b[2 * j], b[2 * j + 1]));
  const double c = (Ra + bmax * snorm) / vnorm;
  if (!(c > 0.0)) return USP_ERR_INVALID;
  c_out[0] = c;
  c_out[1] = 0.0;
  bias_out[0] = centre[0];
  bias_out[1] = centre[1];
  *sym_out = usp_symbol{};
  sym_out->ndim = 1;
  sym_out->shape[0] = n;
  sym_out->spacing[0] = h;
  sym_out->s[0] = 1.0 / c;
  sym_out->a0[0] = centre[0];
  sym_out->a0[1] = centre[1];
  sym_out->a1[0] = 1.0;
  sym_out->nyquist_zero = 1;
  for (int j = 0; j < n; ++j) {
    B_out[2 * j] = 1.0 - (a[2 * j] - centre[0]) / c;
    B_out[2 * j + 1] = -(a[2 * j + 1] - centre[1]) / c;
    idx_out[j] = idx[j];
    g0_out[2 * j] = b[2 * j] * w0[j] / c;
    g0_out[2 * j + 1] = b[2 * j + 1] * w0[j] / c;
    g1_out[2 * j] = b[2 * j] * w1[j] / c;
    g1_out[2 * j + 1] = b[2 * j + 1] * w1[j] / c;
    // b x0(lam t) / c  (complex product)
    const double br = b[2 * j], bi = b[2 * j + 1], xr = x0_lam_t[2 * j], xi = x0_lam_t[2 * j + 1];
    y_out[2 * j] = (br * xr - bi * xi) / c;
    y_out[2 * j + 1] = (br * xi + bi * xr) / c;
  }
  y_out[0] += x0_t0[0] / h / c;
  y_out[1] += x0_t0[1] / h / c;
  return 0;
}

// Steady diffusion in flux form (Sec. 3.2, Eq. diffusion-equation-matrix-form)
// on a 2-D or 3-D grid: biases from smallest circles, symmetric equilibration
// of the radii, c from the largest per-voxel spectral norm of S V~ S.
namespace {
void circle_of(const std::vector<double>& pts, double* centre, double* R, int* rc) {
  const size_t n = pts.size() / 2;
  bool same = true;
  for (size_t i = 1; i < n && same; ++i) same = pts[2 * i] == pts[0] && pts[2 * i + 1] == pts[1];
  if (same) {
    centre[0] = pts[0];
    centre[1] = pts[1];
    *R = 0.0;
    *rc = 0;
    return;
  }
  *rc = usp_smallest_circle(pts.data(), n, USP_BIAS_COMPLEX, centre, R);
}

typedef std::complex<double> cd;

// largest eigenvalue of the Hermitian H = M^H M of a d x d matrix M: exact
// for d = 2; for d = 3 the trigonometric solution of the characteristic
// cubic (accurate to about sqrt(eps) where the top two are close) or, with
// exact = true, cyclic Jacobi
double top_gram_eig(int d, const cd* M, bool exact) {
  cd H[9];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      cd acc = 0.0;
      for (int k = 0; k < d; ++k) acc += std::conj(M[k * d + i]) * M[k * d + j];
      H[i * d + j] = acc;
    }
  if (d == 2) {
    const double p = H[0].real(), r = H[3].real();
    return 0.5 * (p + r) + std::sqrt(0.25 * (p - r) * (p - r) + std::norm(H[1]));
  }
  if (exact) {
    std::vector<cd> a(H, H + 9);
    std::vector<double> w;
    std::vector<cd> Z;
    usp_host::hermitian_jacobi(3, a, w, Z);
    return w[2];
  }
  const double q = (H[0].real() + H[4].real() + H[8].real()) / 3.0;
  const double p1 = std::norm(H[1]) + std::norm(H[2]) + std::norm(H[5]);
  const double d0 = H[0].real() - q, d1 = H[4].real() - q, d2 = H[8].real() - q;
  const double p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * p1;
  if (!(p2 > 0.0)) return q;
  const double pp = std::sqrt(p2 / 6.0);
  // det((H - q I) / pp) / 2, real for Hermitian H
  const cd b00 = d0 / pp, b11 = d1 / pp, b22 = d2 / pp, b01 = H[1] / pp, b02 = H[2] / pp, b12 = H[5] / pp;
  const cd det = b00 * (b11 * b22 - b12 * std::conj(b12)) - b01 * (std::conj(b01) * b22 - b12 * std::conj(b02)) +
                 b02 * (std::conj(b01) * std::conj(b12) - b11 * std::conj(b02));
  const double r = std::max(-1.0, std::min(1.0, 0.5 * det.real()));
  return q + 2.0 * pp * std::cos(std::acos(r) / 3.0);
}
}  // namespace

extern "C" int usp_canonical_flux(const double* mu, const double* D, const double* src, int ndim, const int* shape,
                                  double h, double vnorm, usp_flux_symbol* sym, double* bu_out, double* b2_out,
                                  double* y_out) {
  if (!mu || !D || !src || !shape || !sym || !bu_out || !b2_out || !y_out || (ndim != 2 && ndim != 3) ||
      !(h > 0.0) || !(vnorm > 0.0 && vnorm < 1.0))
    return USP_ERR_INVALID;
  const int d = ndim, dd = ndim * ndim;
  size_t n = 1;
  for (int a = 0; a < d; ++a) {
    if (shape[a] < 2) return USP_ERR_INVALID;
    n *= (size_t)shape[a];
  }
  for (size_t i = 0; i < 2 * n; ++i)
    if (!std::isfinite(mu[i]) || !std::isfinite(src[i])) return USP_ERR_NAN;
  for (size_t i = 0; i < 2 * dd * n; ++i)
    if (!std::isfinite(D[i])) return USP_ERR_NAN;
  // D^-1 per voxel
  std::vector<cd> Di((size_t)dd * n);
  for (size_t v = 0; v < n; ++v) {
    cd m[9];
    for (int e = 0; e < dd; ++e) m[e] = cd(D[2 * (dd * v + e)], D[2 * (dd * v + e) + 1]);
    if (!usp_host::small_inverse(d, m, &Di[(size_t)dd * v])) return USP_ERR_INVALID;
  }
  int rc = 0;
  double mub[2], Rmu;
  {
    std::vector<double> pts(mu, mu + 2 * n);
    circle_of(pts, mub, &Rmu, &rc);
    if (rc) return rc;
  }
  cd dib[9];
  double R2[9];
  for (int e = 0; e < dd; ++e) {
    std::vector<double> pts(2 * n);
    for (size_t v = 0; v < n; ++v) {
      pts[2 * v] = Di[(size_t)dd * v + e].real();
      pts[2 * v + 1] = Di[(size_t)dd * v + e].imag();
    }
    double cc[2];
    circle_of(pts, cc, &R2[e], &rc);
    if (rc) return rc;
    dib[e] = cd(cc[0], cc[1]);
  }
  // symmetric infinity-norm equilibration of the radii blockdiag(R_mu, [R_ab])
  double dV[4][4] = {{0.0}};
  dV[0][0] = Rmu;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) dV[1 + a][1 + b] = R2[a * d + b];
  double s[4] = {1.0, 1.0, 1.0, 1.0};
  for (int sweep = 0; sweep < 50; ++sweep)
    for (int i = 0; i <= d; ++i) {
      double r = 0.0;
      for (int j = 0; j <= d; ++j) r = std::max(r, s[i] * dV[i][j] * s[j]);
      if (r > 0.0) s[i] /= std::sqrt(r);
    }
  // c = max over voxels of ||S V~ S||_2 / vnorm: a fast estimate per voxel,
  // then the exact norm wherever the estimate comes near the maximum
  const cd mubar(mub[0], mub[1]);
  auto v2 = [&](size_t v, cd* M) {
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b)
        M[a * d + b] = s[1 + a] * s[1 + b] * (Di[(size_t)dd * v + a * d + b] - dib[a * d + b]);
  };
  std::vector<double> est(n);
  double emax = 0.0;
  for (size_t v = 0; v < n; ++v) {
    const double vu = s[0] * s[0] * std::abs(cd(mu[2 * v], mu[2 * v + 1]) - mubar);
    cd M[9];
    v2(v, M);
    const double nv = std::sqrt(std::max(top_gram_eig(d, M, false), 0.0));
    est[v] = std::max(vu, nv);
    emax = std::max(emax, est[v]);
  }
  double vmax = emax;
  if (d == 3) {
    vmax = 0.0;
    for (size_t v = 0; v < n; ++v) {
      if (est[v] < emax * (1.0 - 1e-6)) continue;
      const double vu = s[0] * s[0] * std::abs(cd(mu[2 * v], mu[2 * v + 1]) - mubar);
      cd M[9];
      v2(v, M);
      vmax = std::max(vmax, std::max(vu, std::sqrt(std::max(top_gram_eig(d, M, true), 0.0))));
    }
  }
  double c = vmax / vnorm;
  if (!(c > 0.0)) c = 1.0;
  *sym = usp_flux_symbol{};
  sym->ndim = d;
  for (int a = 0; a < 3; ++a) sym->n[a] = a < d ? shape[a] : 1;
  sym->h = h;
  for (int k = 0; k <= d; ++k) sym->s[k] = s[k];
  sym->c = c;
  sym->mubar[0] = mub[0];
  sym->mubar[1] = mub[1];
  for (int e = 0; e < dd; ++e) {
    sym->dibar[e][0] = dib[e].real();
    sym->dibar[e][1] = dib[e].imag();
  }
  const double rsc = 1.0 / std::sqrt(c);
  for (size_t v = 0; v < n; ++v) {
    const cd bu = 1.0 - s[0] * s[0] * (cd(mu[2 * v], mu[2 * v + 1]) - mubar) / c;
    bu_out[2 * v] = bu.real();
    bu_out[2 * v + 1] = bu.imag();
    cd M[9];
    v2(v, M);
    for (int e = 0; e < dd; ++e) {
      const cd b = ((e / d == e % d) ? 1.0 : 0.0) - M[e] / c;
      b2_out[2 * (dd * v + e)] = b.real();
      b2_out[2 * (dd * v + e) + 1] = b.imag();
    }
    y_out[2 * v] = s[0] * src[2 * v] * rsc;
    y_out[2 * v + 1] = s[0] * src[2 * v + 1] * rsc;
    for (int k = 1; k <= d; ++k) y_out[2 * (k * n + v)] = y_out[2 * (k * n + v) + 1] = 0.0;
  }
  return 0;
}
