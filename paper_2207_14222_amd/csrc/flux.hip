// C ABI of steady diffusion in flux form (Sec. 3.2, Eq.
// diffusion-equation-matrix-form): workspace layout, the fixed-point solve
// (Algorithm 1 on the 3-component system) and its FP64 residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/usp.h"
#include "flux.hpp"
#include "op.hpp"

using namespace usp;
using namespace usp_detail;

namespace {

constexpr int kFxHist = 1 << 16;   // device ring of ||Delta||^2 values
constexpr int kFxRows = 32;        // ring of per-iteration partial rows, summed in batches

struct FxLayout {
  size_t t = 0, S = 0, part = 0, hist = 0, scal = 0, tw0f = 0, tw0d = 0, tw1f = 0, tw1d = 0, total = 0;
  long pitch = 0;
};

int fx_check(const usp_flux_symbol* sym, int dtype) {
  if (!sym) return fail(USP_ERR_INVALID, "symbol is NULL");
  if (dtype != USP_C64 && dtype != USP_C128) return fail(USP_ERR_INVALID, "dtype must be USP_C64 or USP_C128");
  if (!pow2_in_range(sym->n0) || !pow2_in_range(sym->n1))
    return fail(USP_ERR_UNSUPPORTED_SHAPE, "flux grid sides must be powers of two in [8, 1024]");
  if (!(sym->h > 0.0) || !(sym->c > 0.0)) return fail(USP_ERR_INVALID, "h and c must be positive");
  return 0;
}

// blocks of the row kernel for a row length n1 (rows of n0)
int fx_row_blocks(int n0, int n1) {
  int lpb = 1;
  with_n(n1, [&](auto NC) { lpb = FxRow<decltype(NC)::value>::LPB; });
  return (n0 + lpb - 1) / lpb;
}

FxLayout fx_layout(const usp_flux_symbol* sym, int dtype) {
  FxLayout L;
  const long N = (long)sym->n0 * sym->n1;
  const size_t es = dtype == USP_C64 ? 8 : 16;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = align_up(off + b);
    return o;
  };
  L.pitch = fx_row_blocks(sym->n0, sym->n1);
  L.t = take(3 * N * es);
  L.S = take(3 * N * 16);
  L.part = take(sizeof(double) * (kFxRows + 2) * L.pitch);
  L.hist = take(sizeof(double) * kFxHist);
  L.scal = take(sizeof(double) * 64);
  L.tw0f = take(sizeof(float2) * sym->n0);
  L.tw0d = take(sizeof(double2) * sym->n0);
  L.tw1f = take(sizeof(float2) * sym->n1);
  L.tw1d = take(sizeof(double2) * sym->n1);
  L.total = off;
  return L;
}

FluxSym fx_sym(const usp_flux_symbol* s) {
  FluxSym f;
  const double ic = 1.0 / s->c;
  f.A[0] = 1.0 + s->s[0] * s->s[0] * s->mubar[0] * ic;
  f.A[1] = s->s[0] * s->s[0] * s->mubar[1] * ic;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const double w = s->s[1 + a] * s->s[1 + b] * ic;
      f.E[2 * a + b][0] = (a == b ? 1.0 : 0.0) + w * s->dibar[2 * a + b][0];
      f.E[2 * a + b][1] = w * s->dibar[2 * a + b][1];
    }
  const double(*E)[2] = f.E;
  f.dE[0] = (E[0][0] * E[3][0] - E[0][1] * E[3][1]) - (E[1][0] * E[2][0] - E[1][1] * E[2][1]);
  f.dE[1] = (E[0][0] * E[3][1] + E[0][1] * E[3][0]) - (E[1][0] * E[2][1] + E[1][1] * E[2][0]);
  f.q1 = s->s[0] * s->s[1] * ic;
  f.q2 = s->s[0] * s->s[2] * ic;
  f.pscale0 = 2.0 * M_PI / (s->n0 * s->h);
  f.pscale1 = 2.0 * M_PI / (s->n1 * s->h);
  f.n0 = s->n0;
  f.n1 = s->n1;
  return f;
}

struct FxRun {
  const usp_flux_symbol* sym;
  FluxSym fs;
  FxLayout L;
  char* ws;
  hipStream_t st;
  long N;
  template <class C> C* t() const { return (C*)(ws + L.t); }
  double2* S() const { return (double2*)(ws + L.S); }
  double* part() const { return (double*)(ws + L.part); }
  double* hist() const { return (double*)(ws + L.hist); }
  double* scal() const { return (double*)(ws + L.scal); }
  template <class C> const C* tw0() const;
  template <class C> const C* tw1() const;
};
template <> const float2* FxRun::tw0<float2>() const { return (const float2*)(ws + L.tw0f); }
template <> const double2* FxRun::tw0<double2>() const { return (const double2*)(ws + L.tw0d); }
template <> const float2* FxRun::tw1<float2>() const { return (const float2*)(ws + L.tw1f); }
template <> const double2* FxRun::tw1<double2>() const { return (const double2*)(ws + L.tw1d); }

int fx_twiddles(const FxRun& R) {
  for (int ax = 0; ax < 2; ++ax) {
    const int n = ax == 0 ? R.sym->n0 : R.sym->n1;
    std::vector<float2> tf(n);
    std::vector<double2> td(n);
    for (int k = 0; k < n; ++k) {
      const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)k / (long double)n;
      const long double c = cosl(a), s = sinl(a);
      td[k].x = (double)c;
      td[k].y = (double)s;
      tf[k].x = (float)c;
      tf[k].y = (float)s;
    }
    HIPCHK(hipMemcpyAsync(R.ws + (ax == 0 ? R.L.tw0f : R.L.tw1f), tf.data(), n * sizeof(float2),
                          hipMemcpyHostToDevice, R.st));
    HIPCHK(hipMemcpyAsync(R.ws + (ax == 0 ? R.L.tw0d : R.L.tw1d), td.data(), n * sizeof(double2),
                          hipMemcpyHostToDevice, R.st));
  }
  HIPCHK(hipStreamSynchronize(R.st));
  return 0;
}

// y-axis pass with the per-mode block: (L + I)^-1 (inv) or L, on the 3 planes of d
template <class C>
int fx_col(const FxRun& R, C* d, bool inv) {
  const bool ok = with_n(R.sym->n0, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    using G = FxCol<C, N>;
    const dim3 grid((unsigned)(R.sym->n1 / G::W));
    if (inv)
      hipLaunchKernelGGL((k_fx_col<C, N, true>), grid, dim3(G::THREADS), 0, R.st, d, R.tw0<C>(), R.fs);
    else
      hipLaunchKernelGGL((k_fx_col<C, N, false>), grid, dim3(G::THREADS), 0, R.st, d, R.tw0<C>(), R.fs);
  });
  if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "flux column pass");
  LAUNCHCHK("k_fx_col");
  return 0;
}

// x-axis pass in the given mode
template <class Cc, class Cx, int MODE>
int fx_row(const FxRun& R, Cc* spec, Cx* x, const Cx* y, const Cx* bu, const Cx* b2, double alpha, int has_x,
           double* row0, double* row1) {
  const bool ok = with_n(R.sym->n1, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    hipLaunchKernelGGL((k_fx_row<Cc, Cx, N, MODE>), dim3((unsigned)R.L.pitch), dim3(3 * FxRow<N>::G), 0, R.st,
                       spec, x, y, bu, b2, R.tw1<Cc>(), alpha, R.sym->n0, has_x, row0, row1);
  });
  if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "flux row pass");
  LAUNCHCHK("k_fx_row");
  return 0;
}

// ordered sums of `nrows` partial rows starting at ring row `first` into out
int fx_sum(const FxRun& R, int first, int nrows, int ring, double* out, int out_first, int out_ring) {
  if (nrows <= 0) return 0;
  hipLaunchKernelGGL(k_fx_sum<0>, dim3(nrows), dim3(256), 0, R.st, R.part(), R.L.pitch, (int)R.L.pitch, first, ring,
                     out, out_first, out_ring);
  LAUNCHCHK("k_fx_sum");
  return 0;
}

template <class C>
int fx_residual(const FxRun& R, const C* bu, const C* b2, const C* y, const C* x, double* rho) {
  int rc;
  double* r0 = R.part() + kFxRows * R.L.pitch;
  if ((rc = fx_row<double2, C, FX_RFWD>(R, R.S(), (C*)x, y, bu, b2, 0.0, 1, nullptr, nullptr))) return rc;
  if ((rc = fx_col<double2>(R, R.S(), false))) return rc;
  if ((rc = fx_row<double2, C, FX_RINV>(R, R.S(), (C*)x, y, bu, b2, 0.0, 1, r0, r0 + R.L.pitch))) return rc;
  if ((rc = fx_sum(R, kFxRows, 2, kFxRows + 2, R.scal(), 0, 2))) return rc;
  double h[2];
  HIPCHK(hipMemcpyAsync(h, R.scal(), 2 * sizeof(double), hipMemcpyDeviceToHost, R.st));
  HIPCHK(hipStreamSynchronize(R.st));
  *rho = std::sqrt(h[0] / h[1]);
  return 0;
}

template <class C>
int fx_solve(const FxRun& R, const C* bu, const C* b2, const C* y, C* x, int x_is_guess, double alpha, double tol,
             int maxit, int check_every, int* iters_out, double* hist_pre, int hist_pre_cap, double* hist_true,
             int hist_true_cap, int* n_true_out) {
  int rc;
  C* t = R.t<C>();
  if (!x_is_guess) HIPCHK(hipMemsetAsync(x, 0, sizeof(C) * 3 * R.N, R.st));
  if ((rc = fx_row<C, C, FX_FIRST>(R, t, x, y, bu, b2, 0.0, x_is_guess ? 1 : 0, nullptr, nullptr))) return rc;
  int it = 0, ntrue = 0, status = USP_MAXIT, pulled = 0, flushed = 0, grow = 0;
  double d0 = -1.0, dprev = -1.0;
  std::vector<double> buf;
  // sum the pending partial rows of iterations [flushed, it) into the history ring
  auto flush = [&]() -> int {
    const int m = it - flushed;
    const int e = fx_sum(R, flushed % kFxRows, m, kFxRows, R.hist(), flushed % kFxHist, kFxHist);
    flushed = it;
    return e;
  };
  auto pull = [&]() -> int {
    const int n = it - pulled;
    if (n <= 0) return 0;
    buf.resize(n);
    for (int done = 0; done < n;) {   // at most two copies around the ring
      const int s = (pulled + done) % kFxHist;
      const int m = std::min(n - done, kFxHist - s);
      HIPCHK(hipMemcpyAsync(buf.data() + done, R.hist() + s, m * sizeof(double), hipMemcpyDeviceToHost, R.st));
      done += m;
    }
    HIPCHK(hipStreamSynchronize(R.st));
    for (int i = 0; i < n; ++i) {
      const double dd = buf[i];
      if (hist_pre && pulled + i < hist_pre_cap) hist_pre[pulled + i] = dd;
      if (!(dd == dd)) status = USP_ERR_NAN;
      if (d0 < 0.0) d0 = dd;
      grow = (dprev >= 0.0 && dd > dprev) ? grow + 1 : 0;
      dprev = dd;
      if (grow >= 3 && dd > d0 && status != USP_ERR_NAN) status = USP_DIVERGED;
    }
    pulled = it;
    return 0;
  };
  while (it < maxit) {
    if ((rc = fx_col<C>(R, t, true))) return rc;
    if ((rc = fx_row<C, C, FX_FUSED>(R, t, x, y, bu, b2, alpha, 1, R.part() + (it % kFxRows) * R.L.pitch,
                                     nullptr)))
      return rc;
    ++it;
    if (it - flushed == kFxRows && (rc = flush())) return rc;
    const bool chk = it % check_every == 0 || it == maxit;
    if (chk || it - pulled >= kFxHist / 2) {
      if ((rc = flush()) || (rc = pull())) return rc;
      if (status == USP_ERR_NAN || status == USP_DIVERGED) break;
    }
    if (chk) {
      double rho;
      if ((rc = fx_residual<C>(R, bu, b2, y, x, &rho))) return rc;
      if (hist_true && ntrue < hist_true_cap) {
        hist_true[2 * ntrue] = it;
        hist_true[2 * ntrue + 1] = rho;
      }
      ++ntrue;
      if (!(rho == rho)) { status = USP_ERR_NAN; break; }
      if (rho < tol) { status = USP_OK; break; }
    }
  }
  if ((rc = flush()) || (rc = pull())) return rc;
  if (iters_out) *iters_out = it;
  if (n_true_out) *n_true_out = ntrue;
  if (status < 0) return fail(status, "non-finite values in the iteration");
  return status;
}

int fx_begin(const usp_flux_symbol* sym, int dtype, void* ws, size_t ws_bytes, void* stream, FxRun* R) {
  int rc = fx_check(sym, dtype);
  if (rc) return rc;
  R->sym = sym;
  R->fs = fx_sym(sym);
  R->L = fx_layout(sym, dtype);
  if (!ws || ws_bytes < R->L.total)
    return fail(USP_ERR_WORKSPACE, "flux workspace too small: need " + std::to_string(R->L.total) + " bytes");
  if (((uintptr_t)ws) & 255) return fail(USP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  R->ws = (char*)ws;
  R->st = (hipStream_t)stream;
  R->N = (long)sym->n0 * sym->n1;
  return fx_twiddles(*R);
}

}  // namespace

extern "C" {

int usp_flux_workspace_bytes(const usp_flux_symbol* sym, int dtype, size_t* bytes) {
  int rc = fx_check(sym, dtype);
  if (rc) return rc;
  if (!bytes) return fail(USP_ERR_INVALID, "bytes is NULL");
  *bytes = fx_layout(sym, dtype).total;
  return 0;
}

int usp_flux_solve(const usp_flux_symbol* sym, int dtype, const void* bu_dev, const void* b2_dev, const void* y_dev,
                   void* x_dev, int x_is_guess, double alpha, double tol, int maxit, int check_every, void* ws_dev,
                   size_t ws_bytes, void* stream, int* iters_out, double* hist_pre, int hist_pre_cap,
                   double* hist_true, int hist_true_cap, int* n_true_out) {
  if (!bu_dev || !b2_dev || !y_dev || !x_dev) return fail(USP_ERR_INVALID, "NULL argument");
  if (!(alpha > 0.0) || maxit < 0 || check_every < 1) return fail(USP_ERR_INVALID, "alpha > 0, maxit >= 0, check_every >= 1");
  FxRun R;
  int rc = fx_begin(sym, dtype, ws_dev, ws_bytes, stream, &R);
  if (rc) return rc;
  if (dtype == USP_C64)
    return fx_solve<float2>(R, (const float2*)bu_dev, (const float2*)b2_dev, (const float2*)y_dev, (float2*)x_dev,
                            x_is_guess, alpha, tol, maxit, check_every, iters_out, hist_pre, hist_pre_cap, hist_true,
                            hist_true_cap, n_true_out);
  return fx_solve<double2>(R, (const double2*)bu_dev, (const double2*)b2_dev, (const double2*)y_dev, (double2*)x_dev,
                           x_is_guess, alpha, tol, maxit, check_every, iters_out, hist_pre, hist_pre_cap, hist_true,
                           hist_true_cap, n_true_out);
}

int usp_flux_residual(const usp_flux_symbol* sym, int dtype, const void* bu_dev, const void* b2_dev,
                      const void* y_dev, const void* x_dev, void* ws_dev, size_t ws_bytes, void* stream,
                      double* rel_out) {
  if (!bu_dev || !b2_dev || !y_dev || !x_dev || !rel_out) return fail(USP_ERR_INVALID, "NULL argument");
  FxRun R;
  int rc = fx_begin(sym, dtype, ws_dev, ws_bytes, stream, &R);
  if (rc) return rc;
  if (dtype == USP_C64)
    return fx_residual<float2>(R, (const float2*)bu_dev, (const float2*)b2_dev, (const float2*)y_dev,
                               (const float2*)x_dev, rel_out);
  return fx_residual<double2>(R, (const double2*)bu_dev, (const double2*)b2_dev, (const double2*)y_dev,
                              (const double2*)x_dev, rel_out);
}

}  // extern "C"
