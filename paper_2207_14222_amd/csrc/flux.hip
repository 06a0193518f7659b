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

constexpr int kFxHist = 1 << 16;
constexpr int kFxBlocks = 2048;

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
  L.pitch = std::min<long>((N + 255) / 256, kFxBlocks);
  L.t = take(3 * N * es);
  L.S = take(3 * N * 16);
  L.part = take(sizeof(double) * 3 * L.pitch);
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
  for (int k = 0; k < 3; ++k) f.s[k] = s->s[k];
  f.c = s->c;
  f.mubar[0] = s->mubar[0];
  f.mubar[1] = s->mubar[1];
  for (int k = 0; k < 4; ++k) {
    f.dibar[k][0] = s->dibar[k][0];
    f.dibar[k][1] = s->dibar[k][1];
  }
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
  int vb;
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

// forward (DIR -1) or inverse (+1) 2-D FFT of the 3 component planes of `d`
template <class C, int DIR>
int fx_fft2(const FxRun& R, C* d) {
  const int n0 = R.sym->n0, n1 = R.sym->n1;
  const int nlines = 3 * n0;
  bool ok = true;
  auto xpass = [&]() {
    ok = with_n(n1, [&](auto NC) {
      constexpr int N = decltype(NC)::value;
      constexpr int TPB = x_threads<C>();
      constexpr int LPB = TPB / (N / PassPlan<N>::E);
      hipLaunchKernelGGL((k_xfft<C, N, DIR>), dim3((nlines + LPB - 1) / LPB), dim3(TPB), 0, R.st, d, R.tw1<C>(),
                         nlines);
    });
  };
  auto ypass = [&]() {
    bool launched = false;
    ok = with_n(n0, [&](auto NC) {
      constexpr int N = decltype(NC)::value;
      constexpr int E = PassPlan<N>::E;
      auto go = [&](auto WC) {
        constexpr int W = decltype(WC)::value;
        if constexpr (s_width_ok<C>(N, W, E)) {
          if (launched || n1 % W) return;
          hipLaunchKernelGGL((k_spass<C, N, W, DIR < 0 ? S_FWD : S_INV>), dim3(n1 / W, 3), dim3(W * (N / E)), 0, R.st,
                             d, R.tw0<C>(), (long)n1, SymArgs{});
          launched = true;
        }
      };
      go(std::integral_constant<int, 16>{});
      go(std::integral_constant<int, 8>{});
      go(std::integral_constant<int, 4>{});
    });
    ok = ok && launched;
  };
  if (DIR < 0) {
    xpass();
    if (ok) ypass();
  } else {
    ypass();
    if (ok) xpass();
  }
  if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "flux grid FFT plan");
  LAUNCHCHK("flux fft");
  return 0;
}

template <class C>
int fx_residual(const FxRun& R, const C* bu, const C* b2, const C* y, const C* x, double* rho) {
  int rc;
  hipLaunchKernelGGL(k_fx_widen<C>, dim3(R.vb), dim3(256), 0, R.st, x, R.S(), 3 * R.N);
  if ((rc = fx_fft2<double2, -1>(R, R.S()))) return rc;
  hipLaunchKernelGGL(k_fx_sym<double2>, dim3(R.vb), dim3(256), 0, R.st, R.S(), R.fs, 0);
  if ((rc = fx_fft2<double2, +1>(R, R.S()))) return rc;
  hipLaunchKernelGGL(k_fx_res<C>, dim3(R.vb), dim3(256), 0, R.st, (const double2*)R.S(), x, y, bu, b2, R.N,
                     R.part() + R.L.pitch, R.part() + 2 * R.L.pitch);
  hipLaunchKernelGGL(k_fx_sum<0>, dim3(2), dim3(256), 0, R.st, R.part() + R.L.pitch, R.L.pitch, R.vb, R.scal());
  LAUNCHCHK("flux residual");
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
  hipLaunchKernelGGL(k_fx_first<C>, dim3(R.vb), dim3(256), 0, R.st, (const C*)x, y, bu, b2, t, R.N, x_is_guess ? 1 : 0);
  LAUNCHCHK("k_fx_first");
  int it = 0, ntrue = 0, status = USP_MAXIT, pulled = 0, grow = 0;
  double d0 = -1.0, dprev = -1.0;
  std::vector<double> buf;
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
    if ((rc = fx_fft2<C, -1>(R, t))) return rc;
    hipLaunchKernelGGL(k_fx_sym<C>, dim3(R.vb), dim3(256), 0, R.st, t, R.fs, 1);
    if ((rc = fx_fft2<C, +1>(R, t))) return rc;
    hipLaunchKernelGGL(k_fx_update<C>, dim3(R.vb), dim3(256), 0, R.st, t, x, y, bu, b2, alpha, R.N, R.part());
    hipLaunchKernelGGL(k_fx_sum<0>, dim3(1), dim3(256), 0, R.st, R.part(), R.L.pitch, R.vb, R.hist() + it % kFxHist);
    LAUNCHCHK("flux iteration");
    ++it;
    const bool chk = it % check_every == 0 || it == maxit;
    if (chk || it - pulled >= kFxHist / 2) {
      if ((rc = pull())) return rc;
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
  if ((rc = pull())) return rc;
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
  R->vb = (int)R->L.pitch;
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
