// C ABI of steady diffusion in flux form (Sec. 3.2, Eq.
// diffusion-equation-matrix-form) on 2-D and 3-D grids: workspace layout, the
// fixed-point solve (Algorithm 1 on the [u; J] system) and its FP64 residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "../../include/usp.h"
#include "flux.hpp"
#include "hermitian.hpp"
#include "op.hpp"

using namespace usp;
using namespace usp_detail;

namespace {

constexpr int kFxHist = 1 << 16;   // device ring of ||Delta||^2 values
constexpr int kFxRows = 32;        // ring of per-iteration partial rows, summed in batches

struct FxLayout {
  size_t t = 0, S = 0, part = 0, hist = 0, scal = 0, twf[3] = {0, 0, 0}, twd[3] = {0, 0, 0}, total = 0;
  // refined solve: complex64 copies of b_u and b2, the residual and the correction
  size_t bu32 = 0, b232 = 0, r32 = 0, d32 = 0;
  long pitch = 0;
};

int fx_check(const usp_flux_symbol* sym, int dtype) {
  if (!sym) return fail(USP_ERR_INVALID, "symbol is NULL");
  if (dtype != USP_C64 && dtype != USP_C128) return fail(USP_ERR_INVALID, "dtype must be USP_C64 or USP_C128");
  if (sym->ndim != 2 && sym->ndim != 3) return fail(USP_ERR_INVALID, "ndim must be 2 or 3");
  for (int a = 0; a < sym->ndim; ++a)
    if (!pow2_in_range(sym->n[a]))
      return fail(USP_ERR_UNSUPPORTED_SHAPE, "flux grid sides must be powers of two in [8, 1024]");
  if (!(sym->h > 0.0) || !(sym->c > 0.0)) return fail(USP_ERR_INVALID, "h and c must be positive");
  return 0;
}

long fx_voxels(const usp_flux_symbol* sym) {
  long n = 1;
  for (int a = 0; a < sym->ndim; ++a) n *= sym->n[a];
  return n;
}

// grid rows along the contiguous axis, and blocks of the row kernel
long fx_nrows(const usp_flux_symbol* sym) { return fx_voxels(sym) / sym->n[sym->ndim - 1]; }
int fx_row_blocks(const usp_flux_symbol* sym) {
  int lpb = 1;
  with_n(sym->n[sym->ndim - 1], [&](auto NC) { lpb = FxRow<decltype(NC)::value>::LPB; });
  return (int)((fx_nrows(sym) + lpb - 1) / lpb);
}

// refined: complex64 spectrum for the inner iterations plus the refinement
// arrays (dtype is then USP_C64 for the layout of t)
FxLayout fx_layout(const usp_flux_symbol* sym, int dtype, bool refined = false) {
  FxLayout L;
  const long N = fx_voxels(sym);
  const int np = sym->ndim + 1;
  const size_t es = dtype == USP_C64 ? 8 : 16;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off = align_up(off + b);
    return o;
  };
  L.pitch = fx_row_blocks(sym);
  L.t = take(np * N * es);
  L.S = take(np * N * 16);
  L.part = take(sizeof(double) * (kFxRows + 2) * L.pitch);
  L.hist = take(sizeof(double) * kFxHist);
  L.scal = take(sizeof(double) * 64);
  for (int a = 0; a < sym->ndim; ++a) {
    L.twf[a] = take(sizeof(float2) * sym->n[a]);
    L.twd[a] = take(sizeof(double2) * sym->n[a]);
  }
  if (refined) {
    L.bu32 = take(sizeof(float2) * N);
    L.b232 = take(sizeof(float2) * sym->ndim * sym->ndim * N);
    L.r32 = take(sizeof(float2) * np * N);
    L.d32 = take(sizeof(float2) * np * N);
  }
  L.total = off;
  return L;
}

int fx_sym(const usp_flux_symbol* s, FluxSym* f) {
  const int d = s->ndim;
  *f = FluxSym{};
  const double ic = 1.0 / s->c;
  f->A[0] = 1.0 + s->s[0] * s->s[0] * s->mubar[0] * ic;
  f->A[1] = s->s[0] * s->s[0] * s->mubar[1] * ic;
  std::complex<double> E[9], Ei[9];
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      const double w = s->s[1 + a] * s->s[1 + b] * ic;
      E[a * d + b] = std::complex<double>((a == b ? 1.0 : 0.0) + w * s->dibar[a * d + b][0],
                                          w * s->dibar[a * d + b][1]);
    }
  if (!usp_host::small_inverse(d, E, Ei)) return fail(USP_ERR_INVALID, "I + S' Dibar S' / c is singular");
  for (int e = 0; e < d * d; ++e) {
    f->E[e][0] = E[e].real();
    f->E[e][1] = E[e].imag();
    f->Einv[e][0] = Ei[e].real();
    f->Einv[e][1] = Ei[e].imag();
  }
  for (int k = 0; k < d; ++k) f->q[k] = s->s[0] * s->s[1 + k] * ic;
  for (int a = 0; a < 3; ++a) {
    f->n[a] = a < d ? s->n[a] : 1;
    f->pscale[a] = a < d ? 2.0 * M_PI / (s->n[a] * s->h) : 0.0;
  }
  return 0;
}

struct FxRun {
  const usp_flux_symbol* sym;
  FluxSym fs;
  FxLayout L;
  char* ws;
  hipStream_t st;
  long N;        // voxels
  long nrows;    // grid rows along the contiguous axis
  int d;
  template <class C> C* t() const { return (C*)(ws + L.t); }
  double2* S() const { return (double2*)(ws + L.S); }
  double* part() const { return (double*)(ws + L.part); }
  double* hist() const { return (double*)(ws + L.hist); }
  double* scal() const { return (double*)(ws + L.scal); }
  template <class C> const C* tw(int a) const;
  float2* f32(size_t off) const { return (float2*)(ws + off); }
};
template <> const float2* FxRun::tw<float2>(int a) const { return (const float2*)(ws + L.twf[a]); }
template <> const double2* FxRun::tw<double2>(int a) const { return (const double2*)(ws + L.twd[a]); }

int fx_twiddles(const FxRun& R) {
  for (int ax = 0; ax < R.d; ++ax) {
    const int n = R.sym->n[ax];
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
    HIPCHK(hipMemcpyAsync(R.ws + R.L.twf[ax], tf.data(), n * sizeof(float2), hipMemcpyHostToDevice, R.st));
    HIPCHK(hipMemcpyAsync(R.ws + R.L.twd[ax], td.data(), n * sizeof(double2), hipMemcpyHostToDevice, R.st));
  }
  HIPCHK(hipStreamSynchronize(R.st));
  return 0;
}

// axis-0 pass with the per-mode block: (L + I)^-1 (inv) or L, on the planes of
// data, in tiles of 2 columns (1 where the planes' tiles exceed LDS).
// Measured: 2 columns beat 4, 8 and 16 both at 256 x 256 (more blocks in
// flight) and at 128^3 (wider tiles, up to 128-byte segments in 1024-thread
// blocks, ran the pass up to 1.4x slower).
template <class C>
int fx_col(const FxRun& R, C* data, bool inv) {
  const long ncols = R.N / R.sym->n[0];
  bool launched = false;
  auto go = [&](auto DC) {
    constexpr int D = decltype(DC)::value;
    return with_n(R.sym->n[0], [&](auto NC) {
      constexpr int N = decltype(NC)::value;
      auto try_w = [&](auto WC) {
        constexpr int W = decltype(WC)::value;
        if constexpr (FxCol<C, N, D + 1, W>::VALID) {
          using G = FxCol<C, N, D + 1, W>;
          if (launched || ncols % W) return;
          const dim3 grid((unsigned)(ncols / W));
          if (inv)
            hipLaunchKernelGGL((k_fx_col<C, N, D, W, true>), grid, dim3(G::THREADS), 0, R.st, data, R.tw<C>(0), R.fs);
          else
            hipLaunchKernelGGL((k_fx_col<C, N, D, W, false>), grid, dim3(G::THREADS), 0, R.st, data, R.tw<C>(0),
                               R.fs);
          launched = true;
        }
      };
      try_w(std::integral_constant<int, 2>{});
      try_w(std::integral_constant<int, 1>{});
    });
  };
  const bool ok = R.d == 2 ? go(std::integral_constant<int, 2>{}) : go(std::integral_constant<int, 3>{});
  if (!ok || !launched) return fail(USP_ERR_UNSUPPORTED_SHAPE, "flux column pass");
  LAUNCHCHK("k_fx_col");
  return 0;
}

// 3-D: FFT (DIR -1) or inverse FFT (+1) along axis 1 of every plane (batch of
// planes x n0 slabs, column tiles along the contiguous axis)
template <class C, int DIR>
int fx_mid(const FxRun& R, C* data) {
  const int n1 = R.sym->n[1], n2 = R.sym->n[2];
  const int batch = (R.d + 1) * R.sym->n[0];
  bool launched = false;
  const bool ok = with_n(n1, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    constexpr int E = PassPlan<N>::E;
    auto go = [&](auto WC) {
      constexpr int W = decltype(WC)::value;
      if constexpr (s_width_ok<C>(N, W, E)) {
        if (launched || n2 % W) return;
        hipLaunchKernelGGL((k_spass<C, N, W, DIR < 0 ? S_FWD : S_INV>), dim3(n2 / W, batch), dim3(W * (N / E)), 0,
                           R.st, data, R.tw<C>(1), (long)n2, SymArgs{});
        launched = true;
      }
    };
    go(std::integral_constant<int, sizeof(C) == 8 ? 16 : 8>{});
    go(std::integral_constant<int, 8>{});
    go(std::integral_constant<int, 4>{});
  });
  if (!ok || !launched) return fail(USP_ERR_UNSUPPORTED_SHAPE, "flux middle-axis pass");
  LAUNCHCHK("k_spass");
  return 0;
}

// (L + I)^-1 (inv) or L between the contiguous-axis passes
template <class C>
int fx_symbol(const FxRun& R, C* data, bool inv) {
  int rc;
  if (R.d == 3 && (rc = fx_mid<C, -1>(R, data))) return rc;
  if ((rc = fx_col<C>(R, data, inv))) return rc;
  if (R.d == 3 && (rc = fx_mid<C, +1>(R, data))) return rc;
  return 0;
}

// contiguous-axis pass in the given mode
template <class Cc, class Cx, int MODE>
int fx_row(const FxRun& R, Cc* spec, Cx* x, const Cx* y, const Cx* bu, const Cx* b2, double alpha, int has_x,
           double* row0, double* row1, const float2* dcor = nullptr, float2* r32 = nullptr) {
  auto go = [&](auto DC) {
    constexpr int D = decltype(DC)::value;
    return with_n(R.sym->n[R.d - 1], [&](auto NC) {
      constexpr int N = decltype(NC)::value;
      hipLaunchKernelGGL((k_fx_row<Cc, Cx, N, D, MODE>), dim3((unsigned)R.L.pitch), dim3((D + 1) * FxRow<N>::G), 0,
                         R.st, spec, x, y, bu, b2, R.tw<Cc>(R.d - 1), alpha, R.nrows, has_x, row0, row1, dcor, r32);
    });
  };
  const bool ok = R.d == 2 ? go(std::integral_constant<int, 2>{}) : go(std::integral_constant<int, 3>{});
  if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "flux row pass");
  LAUNCHCHK("k_fx_row");
  return 0;
}

// ordered sums of `nrows` partial rows starting at ring row `first` into out
// (FP32 partials of complex64 iterations if f32)
int fx_sum(const FxRun& R, int first, int nrows, int ring, double* out, int out_first, int out_ring,
           bool f32 = false) {
  if (nrows <= 0) return 0;
  if (f32)
    hipLaunchKernelGGL(k_fx_sum<float>, dim3(nrows), dim3(256), 0, R.st, reinterpret_cast<const float*>(R.part()),
                       2 * R.L.pitch, (int)R.L.pitch, first, ring, out, out_first, out_ring);
  else
    hipLaunchKernelGGL(k_fx_sum<double>, dim3(nrows), dim3(256), 0, R.st, R.part(), R.L.pitch, (int)R.L.pitch, first,
                       ring, out, out_first, out_ring);
  LAUNCHCHK("k_fx_sum");
  return 0;
}

// rho = ||y - A x|| / ||y|| in FP64.  Refined solve: dcor (complex64) is
// first added to x in place, and r is also stored as complex64 in r32.
template <class C>
int fx_residual(const FxRun& R, const C* bu, const C* b2, const C* y, const C* x, double* rho,
                const float2* dcor = nullptr, float2* r32 = nullptr) {
  int rc;
  double* r0 = R.part() + kFxRows * R.L.pitch;
  if ((rc = fx_row<double2, C, FX_RFWD>(R, R.S(), (C*)x, y, bu, b2, 0.0, 1, nullptr, nullptr, dcor))) return rc;
  if ((rc = fx_symbol<double2>(R, R.S(), false))) return rc;
  if ((rc = fx_row<double2, C, FX_RINV>(R, R.S(), (C*)x, y, bu, b2, 0.0, 1, r0, r0 + R.L.pitch, nullptr, r32)))
    return rc;
  if ((rc = fx_sum(R, kFxRows, 2, kFxRows + 2, R.scal(), 0, 2))) return rc;
  double h[2];
  HIPCHK(hipMemcpyAsync(h, R.scal(), 2 * sizeof(double), hipMemcpyDeviceToHost, R.st));
  HIPCHK(hipStreamSynchronize(R.st));
  *rho = std::sqrt(h[0] / h[1]);
  return 0;
}

// ||Delta||^2 history: per-iteration partial rows in a ring of kFxRows, summed
// in batches into the device ring `hist`, pulled to the host at checks
struct FxHist {
  const FxRun& R;
  double* hist_pre;
  int hist_pre_cap;
  bool f32;          // the rows hold complex64 iterations' FP32 partials
  int it = 0, pulled = 0, flushed = 0, grow = 0, status = USP_MAXIT;
  double d0 = -1.0, dprev = -1.0;
  double tail[16];   // latest values (ring), for the refined solve's rate
  int ntail = 0;
  std::vector<double> buf;
  double* row() const { return R.part() + (it % kFxRows) * R.L.pitch; }
  // one iteration's partial row was written at row(): advance
  int step() {
    ++it;
    return it - flushed == kFxRows ? flush() : 0;
  }
  // sum the pending partial rows of iterations [flushed, it) into the history ring
  int flush() {
    const int m = it - flushed;
    const int e = fx_sum(R, flushed % kFxRows, m, kFxRows, R.hist(), flushed % kFxHist, kFxHist, f32);
    flushed = it;
    return e;
  }
  int pull() {
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
      tail[ntail++ % 16] = dd;
    }
    pulled = it;
    return 0;
  }
  int sync() {
    int rc;
    if ((rc = flush()) || (rc = pull())) return rc;
    return 0;
  }
};

template <class C>
int fx_solve(const FxRun& R, const C* bu, const C* b2, const C* y, C* x, int x_is_guess, double alpha, double tol,
             int maxit, int check_every, int* iters_out, double* hist_pre, int hist_pre_cap, double* hist_true,
             int hist_true_cap, int* n_true_out) {
  int rc;
  C* t = R.t<C>();
  if (!x_is_guess) HIPCHK(hipMemsetAsync(x, 0, sizeof(C) * (R.d + 1) * R.N, R.st));
  if ((rc = fx_row<C, C, FX_FIRST>(R, t, x, y, bu, b2, 0.0, x_is_guess ? 1 : 0, nullptr, nullptr))) return rc;
  FxHist H{R, hist_pre, hist_pre_cap, sizeof(C) == 8};
  int ntrue = 0;
  while (H.it < maxit) {
    if ((rc = fx_symbol<C>(R, t, true))) return rc;
    if ((rc = fx_row<C, C, FX_FUSED>(R, t, x, y, bu, b2, alpha, 1, H.row(), nullptr))) return rc;
    if ((rc = H.step())) return rc;
    const int it = H.it;
    const bool chk = it % check_every == 0 || it == maxit;
    if (chk || it - H.pulled >= kFxHist / 2) {
      if ((rc = H.sync())) return rc;
      if (H.status == USP_ERR_NAN || H.status == USP_DIVERGED) break;
    }
    if (chk) {
      double rho;
      if ((rc = fx_residual<C>(R, bu, b2, y, x, &rho))) return rc;
      if (hist_true && ntrue < hist_true_cap) {
        hist_true[2 * ntrue] = it;
        hist_true[2 * ntrue + 1] = rho;
      }
      ++ntrue;
      if (!(rho == rho)) { H.status = USP_ERR_NAN; break; }
      if (rho < tol) { H.status = USP_OK; break; }
    }
  }
  if ((rc = H.sync())) return rc;
  if (iters_out) *iters_out = H.it;
  if (n_true_out) *n_true_out = ntrue;
  if (H.status < 0) return fail(H.status, "non-finite values in the iteration");
  return H.status;
}

// Refined solve (complex128 x): FP64 residual r = y - A x every cycle, then up
// to k complex64 iterations of Algorithm 1 on A d = r from d = 0, added to x by
// the next residual's first pass.  As in the main path, the final cycle is cut
// to the count that the latest rate of ||Delta|| predicts for reaching tol
// when that is under half a cycle.
int fx_solve_refined(const FxRun& R, const double2* bu, const double2* b2, const double2* y, double2* x,
                     int x_is_guess, double alpha, double tol, int maxit, int k, int* iters_out, double* hist_pre,
                     int hist_pre_cap, double* hist_true, int hist_true_cap, int* n_true_out) {
  int rc;
  const long nb2 = (long)R.d * R.d * R.N;
  float2 *bu32 = R.f32(R.L.bu32), *b232 = R.f32(R.L.b232), *r32 = R.f32(R.L.r32), *d32 = R.f32(R.L.d32);
  float2* t = R.t<float2>();
  hipLaunchKernelGGL(k_fx_to32<0>, dim3(1024), dim3(256), 0, R.st, bu, bu32, R.N);
  hipLaunchKernelGGL(k_fx_to32<0>, dim3(1024), dim3(256), 0, R.st, b2, b232, nb2);
  LAUNCHCHK("k_fx_to32");
  if (!x_is_guess) HIPCHK(hipMemsetAsync(x, 0, sizeof(double2) * (R.d + 1) * R.N, R.st));
  FxHist H{R, hist_pre, hist_pre_cap, true};
  int ntrue = 0;
  bool judge = x_is_guess == 2;
  const float2* dcor = nullptr;
  std::vector<double> rhos;
  while (true) {
    double rho;
    if ((rc = fx_residual<double2>(R, bu, b2, y, x, &rho, dcor, r32))) return rc;
    dcor = nullptr;
    if ((rc = H.sync())) return rc;
    if (hist_true && ntrue < hist_true_cap) {
      hist_true[2 * ntrue] = H.it;
      hist_true[2 * ntrue + 1] = rho;
    }
    ++ntrue;
    if (judge) {
      // a guess whose residual is not below ||y|| is discarded: restart from x = 0
      judge = false;
      if (!(rho < 1.0)) {
        HIPCHK(hipMemsetAsync(x, 0, sizeof(double2) * (R.d + 1) * R.N, R.st));
        continue;
      }
    }
    if (!(rho == rho) || H.status == USP_ERR_NAN) { H.status = USP_ERR_NAN; break; }
    if (rho < tol) { H.status = USP_OK; break; }
    if (H.status == USP_DIVERGED) break;
    // no 1% improvement of the FP64 residual over 8 checks
    rhos.push_back(rho);
    if (rhos.size() > 8 && rho > 0.99 * rhos[rhos.size() - 9]) { H.status = USP_STAGNATED; break; }
    if (H.it >= maxit) break;
    int m = std::min(k, maxit - H.it);
    if (H.ntail >= 11) {
      const double a = H.tail[(H.ntail - 1) % 16], b = H.tail[(H.ntail - 11) % 16];
      if (a > 0.0 && a < b) {
        const double lrate = 0.05 * std::log(a / b);   // log of the per-iteration factor of ||Delta||
        const double need = std::log(tol / rho) / lrate;
        if (need < 0.5 * m) m = std::max(1, (int)std::ceil(1.05 * need) + 1);
      }
    }
    HIPCHK(hipMemsetAsync(d32, 0, sizeof(float2) * (R.d + 1) * R.N, R.st));
    if ((rc = fx_row<float2, float2, FX_FIRST>(R, t, d32, r32, bu32, b232, 0.0, 0, nullptr, nullptr))) return rc;
    for (int j = 0; j < m; ++j) {
      if ((rc = fx_symbol<float2>(R, t, true))) return rc;
      if ((rc = fx_row<float2, float2, FX_FUSED>(R, t, d32, r32, bu32, b232, alpha, 1, H.row(), nullptr))) return rc;
      if ((rc = H.step())) return rc;
    }
    dcor = d32;
  }
  HIPCHK(hipStreamSynchronize(R.st));
  if (iters_out) *iters_out = H.it;
  if (n_true_out) *n_true_out = ntrue;
  if (H.status < 0) return fail(H.status, "non-finite values in the iteration");
  return H.status;
}

int fx_begin(const usp_flux_symbol* sym, int dtype, void* ws, size_t ws_bytes, void* stream, FxRun* R,
             bool refined = false) {
  int rc = fx_check(sym, dtype);
  if (rc) return rc;
  R->sym = sym;
  R->d = sym->ndim;
  if ((rc = fx_sym(sym, &R->fs))) return rc;
  R->L = refined ? fx_layout(sym, USP_C64, true) : fx_layout(sym, dtype);
  if (!ws || ws_bytes < R->L.total)
    return fail(USP_ERR_WORKSPACE, "flux workspace too small: need " + std::to_string(R->L.total) + " bytes");
  if (((uintptr_t)ws) & 255) return fail(USP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  R->ws = (char*)ws;
  R->st = (hipStream_t)stream;
  R->N = fx_voxels(sym);
  R->nrows = fx_nrows(sym);
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

int usp_flux_refined_workspace_bytes(const usp_flux_symbol* sym, size_t* bytes) {
  int rc = fx_check(sym, USP_C128);
  if (rc) return rc;
  if (!bytes) return fail(USP_ERR_INVALID, "bytes is NULL");
  *bytes = fx_layout(sym, USP_C64, true).total;
  return 0;
}

int usp_flux_solve_refined(const usp_flux_symbol* sym, const void* bu_dev, const void* b2_dev, const void* y_dev,
                           void* x_dev, int x_is_guess, double alpha, double tol, int maxit, int refine_every,
                           void* ws_dev, size_t ws_bytes, void* stream, int* iters_out, double* hist_pre,
                           int hist_pre_cap, double* hist_true, int hist_true_cap, int* n_true_out) {
  if (!bu_dev || !b2_dev || !y_dev || !x_dev) return fail(USP_ERR_INVALID, "NULL argument");
  if (!(alpha > 0.0) || maxit < 0 || refine_every < 1)
    return fail(USP_ERR_INVALID, "alpha > 0, maxit >= 0, refine_every >= 1");
  FxRun R;
  int rc = fx_begin(sym, USP_C128, ws_dev, ws_bytes, stream, &R, true);
  if (rc) return rc;
  return fx_solve_refined(R, (const double2*)bu_dev, (const double2*)b2_dev, (const double2*)y_dev,
                          (double2*)x_dev, x_is_guess, alpha, tol, maxit, refine_every, iters_out, hist_pre,
                          hist_pre_cap, hist_true, hist_true_cap, n_true_out);
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
