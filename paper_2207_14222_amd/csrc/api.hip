// C ABI of the solver: operator handles, workspace layout, pass scheduling,
// the fixed-point solve loop (Algorithm 1, Sec. 2.1), FP64 residual checks and
// outer refinement, and host canonicalisation helpers (Sec. 2.2, 3.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/usp.h"
#include "hermitian.hpp"
#include "krylov.hpp"
#include "op.hpp"
#include "passes.hpp"
#include "solve1d.hpp"
#include "util.hpp"

using namespace usp;

namespace usp_detail {
thread_local std::string g_err;
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
}  // namespace usp_detail

namespace {

void prof_mark(usp_op op) {
  if (!op->prof) return;
  hipEvent_t e;
  if (hipEventCreate(&e) == hipSuccess) {
    hipEventRecord(e, op->st);
    op->prof[op->kind].push_back(e);
  }
}

template <class C> C* tw_for(usp_op op, int n);
template <> float2* tw_for<float2>(usp_op op, int n) { return op->twf[ilog2(n)]; }
template <> double2* tw_for<double2>(usp_op op, int n) { return op->twd[ilog2(n)]; }

RedArgs red_row(usp_op op, int row) {
  RedArgs r;
  r.row = row < 0 ? nullptr : op->partials + (long)row * op->pitch;
  return r;
}

template <class Cc> int x_blocks(usp_op op) {
  int nb = 0;
  with_n(op->d.n2, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    constexpr int LPB = x_threads<Cc>() / (N / PassPlan<N>::E);
    nb = (op->d.n0 * op->d.n1 + LPB - 1) / LPB;
  });
  return nb;
}

// add up `nrows` partial rows starting at `row` (ncols partials each, FP32 if
// f32 else FP64) into out[(first + r) % nmod]
int sum_rows(usp_op op, int row, int nrows, int ncols, double* out, int first, int nmod, bool f32 = false) {
  if (nrows <= 0) return 0;
  prof_mark(op);
  if (f32)
    hipLaunchKernelGGL(k_sum_rows<float>, dim3(nrows), dim3(256), 0, op->st,
                       reinterpret_cast<const float*>(op->partials + (long)row * op->pitch), 2 * op->pitch, ncols,
                       out, first, nmod);
  else
    hipLaunchKernelGGL(k_sum_rows<double>, dim3(nrows), dim3(256), 0, op->st, op->partials + (long)row * op->pitch,
                       op->pitch, ncols, out, first, nmod);
  prof_mark(op);
  LAUNCHCHK("k_sum_rows");
  return 0;
}

// move pending per-iteration ||Delta||^2 partial rows into the history ring
int finalize_hist(usp_op op) {
  const int kind = op->kind;
  op->kind = USP_PASS_REDUCE;
  int rc = sum_rows(op, 0, op->pending, op->xblocks, op->hist, op->pending_first, kHist, op->pending_f32);
  op->kind = kind;
  op->pending_first += op->pending;
  op->pending = 0;
  return rc;
}

// ---- pass launchers --------------------------------------------------------
template <class Cc, class Cx, int MODE>
int launch_x(usp_op op, Cc* t, Cx* x, const Cx* y, const Cx* B, const float2* d, float2* r32, double alpha,
             int has_x, RedArgs red) {
  const Dims& D = op->d;
  const int nlines = D.n0 * D.n1;
  const int fl = (MODE == X_FUSED) ? ((op->plan.x_prefetch ? 1 : 0) | (op->plan.x_stream ? 2 : 0))
                 : (MODE == X_RINV) ? (op->plan.r_load & 3) : 0;
  bool ok = with_n(D.n2, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    constexpr int E = PassPlan<N>::E, T = N / E;
    constexpr int TPB = x_threads<Cc>();
    constexpr int LPB = TPB / T;
    const int blocks = (nlines + LPB - 1) / LPB;
    if (MODE == X_FUSED) op->xblocks = blocks;
    prof_mark(op);
    auto go = [&](auto FC) {
      constexpr int F = decltype(FC)::value;
      hipLaunchKernelGGL((k_xpass<Cc, Cx, N, MODE, F>), dim3(blocks), dim3(TPB), 0, op->st, t, x, y, B, d, r32,
                         tw_for<Cc>(op, N), alpha, nlines, has_x, red);
    };
    switch (fl) {
      case 1: go(std::integral_constant<int, 1>{}); break;
      case 2: go(std::integral_constant<int, 2>{}); break;
      case 3: go(std::integral_constant<int, 3>{}); break;
      default: go(std::integral_constant<int, 0>{}); break;
    }
    prof_mark(op);
  });
  if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "contiguous axis length");
  LAUNCHCHK("k_xpass");
  return 0;
}

template <class C> int default_w(int N) {
  if (sizeof(C) == 8) return N >= 1024 ? 8 : 16;
  return N >= 1024 ? 4 : 8;
}

template <class C> bool width_ok(int N, int W) {
  bool ok = false;
  with_n(N, [&](auto NC) {
    constexpr int Nn = decltype(NC)::value;
    ok = s_width_ok<C>(Nn, W, PassPlan<Nn>::E);
  });
  return ok && (W == 4 || W == 8 || W == 16 || W == 32);
}

// strided pass along axis 0 (ax = 0) or axis 1 (ax = 1, 3-D only) with column
// tiles of W elements (W <= the axis stride S; the largest valid width <= W is used)
template <class C, int MODE>
int launch_s(usp_op op, C* data, int ax, const SymArgs& sym, int W) {
  const Dims& D = op->d;
  const int n = ax == 0 ? D.n0 : D.n1;
  const long S = ax == 0 ? (long)D.n1 * D.n2 : (long)D.n2;
  const int batch = ax == 0 ? 1 : D.n0;
  if (W <= 0) W = default_w<C>(n);
  while (W > 4 && (W > S || !width_ok<C>(n, W))) W >>= 1;
  bool launched = false;
  bool ok = with_n(n, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    constexpr int E = PassPlan<N>::E, T = N / E;
    auto go = [&](auto WC) {
      constexpr int Wc = decltype(WC)::value;
      if constexpr (s_width_ok<C>(N, Wc, E)) {
        prof_mark(op);
        hipLaunchKernelGGL((k_spass<C, N, Wc, MODE>), dim3((unsigned)(S / Wc), batch), dim3(Wc * T), 0, op->st,
                           data, tw_for<C>(op, N), S, sym);
        prof_mark(op);
        launched = true;
      }
    };
    switch (W) {
      case 4: go(std::integral_constant<int, 4>{}); break;
      case 8: go(std::integral_constant<int, 8>{}); break;
      case 16: go(std::integral_constant<int, 16>{}); break;
      case 32: go(std::integral_constant<int, 32>{}); break;
      default: break;
    }
  });
  if (!ok || !launched) return fail(USP_ERR_UNSUPPORTED_SHAPE, "strided axis length / tile width");
  LAUNCHCHK("k_spass");
  return 0;
}

SymArgs sym_args(usp_op op, bool plus_one) {
  SymArgs a;
  const Dims& D = op->d;
  auto sc = [](int n, double h) { return n > 1 ? std::pow(2.0 * M_PI / (n * h), 2) : 0.0; };
  a.sa = sc(D.n0, op->sym.spacing[0]);
  a.sm = D.ndim == 3 ? sc(D.n1, op->sym.spacing[1]) : 0.0;
  a.sx = sc(D.n2, op->sym.spacing[D.ndim - 1]);
  a.n1 = D.n1;
  a.log2_n2 = ilog2(D.n2);
  a.c0r = op->sa0[0] + (plus_one ? 1.0 : 0.0);
  a.c0i = op->sa0[1];
  a.c2r = op->sa2[0];
  a.c2i = op->sa2[1];
  a.scale = 1.0 / (double)op->d.N;
  return a;
}

// Forward FFT (axis n2) of the first t = B x + y.
template <class C>
int first_pass(usp_op op, C* x, const C* y, const C* B, int has_x) {
  op->kind = 4;
  return launch_x<C, C, X_FIRST>(op, (C*)op->t, x, y, B, nullptr, nullptr, 0.0, has_x, red_row(op, -1));
}

// Middle passes of one iteration plus the fused update/first pass of the next.
template <class C>
int iteration(usp_op op, C* x, const C* y, const C* B, double alpha) {
  C* t = (C*)op->t;
  const SymArgs sa = sym_args(op, true);
  int rc;
  op->kind = 1;
  const int wm = sizeof(C) == 8 ? op->plan.w_mid : 0, ws = sizeof(C) == 8 ? op->plan.w_sym : 0;
  if (op->d.ndim == 3 && (rc = launch_s<C, S_FWD>(op, t, 1, sa, wm))) return rc;
  op->kind = 2;
  if ((rc = launch_s<C, S_SYM>(op, t, 0, sa, ws))) return rc;
  op->kind = 3;
  if (op->d.ndim == 3 && (rc = launch_s<C, S_INV>(op, t, 1, sa, wm))) return rc;
  op->kind = 0;
  if ((rc = launch_x<C, C, X_FUSED>(op, t, x, y, B, nullptr, nullptr, alpha, 1, red_row(op, op->pending)))) return rc;
  // a solve finalises the pending rows before it switches precision
  op->pending_f32 = sizeof(C) == 8;
  if (++op->pending == kRows) return finalize_hist(op);
  return 0;
}

// FP64 true residual of x (storage Cx); ||r||^2 -> scal[0].  d: correction added
// into x first (refinement), r32: complex64 copy of r (refinement).
template <class Cx>
int residual_passes(usp_op op, Cx* x, const Cx* y, const Cx* B, const float2* d, float2* r32) {
  double2* S = op->S;
  const SymArgs sa = sym_args(op, false);
  int rc;
  op->kind = 5;
  if ((rc = launch_x<double2, Cx, X_RFWD>(op, S, x, y, B, d, nullptr, 0.0, 0, red_row(op, -1)))) return rc;
  op->kind = 6;
  if (op->d.ndim == 3 && (rc = launch_s<double2, S_FWD>(op, S, 1, sa, 0))) return rc;
  op->kind = 7;
  if ((rc = launch_s<double2, S_SYMA>(op, S, 0, sa, 0))) return rc;
  op->kind = 8;
  if (op->d.ndim == 3 && (rc = launch_s<double2, S_INV>(op, S, 1, sa, 0))) return rc;
  op->kind = 9;
  if ((rc = launch_x<double2, Cx, X_RINV>(op, S, x, y, B, nullptr, r32, 0.0, 0, red_row(op, kRows)))) return rc;
  op->kind = USP_PASS_REDUCE;
  return sum_rows(op, kRows, 1, x_blocks<double2>(op), op->scal, 0, 1);
}

template <class C>
int norm2(usp_op op, const C* z, double* out) {
  const long n = op->d.N;
  int blocks = (int)std::min<long>((n + 255) / 256, 2048);
  hipLaunchKernelGGL((k_norm2<C>), dim3(blocks), dim3(256), 0, op->st, z, n, op->partials + (long)(kRows + 1) * op->pitch);
  LAUNCHCHK("k_norm2");
  return sum_rows(op, kRows + 1, 1, blocks, out, 0, 1);
}

Sym1D sym1d(usp_op op) {
  Sym1D s;
  s.c0r = op->sa0[0]; s.c0i = op->sa0[1];
  s.c1r = op->sa1[0]; s.c1i = op->sa1[1];
  s.c2r = op->sa2[0]; s.c2i = op->sa2[1];
  s.pscale = 2.0 * M_PI / (op->d.n2 * op->sym.spacing[0]);
  s.nyq_zero = op->sym.nyquist_zero;
  return s;
}

// ---- host-side bookkeeping of a solve ---------------------------------------
struct Monitor {
  double* hist_pre;
  int hist_pre_cap;
  double* hist_true;
  int hist_true_cap;
  int n_true = 0;
  double best = INFINITY;
  int since_best = 0;
  double d_first = -1.0, d_prev = -1.0;
  int grow = 0;
  bool diverged = false, nan = false;
  double tail[16];   // the latest ||Delta||^2 values (ring)
  int ntail = 0;

  void delta(int it, double dd) {
    if (hist_pre && it < hist_pre_cap) hist_pre[it] = dd;
    tail[ntail % 16] = dd;
    ++ntail;
    if (!(dd == dd)) nan = true;
    if (d_first < 0) d_first = dd;
    grow = (d_prev >= 0 && dd > d_prev) ? grow + 1 : 0;
    d_prev = dd;
    if (grow >= 3 && dd > d_first) diverged = true;
  }
  // returns true if stagnated
  bool check(int it, double rho) {
    if (hist_true && n_true < hist_true_cap) {
      hist_true[2 * n_true] = it;
      hist_true[2 * n_true + 1] = rho;
    }
    ++n_true;
    if (!(rho == rho)) nan = true;
    if (rho < 0.99 * best) {
      best = rho;
      since_best = 0;
    } else {
      ++since_best;
    }
    return since_best >= 8;
  }
};

// copy ring entries [from, to) of ||Delta||^2 to the monitor
int pull_hist(usp_op op, int from, int to, Monitor& mon, std::vector<double>& buf) {
  if (to <= from) return 0;
  const int n = to - from;
  buf.resize(n);
  int done = 0;
  while (done < n) {
    const int s = (from + done) % kHist;
    const int cnt = std::min(n - done, kHist - s);
    HIPCHK(hipMemcpyAsync(buf.data() + done, op->hist + s, cnt * sizeof(double), hipMemcpyDeviceToHost, op->st));
    done += cnt;
  }
  HIPCHK(hipStreamSynchronize(op->st));
  for (int i = 0; i < n; ++i) mon.delta(from + i, buf[i]);
  return 0;
}

template <class C>
int solve_plain(usp_op op, const C* y, C* x, int x_is_guess, double alpha, double tol, int maxit, int check_every,
                int* iters_out, Monitor& mon, bool check_residual) {
  int rc;
  const C* B = (const C*)op->B;
  if ((rc = norm2(op, y, op->scal + 1))) return rc;
  op->pending = op->pending_first = 0;
  if (!x_is_guess) HIPCHK(hipMemsetAsync(x, 0, sizeof(C) * op->d.N, op->st));
  if (x_is_guess == 2 && check_residual) {
    // a guess whose residual is not below ||y|| is discarded: start from x = 0
    if ((rc = residual_passes<C>(op, x, y, B, nullptr, nullptr))) return rc;
    double h0[2];
    HIPCHK(hipMemcpyAsync(h0, op->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, op->st));
    HIPCHK(hipStreamSynchronize(op->st));
    const double rho0 = std::sqrt(h0[0] / h0[1]);
    mon.check(0, rho0);
    if (rho0 < tol) {  // the guess already solves the system
      if (iters_out) *iters_out = 0;
      return USP_OK;
    }
    if (!(rho0 < 1.0)) {
      HIPCHK(hipMemsetAsync(x, 0, sizeof(C) * op->d.N, op->st));
      x_is_guess = 0;
    }
  }
  if ((rc = first_pass<C>(op, x, y, B, x_is_guess ? 1 : 0))) return rc;
  std::vector<double> buf;
  int it = 0, pulled = 0, status = USP_MAXIT;
  double host[2];
  while (it < maxit) {
    if ((rc = iteration<C>(op, x, y, B, alpha))) return rc;
    ++it;
    const bool chk = check_residual && (it % check_every == 0 || it == maxit);
    if (chk) {
      if ((rc = finalize_hist(op))) return rc;
      if ((rc = residual_passes<C>(op, x, y, B, nullptr, nullptr))) return rc;
      HIPCHK(hipMemcpyAsync(host, op->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, op->st));
      if ((rc = pull_hist(op, pulled, it, mon, buf))) return rc;
      pulled = it;
      const double rho = std::sqrt(host[0] / host[1]);
      const bool stag = mon.check(it, rho);
      if (mon.nan) { status = USP_ERR_NAN; break; }
      if (rho < tol) { status = USP_OK; break; }
      if (mon.diverged) { status = USP_DIVERGED; break; }
      if (stag) { status = USP_STAGNATED; break; }
    } else if (it - pulled >= kHist / 2) {
      if ((rc = finalize_hist(op))) return rc;
      if ((rc = pull_hist(op, pulled, it, mon, buf))) return rc;
      pulled = it;
    }
  }
  if ((rc = finalize_hist(op))) return rc;
  if ((rc = pull_hist(op, pulled, it, mon, buf))) return rc;
  HIPCHK(hipStreamSynchronize(op->st));
  if (iters_out) *iters_out = it;
  if (status == USP_MAXIT && mon.nan) status = USP_ERR_NAN;
  if (status < 0) return fail(status, "non-finite values in the iteration");
  return status;
}

int solve_refined(usp_op op, const double2* y, double2* x, int x_is_guess, double alpha, double tol, int maxit,
                  int k, int* iters_out, Monitor& mon) {
  int rc;
  const double2* B = (const double2*)op->B;
  if ((rc = norm2(op, y, op->scal + 1))) return rc;
  op->pending = op->pending_first = 0;
  if (!x_is_guess) HIPCHK(hipMemsetAsync(x, 0, sizeof(double2) * op->d.N, op->st));
  std::vector<double> buf;
  int it = 0, pulled = 0, status = USP_MAXIT;
  double host[2];
  const float2* d = nullptr;
  bool judge_guess = x_is_guess == 2;
  while (true) {
    // r = y - A (x + d) in FP64; x <- x + d; r32 = complex64(r)
    if ((rc = finalize_hist(op))) return rc;
    if (!d && !x_is_guess) {
      // x = 0: the residual is y itself (relative residual 1) and needs no passes
      hipLaunchKernelGGL(k_to_c64, dim3(1024), dim3(256), 0, op->st, y, op->r32, op->d.N);
      LAUNCHCHK("k_to_c64");
      HIPCHK(hipMemcpyAsync(op->scal, op->scal + 1, sizeof(double), hipMemcpyDeviceToDevice, op->st));
    } else if ((rc = residual_passes<double2>(op, x, y, B, d, op->r32))) {
      return rc;
    }
    HIPCHK(hipMemcpyAsync(host, op->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, op->st));
    if ((rc = pull_hist(op, pulled, it, mon, buf))) return rc;
    pulled = it;
    const double rho = std::sqrt(host[0] / host[1]);
    if (judge_guess) {
      // a guess whose residual is not below ||y|| is discarded: restart from x = 0
      judge_guess = false;
      if (!(rho < 1.0)) {
        mon.check(it, rho);
        HIPCHK(hipMemsetAsync(x, 0, sizeof(double2) * op->d.N, op->st));
        x_is_guess = 0;
        continue;
      }
    }
    const bool stag = mon.check(it, rho);
    if (mon.nan) { status = USP_ERR_NAN; break; }
    if (rho < tol) { status = USP_OK; break; }
    if (mon.diverged) { status = USP_DIVERGED; break; }
    if (stag) { status = USP_STAGNATED; break; }
    if (it >= maxit) break;
    // inner complex64 iterations on A d = r from d = 0: k of them, or fewer when
    // the current convergence rate predicts the crossing of tol sooner (the
    // iteration keeps no state besides x, so x + d_m is the m-th iterate from x
    // and the residual keeps decaying at the rate of ||Delta||)
    int m = std::min(k, maxit - it);
    if (mon.ntail >= 11) {
      // current rate per iteration from the last 10 ||Delta|| values (it
      // slows as the slowest modes take over, so the latest is the best guide)
      const double a = mon.tail[(mon.ntail - 1) % 16], b = mon.tail[(mon.ntail - 11) % 16];
      if (a > 0.0 && a < b) {
        const double lrate = 0.05 * std::log(a / b);   // log of the per-iteration factor of ||Delta||
        const double need = std::log(tol / rho) / lrate;
        // trusted only within half a cycle: further out the slowing rate makes
        // it stop short, and a short cycle costs a whole FP64 check
        if (need < 0.5 * m) m = std::max(1, (int)std::ceil(1.05 * need) + 1);
      }
    }
    HIPCHK(hipMemsetAsync(op->d32, 0, sizeof(float2) * op->d.N, op->st));
    if ((rc = first_pass<float2>(op, op->d32, op->r32, op->B32, 0))) return rc;
    for (int j = 0; j < m; ++j)
      if ((rc = iteration<float2>(op, op->d32, op->r32, op->B32, alpha))) return rc;
    it += m;
    d = op->d32;
  }
  HIPCHK(hipStreamSynchronize(op->st));
  if (iters_out) *iters_out = it;
  if (status < 0) return fail(status, "non-finite values in the iteration");
  return status;
}

template <class C>
int solve_1d(usp_op op, const C* y, C* x, int x_is_guess, double alpha, double tol, int maxit, int check_every,
             int* iters_out, Monitor& mon) {
  const int n = op->d.n2;
  const int* gi = op->has_gather ? op->g.idx_dev : nullptr;
  const C* g0 = op->has_gather ? (const C*)op->g.g0_dev : nullptr;
  const C* g1 = op->has_gather ? (const C*)op->g.g1_dev : nullptr;
  const Sym1D s = sym1d(op);
  bool ok = with_n(n, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    constexpr int T = N / LinePlan<N>::E;
    if (op->antisym)
      hipLaunchKernelGGL((k_solve1d_as<C, N>), dim3(1), dim3(T), 0, op->st, x, y, (const C*)op->B, gi, g0, g1,
                         (const int*)(gi ? op->adj_j : nullptr), (const C*)op->adj_w, tw_for<C>(op, N), s, alpha, tol,
                         maxit, check_every, x_is_guess, op->hist, op->hist_true, kHist, op->info, (double*)nullptr);
    else
      hipLaunchKernelGGL((k_solve1d<C, N>), dim3(1), dim3(T), 0, op->st, x, y, (const C*)op->B, gi, g0, g1,
                         tw_for<C>(op, N), s, alpha, tol, maxit, check_every, x_is_guess, op->hist, op->hist_true,
                         kHist, op->info);
  });
  if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "1-D length");
  LAUNCHCHK("k_solve1d");
  Solve1DInfo info;
  HIPCHK(hipMemcpyAsync(&info, op->info, sizeof(info), hipMemcpyDeviceToHost, op->st));
  HIPCHK(hipStreamSynchronize(op->st));
  const int nh = std::min(info.iterations, kHist);
  std::vector<double> hp(nh);
  if (nh) HIPCHK(hipMemcpy(hp.data(), op->hist, nh * sizeof(double), hipMemcpyDeviceToHost));
  for (int i = 0; i < nh; ++i)
    if (mon.hist_pre && i < mon.hist_pre_cap) mon.hist_pre[i] = hp[i];
  const int nt = std::min(info.n_true, kHist);
  std::vector<double> ht(2 * nt);
  if (nt) HIPCHK(hipMemcpy(ht.data(), op->hist_true, 2 * nt * sizeof(double), hipMemcpyDeviceToHost));
  for (int i = 0; i < nt && mon.hist_true && i < mon.hist_true_cap; ++i) {
    mon.hist_true[2 * i] = ht[2 * i];
    mon.hist_true[2 * i + 1] = ht[2 * i + 1];
  }
  mon.n_true = info.n_true;
  if (iters_out) *iters_out = info.iterations;
  if (info.status == -5) return fail(USP_ERR_NAN, "non-finite values in the iteration");
  return info.status;
}

template <class C>
int residual_1d(usp_op op, const C* y, const C* x, double* out2) {
  const int n = op->d.n2;
  const int* gi = op->has_gather ? op->g.idx_dev : nullptr;
  const C* g0 = op->has_gather ? (const C*)op->g.g0_dev : nullptr;
  const C* g1 = op->has_gather ? (const C*)op->g.g1_dev : nullptr;
  const Sym1D s = sym1d(op);
  bool ok = with_n(n, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    constexpr int T = N / LinePlan<N>::E;
    if (op->antisym)
      hipLaunchKernelGGL((k_solve1d_as<C, N>), dim3(1), dim3(T), 0, op->st, (C*)x, y, (const C*)op->B, gi, g0, g1,
                         (const int*)(gi ? op->adj_j : nullptr), (const C*)op->adj_w, tw_for<C>(op, N), s, 0.0, 0.0,
                         0, 1, 1, op->hist, op->hist_true, kHist, op->info, op->scal);
    else
      hipLaunchKernelGGL((k_residual1d<C, N>), dim3(1), dim3(T), 0, op->st, x, y, (const C*)op->B, gi, g0, g1,
                         op->twd[ilog2(N)], s, op->scal);
  });
  if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "1-D length");
  LAUNCHCHK("k_residual1d");
  HIPCHK(hipMemcpyAsync(out2, op->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, op->st));
  HIPCHK(hipStreamSynchronize(op->st));
  return 0;
}

// ---- Krylov drivers on P x = b (P v = B [v - (L + I)^-1 B v], b = B (L + I)^-1 y)

constexpr int kMaxRestart = 64;
constexpr int kVecBlocks = 2048;
constexpr int kMdotKE = 16;
constexpr int kKsDoubles = 1024;

struct KWork {
  long N = 0;
  long pitch = 0;
  int nvec = 0, nrows = 0;
  size_t vec_bytes = 0;
  char* base = nullptr;
  double* rows = nullptr;
  double* ks = nullptr;
  size_t total = 0;
  template <class C> C* vec(int i) const { return (C*)(base + (size_t)i * vec_bytes); }
};

int krylov_layout(usp_op op, int method, int restart, KWork* kw) {
  if (op->d.ndim < 2 || op->has_gather) return fail(USP_ERR_UNSUPPORTED_SHAPE, "Krylov drivers need a 2-D or 3-D grid");
  if (op->refine) return fail(USP_ERR_INVALID, "Krylov drivers need a plain (not refined) handle");
  if (method != USP_KRYLOV_BICGSTAB && method != USP_KRYLOV_GMRES && method != USP_KRYLOV_CG)
    return fail(USP_ERR_INVALID, "unknown method");
  if (method == USP_KRYLOV_GMRES && (restart < 1 || restart > kMaxRestart))
    return fail(USP_ERR_INVALID, "restart must be in [1, 64]");
  const size_t es = op->dtype == USP_C64 ? 8 : 16;
  const long N = op->d.N;
  const long xb = op->dtype == USP_C64 ? x_blocks<float2>(op) : x_blocks<double2>(op);
  const long mb = (N + 256L * kMdotKE - 1) / (256L * kMdotKE);
  kw->N = N;
  kw->pitch = std::max<long>(std::max<long>(xb, mb), kVecBlocks);
  kw->nvec = method == USP_KRYLOV_BICGSTAB ? 6 : method == USP_KRYLOV_CG ? 4 : restart + 3;
  kw->nrows = method == USP_KRYLOV_GMRES ? std::max(5, 2 * (restart + 1)) : 6;
  kw->vec_bytes = align_up(N * es);
  kw->total = kw->vec_bytes * kw->nvec + align_up(sizeof(double) * kw->nrows * kw->pitch) + sizeof(double) * kKsDoubles;
  return 0;
}

int krylov_bind(KWork* kw, void* ws, size_t ws_bytes) {
  if (!ws || ws_bytes < kw->total)
    return fail(USP_ERR_WORKSPACE, "Krylov workspace too small: need " + std::to_string(kw->total) + " bytes");
  if (((uintptr_t)ws) & 255) return fail(USP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  kw->base = (char*)ws;
  kw->rows = (double*)(kw->base + kw->vec_bytes * kw->nvec);
  kw->ks = (double*)((char*)kw->rows + align_up(sizeof(double) * kw->nrows * kw->pitch));
  return 0;
}

int vec_blocks(long n) { return (int)std::min<long>((n + 255) / 256, kVecBlocks); }

// add rows [row0, row0 + nrows) of `ncols` partials each into out[0 .. nrows)
int ksum(usp_op op, const KWork& kw, int row0, int nrows, int ncols, double* out) {
  hipLaunchKernelGGL(k_sum_rows<double>, dim3(nrows), dim3(256), 0, op->st, kw.rows + (long)row0 * kw.pitch, kw.pitch,
                     ncols, out, 0, 1 << 30);
  LAUNCHCHK("k_sum_rows");
  return 0;
}

// the strided passes of P v and its last pass: t (already transformed along
// n2) -> w = B (v - u) or w = B u (rhs), with fused dot partials
template <class C>
int kapply_tail(usp_op op, const C* v, C* w, bool rhs, const C* q, int dots, const KWork& kw) {
  const Dims& D = op->d;
  const int nlines = D.n0 * D.n1;
  C* t = (C*)op->t;
  const C* B = (const C*)op->B;
  int rc;
  const SymArgs sa = sym_args(op, true);
  const int wm = sizeof(C) == 8 ? op->plan.w_mid : 0, wsy = sizeof(C) == 8 ? op->plan.w_sym : 0;
  if (D.ndim == 3 && (rc = launch_s<C, S_FWD>(op, t, 1, sa, wm))) return rc;
  if ((rc = launch_s<C, S_SYM>(op, t, 0, sa, wsy))) return rc;
  if (D.ndim == 3 && (rc = launch_s<C, S_INV>(op, t, 1, sa, wm))) return rc;
  with_n(D.n2, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    constexpr int TPB = x_threads<C>();
    constexpr int LPB = TPB / (N / PassPlan<N>::E);
    const int blocks = (nlines + LPB - 1) / LPB;
    if (rhs)
      hipLaunchKernelGGL((k_klast<C, N, true>), dim3(blocks), dim3(TPB), 0, op->st, t, (const C*)nullptr, B, w, q,
                         tw_for<C>(op, N), nlines, kw.rows, kw.pitch, dots);
    else
      hipLaunchKernelGGL((k_klast<C, N, false>), dim3(blocks), dim3(TPB), 0, op->st, t, v, B, w, q, tw_for<C>(op, N),
                         nlines, kw.rows, kw.pitch, dots);
  });
  LAUNCHCHK("k_klast");
  return 0;
}

// w = P v (rhs = false) or w = b from v = y (rhs = true), with fused dot partials
template <class C>
int kapply(usp_op op, const C* v, C* w, bool rhs, const C* q, int dots, const KWork& kw) {
  const Dims& D = op->d;
  const int nlines = D.n0 * D.n1;
  C* t = (C*)op->t;
  const C* B = (const C*)op->B;
  bool ok = with_n(D.n2, [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    constexpr int TPB = x_threads<C>();
    constexpr int LPB = TPB / (N / PassPlan<N>::E);
    const int blocks = (nlines + LPB - 1) / LPB;
    hipLaunchKernelGGL((k_kfirst<C, N>), dim3(blocks), dim3(TPB), 0, op->st, t, v, rhs ? nullptr : B, tw_for<C>(op, N),
                       nlines);
  });
  if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "contiguous axis length");
  LAUNCHCHK("k_kfirst");
  return kapply_tail<C>(op, v, w, rhs, q, dots, kw);
}

// true residual ||y - A x||^2 / ||y||^2 (FP64 passes) -> host
template <class C>
int krylov_check(usp_op op, const C* y, C* x, double* rho) {
  int rc;
  if ((rc = residual_passes<C>(op, x, y, (const C*)op->B, nullptr, nullptr))) return rc;
  double host[2];
  HIPCHK(hipMemcpyAsync(host, op->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, op->st));
  HIPCHK(hipStreamSynchronize(op->st));
  *rho = std::sqrt(host[0] / host[1]);
  return 0;
}

template <class C>
int solve_bicgstab(usp_op op, const C* y, C* x, int x_is_guess, double tol, int maxit, int check_every,
                   const KWork& kw, int* iters_out, Monitor& mon) {
  const long n = op->d.N;
  C *r = kw.vec<C>(0), *rh = kw.vec<C>(1), *p = kw.vec<C>(2), *v = kw.vec<C>(3), *s = kw.vec<C>(4),
    *t2 = kw.vec<C>(5);
  double* ks = kw.ks;
  const int vb = vec_blocks(n);
  const int xb = x_blocks<C>(op);
  int rc;
  if ((rc = norm2(op, y, op->scal + 1))) return rc;
  HIPCHK(hipMemsetAsync(ks, 0, sizeof(double) * kKsDoubles, op->st));
  if ((rc = kapply<C>(op, y, s, true, nullptr, 0, kw))) return rc;   // s = b
  if (x_is_guess) {
    if ((rc = kapply<C>(op, x, t2, false, nullptr, 0, kw))) return rc;
  } else {
    HIPCHK(hipMemsetAsync(x, 0, sizeof(C) * n, op->st));
    HIPCHK(hipMemsetAsync(t2, 0, sizeof(C) * n, op->st));
  }
  hipLaunchKernelGGL(k_ksub<C>, dim3(vb), dim3(256), 0, op->st, r, s, t2, n, kw.rows);   // r = b - P x
  LAUNCHCHK("k_ksub");
  if ((rc = ksum(op, kw, 0, 1, vb, ks + KS_RHON))) return rc;   // <r^, r> = |r|^2 with r^ = r
  HIPCHK(hipMemcpyAsync(rh, r, sizeof(C) * n, hipMemcpyDeviceToDevice, op->st));
  HIPCHK(hipMemsetAsync(p, 0, sizeof(C) * n, op->st));
  HIPCHK(hipMemsetAsync(v, 0, sizeof(C) * n, op->st));
  hipLaunchKernelGGL(k_kscal, dim3(1), dim3(64), 0, op->st, ks, (int)KSM_INIT);
  int it = 0, status = USP_MAXIT;
  while (it < maxit) {
    hipLaunchKernelGGL(k_kscal, dim3(1), dim3(64), 0, op->st, ks, (int)KSM_BETA);
    hipLaunchKernelGGL(k_bicg_p<C>, dim3(vb), dim3(256), 0, op->st, p, r, v, ks, n);
    if ((rc = kapply<C>(op, p, v, false, rh, 1, kw))) return rc;          // v = P p, <r^, v>
    if ((rc = ksum(op, kw, 0, 2, xb, ks + KS_RV))) return rc;
    hipLaunchKernelGGL(k_kscal, dim3(1), dim3(64), 0, op->st, ks, (int)KSM_ALPHA);
    hipLaunchKernelGGL(k_bicg_s<C>, dim3(vb), dim3(256), 0, op->st, s, r, v, x, p, ks, n);
    if ((rc = kapply<C>(op, s, t2, false, nullptr, 6, kw))) return rc;    // t = P s, <t, s>, |t|^2
    if ((rc = ksum(op, kw, 2, 3, xb, ks + KS_TS))) return rc;
    hipLaunchKernelGGL(k_kscal, dim3(1), dim3(64), 0, op->st, ks, (int)KSM_OMEGA);
    hipLaunchKernelGGL(k_bicg_r<C>, dim3(vb), dim3(256), 0, op->st, x, s, t2, r, rh, ks, n, kw.rows, kw.pitch);
    if ((rc = ksum(op, kw, 0, 2, vb, ks + KS_RHON))) return rc;
    if ((rc = ksum(op, kw, 2, 1, vb, ks + KS_RR))) return rc;
    LAUNCHCHK("bicgstab iteration");
    ++it;
    if (it % check_every == 0 || it == maxit) {
      double rho, hk[2];
      if ((rc = krylov_check<C>(op, y, x, &rho))) return rc;
      HIPCHK(hipMemcpyAsync(hk, ks + KS_RR, 2 * sizeof(double), hipMemcpyDeviceToHost, op->st));
      HIPCHK(hipStreamSynchronize(op->st));
      mon.delta(it - 1, hk[0]);
      const bool stag = mon.check(it, rho);
      if (mon.nan) { status = USP_ERR_NAN; break; }
      if (rho < tol) { status = USP_OK; break; }
      if (hk[1] > 0.0 || stag) { status = USP_STAGNATED; break; }   // breakdown or no progress
    }
  }
  if (iters_out) *iters_out = it;
  if (status < 0) return fail(status, "non-finite values in the iteration");
  return status;
}

// Conjugate gradients on P x = b for a Hermitian canonical operator (A, L, V
// Hermitian; P is then Hermitian, and positive definite when A is), in the
// Chronopoulos-Gear arrangement: the two inner products of an iteration
// (|r|^2 and r^H P r) come from the same pass and s = P p is carried by a
// recurrence, so the vector update joins the first pass of the next operator
// application.  An iteration is three launches: k_cgcg_first (alpha, beta
// from the summed partials, p, s, x, r and the FFT along n2 of B r), the
// strided passes, and k_klast (w = P r with the <w, r> and |r|^2 partials).
// Every block sums the partial rows it needs in the same fixed order, so no
// scalar kernel or host round trip sits between them.  The host synchronises
// at true-residual checks only.
// first_check > 0: the first check at that iteration, then every check_every
// (a caller that knows roughly how many iterations a solve takes checks
// around the end only); 0: every check_every from the start.
template <class C>
int solve_cg(usp_op op, const C* y, C* x, int x_is_guess, double tol, int maxit, int check_every, const KWork& kw,
             int* iters_out, Monitor& mon, int first_check = 0) {
  if (first_check <= 0) first_check = check_every;
  const long n = op->d.N;
  const Dims& D = op->d;
  const int nlines = D.n0 * D.n1;
  C *r = kw.vec<C>(0), *p = kw.vec<C>(1), *s = kw.vec<C>(2), *w = kw.vec<C>(3);
  double* ks = kw.ks;
  const int vb = vec_blocks(n);
  const int xb = x_blocks<C>(op);   // blocks of the last pass = width of its partial rows
  int rc;
  if ((rc = norm2(op, y, op->scal + 1))) return rc;
  HIPCHK(hipMemsetAsync(ks, 0, sizeof(double) * 32, op->st));
  if ((rc = kapply<C>(op, y, r, true, nullptr, 0, kw))) return rc;   // r = b
  if (x_is_guess) {
    if ((rc = kapply<C>(op, x, w, false, nullptr, 0, kw))) return rc;
    hipLaunchKernelGGL(k_ksub<C>, dim3(vb), dim3(256), 0, op->st, p, (const C*)r, (const C*)w, n, kw.rows);
    LAUNCHCHK("k_ksub");                                              // p = b - P x
    HIPCHK(hipMemcpyAsync(r, p, sizeof(C) * n, hipMemcpyDeviceToDevice, op->st));
  } else {
    HIPCHK(hipMemsetAsync(x, 0, sizeof(C) * n, op->st));
  }
  HIPCHK(hipMemsetAsync(p, 0, sizeof(C) * n, op->st));
  HIPCHK(hipMemsetAsync(s, 0, sizeof(C) * n, op->st));
  // w_0 = P r_0 with <w, r> (rows 2, 3) and |r|^2 (row 5)
  if ((rc = kapply<C>(op, r, w, false, nullptr, 2 | 8, kw))) return rc;
  int it = 0, status = USP_MAXIT;
  while (it < maxit) {
    bool ok = with_n(D.n2, [&](auto NC) {
      constexpr int N = decltype(NC)::value;
      constexpr int TPB = x_threads<C>();
      constexpr int LPB = TPB / (N / PassPlan<N>::E);
      const int blocks = (nlines + LPB - 1) / LPB;
      hipLaunchKernelGGL((k_cgcg_first<C, N>), dim3(blocks), dim3(TPB), 0, op->st, (C*)op->t, x, r, p, s,
                         (const C*)w, (const C*)op->B, tw_for<C>(op, N), nlines, (const double*)kw.rows, kw.pitch, xb,
                         ks, it);
    });
    if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "contiguous axis length");
    LAUNCHCHK("k_cgcg_first");                                       // x_{it+1}, r_{it+1}, t = F B r
    if ((rc = kapply_tail<C>(op, r, w, false, nullptr, 2 | 8, kw))) return rc;   // w = P r, <w, r>, |r|^2
    ++it;
    if ((it >= first_check && (it - first_check) % check_every == 0) || it == maxit) {
      double rho, hk[2];
      if ((rc = krylov_check<C>(op, y, x, &rho))) return rc;
      if ((rc = ksum(op, kw, 5, 1, xb, ks + KS_CRR))) return rc;   // |r_it|^2
      HIPCHK(hipMemcpyAsync(hk, ks + KS_FLAG, sizeof(double), hipMemcpyDeviceToHost, op->st));
      HIPCHK(hipMemcpyAsync(hk + 1, ks + KS_CRR, sizeof(double), hipMemcpyDeviceToHost, op->st));
      HIPCHK(hipStreamSynchronize(op->st));
      mon.delta(it - 1, hk[1]);
      const bool stag = mon.check(it, rho);
      if (mon.nan) { status = USP_ERR_NAN; break; }
      if (rho < tol) { status = USP_OK; break; }
      if (hk[0] > 0.0 || stag) { status = USP_STAGNATED; break; }   // breakdown or no progress
    }
  }
  if (iters_out) *iters_out = it;
  if (status < 0) return fail(status, "non-finite values in the iteration");
  return status;
}

template <class C>
int solve_gmres(usp_op op, const C* y, C* x, int x_is_guess, int m, double tol, int maxit, const KWork& kw,
                int* iters_out, Monitor& mon) {
  const long n = op->d.N;
  C* V = kw.vec<C>(0);   // m + 1 basis vectors, then w, then b
  C* w = kw.vec<C>(m + 1);
  C* b = kw.vec<C>(m + 2);
  double* ks = kw.ks;
  double* h1 = ks + KS_H;
  double* h2 = h1 + 2 * (m + 1);
  double* zc = h2 + 2 * (m + 1);
  const int vb = vec_blocks(n);
  const int mb = (int)((n + 256L * kMdotKE - 1) / (256L * kMdotKE));
  auto basis = [&](int i) { return (C*)((char*)V + (size_t)i * kw.vec_bytes); };
  const long stride = (long)(kw.vec_bytes / sizeof(C));   // elements between basis vectors
  int rc;
  if ((rc = norm2(op, y, op->scal + 1))) return rc;
  if ((rc = kapply<C>(op, y, b, true, nullptr, 0, kw))) return rc;
  if ((rc = norm2(op, b, ks + KS_NRM))) return rc;
  double bn2 = 0.0;
  HIPCHK(hipMemcpyAsync(&bn2, ks + KS_NRM, sizeof(double), hipMemcpyDeviceToHost, op->st));
  if (!x_is_guess) HIPCHK(hipMemsetAsync(x, 0, sizeof(C) * n, op->st));
  HIPCHK(hipStreamSynchronize(op->st));
  const double bn = std::sqrt(bn2);
  typedef std::complex<double> zd;
  std::vector<zd> H((m + 1) * m), cs(m), sn(m), g(m + 1), z(m);
  std::vector<double> hh(4 * (m + 1) + 1);
  double ratio = 1.0, last_rho = -1.0;
  int total = 0, status = USP_MAXIT;
  if (!(bn > 0.0)) {
    if (iters_out) *iters_out = 0;
    return fail(USP_ERR_INVALID, "the preconditioned right-hand side is zero");
  }
  while (total < maxit) {
    if ((rc = kapply<C>(op, x, w, false, nullptr, 0, kw))) return rc;
    hipLaunchKernelGGL(k_ksub<C>, dim3(vb), dim3(256), 0, op->st, basis(0), b, w, n, kw.rows);   // r = b - P x
    LAUNCHCHK("k_ksub");
    if ((rc = ksum(op, kw, 0, 1, vb, ks + KS_NRM))) return rc;
    double beta2 = 0.0;
    HIPCHK(hipMemcpyAsync(&beta2, ks + KS_NRM, sizeof(double), hipMemcpyDeviceToHost, op->st));
    HIPCHK(hipStreamSynchronize(op->st));
    const double beta = std::sqrt(beta2);
    if (!(beta == beta)) { status = USP_ERR_NAN; break; }
    if (beta == 0.0) { status = USP_OK; break; }
    if (last_rho >= 0.0) ratio = last_rho / std::max(beta / bn, 1e-300);
    hipLaunchKernelGGL(k_kscale<C>, dim3(vb), dim3(256), 0, op->st, basis(0), basis(0), n, ks + KS_NRM);
    std::fill(H.begin(), H.end(), zd(0.0));
    std::fill(g.begin(), g.end(), zd(0.0));
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      if ((rc = kapply<C>(op, basis(j), w, false, nullptr, 0, kw))) return rc;
      // classical Gram-Schmidt, twice
      for (int pass = 0; pass < 2; ++pass) {
        double* hc = pass == 0 ? h1 : h2;
        hipLaunchKernelGGL((k_mdot<C, kMdotKE>), dim3(mb), dim3(256), 0, op->st, (const C*)V, stride, n, j + 1,
                           (const C*)w, kw.rows, kw.pitch);
        if ((rc = ksum(op, kw, 0, 2 * (j + 1), mb, hc))) return rc;
        hipLaunchKernelGGL(k_maxpy<C>, dim3(vb), dim3(256), 0, op->st, w, (const C*)V, stride, n, j + 1,
                           (const double*)hc, -1.0, pass == 1 ? kw.rows : nullptr);
      }
      LAUNCHCHK("gmres orthogonalisation");
      if ((rc = ksum(op, kw, 0, 1, vb, ks + KS_NRM))) return rc;
      HIPCHK(hipMemcpyAsync(hh.data(), h1, sizeof(double) * 4 * (m + 1), hipMemcpyDeviceToHost, op->st));
      HIPCHK(hipMemcpyAsync(hh.data() + 4 * (m + 1), ks + KS_NRM, sizeof(double), hipMemcpyDeviceToHost, op->st));
      HIPCHK(hipStreamSynchronize(op->st));
      for (int i = 0; i <= j; ++i)
        H[i * m + j] = zd(hh[2 * i] + hh[2 * (m + 1) + 2 * i], hh[2 * i + 1] + hh[2 * (m + 1) + 2 * i + 1]);
      const double hn = std::sqrt(hh[4 * (m + 1)]);
      if (!(hn == hn)) { status = USP_ERR_NAN; break; }
      H[(j + 1) * m + j] = hn;
      if (hn > 0.0) hipLaunchKernelGGL(k_kscale<C>, dim3(vb), dim3(256), 0, op->st, basis(j + 1), w, n, ks + KS_NRM);
      for (int i = 0; i < j; ++i) {
        const zd a = H[i * m + j], c = H[(i + 1) * m + j];
        H[i * m + j] = std::conj(cs[i]) * a + std::conj(sn[i]) * c;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      const double den = std::sqrt(std::norm(H[j * m + j]) + std::norm(H[(j + 1) * m + j]));
      cs[j] = H[j * m + j] / den;
      sn[j] = H[(j + 1) * m + j] / den;
      H[j * m + j] = den;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = std::conj(cs[j]) * g[j];
      k = j + 1;
      mon.delta(total, std::norm(g[j + 1]));
      ++total;
      if (hn == 0.0 || total >= maxit || std::abs(g[j + 1]) / bn * ratio < tol) break;
    }
    if (status == USP_ERR_NAN) break;
    for (int i = k - 1; i >= 0; --i) {
      zd acc = g[i];
      for (int l = i + 1; l < k; ++l) acc -= H[i * m + l] * z[l];
      z[i] = acc / H[i * m + i];
    }
    for (int i = 0; i < k; ++i) {
      hh[2 * i] = z[i].real();
      hh[2 * i + 1] = z[i].imag();
    }
    HIPCHK(hipMemcpyAsync(zc, hh.data(), sizeof(double) * 2 * k, hipMemcpyHostToDevice, op->st));
    hipLaunchKernelGGL(k_maxpy<C>, dim3(vb), dim3(256), 0, op->st, x, (const C*)V, stride, n, k, (const double*)zc,
                       1.0, (double*)nullptr);
    LAUNCHCHK("k_maxpy");
    double rho;
    if ((rc = krylov_check<C>(op, y, x, &rho))) return rc;
    last_rho = rho;
    const bool stag = mon.check(total, rho);
    if (mon.nan) { status = USP_ERR_NAN; break; }
    if (rho < tol) { status = USP_OK; break; }
    if (stag) { status = USP_STAGNATED; break; }
  }
  HIPCHK(hipStreamSynchronize(op->st));
  if (iters_out) *iters_out = total;
  if (status < 0) return fail(status, "non-finite values in the iteration");
  return status;
}

// ---- eigenmodes: shift-invert Lanczos with thick restart ---------------------

typedef std::complex<double> zd;
using usp_host::hermitian_jacobi;

struct EigWork {
  KWork kw;            // CG inner solves
  size_t basis = 0, w = 0, tmp = 0, total = 0;
  int ncv = 0;
};

int eigs_layout(usp_op op, int nev, int ncv, EigWork* ew) {
  if (nev < 1 || nev > USP_EIGS_MAX_NEV) return fail(USP_ERR_INVALID, "nev must be in [1, 16]");
  if (ncv < nev + 2 || ncv > USP_EIGS_MAX_NCV) return fail(USP_ERR_INVALID, "ncv must be in [nev + 2, 64]");
  int rc = krylov_layout(op, USP_KRYLOV_CG, 0, &ew->kw);
  if (rc) return rc;
  // partial rows for the Gram-Schmidt dot products (2 per basis vector)
  KWork& kw = ew->kw;
  kw.nrows = std::max(kw.nrows, 2 * (ncv + 1));
  kw.total = kw.vec_bytes * kw.nvec + align_up(sizeof(double) * kw.nrows * kw.pitch) + sizeof(double) * kKsDoubles;
  const size_t vb = ew->kw.vec_bytes;
  ew->ncv = ncv;
  ew->basis = align_up(ew->kw.total);
  ew->w = ew->basis + vb * (ncv + 1);
  ew->tmp = ew->w + vb;
  ew->total = ew->tmp + vb * ncv;
  return 0;
}

template <class C>
int eigs_run(usp_op op, int nev, int ncv, const C* v0, double tol, int max_restarts, double inner_tol, int inner_maxit,
             C* evecs, double* evals, double* resid, char* ws, const EigWork& ew, int* restarts_out,
             int* inner_out) {
  const long n = op->d.N;
  const KWork& kw = ew.kw;
  const size_t vbytes = kw.vec_bytes;
  const long stride = (long)(vbytes / sizeof(C));
  C* V = (C*)(ws + ew.basis);
  C* w = (C*)(ws + ew.w);
  C* T = (C*)(ws + ew.tmp);
  auto basis = [&](int i) { return (C*)((char*)V + (size_t)i * vbytes); };
  auto tmpv = [&](int i) { return (C*)((char*)T + (size_t)i * vbytes); };
  double* ks = kw.ks;
  double* h1 = ks + KS_H;
  double* h2 = h1 + 2 * (ncv + 1);
  double* coef = ks + KS_COEF;
  const int vb = vec_blocks(n);
  const int mb = (int)((n + 256L * kMdotKE - 1) / (256L * kMdotKE));
  const C* B = (const C*)op->B;
  int rc;
  // the handle must be Hermitian: real symbol, real B
  {
    const double sa0i = op->sa0[1], sa2i = op->sa2[1];
    if (std::fabs(sa0i) > 1e-14 * (std::fabs(op->sa0[0]) + 1e-300) ||
        std::fabs(sa2i) > 1e-14 * (std::fabs(op->sa2[0]) + 1e-300))
      return fail(USP_ERR_INVALID, "eigenmodes need a Hermitian operator (real symbol)");
    hipLaunchKernelGGL(k_imag2<C>, dim3(vb), dim3(256), 0, op->st, B, n, kw.rows);
    LAUNCHCHK("k_imag2");
    double im2 = 0.0;
    if ((rc = ksum(op, kw, 0, 1, vb, ks + KS_NRM))) return rc;
    HIPCHK(hipMemcpyAsync(&im2, ks + KS_NRM, sizeof(double), hipMemcpyDeviceToHost, op->st));
    HIPCHK(hipStreamSynchronize(op->st));
    if (im2 != 0.0) return fail(USP_ERR_INVALID, "eigenmodes need a Hermitian operator (real B)");
  }
  // v_0 = v0 / ||v0||
  if ((rc = norm2(op, v0, ks + KS_NRM))) return rc;
  hipLaunchKernelGGL(k_kscale<C>, dim3(vb), dim3(256), 0, op->st, basis(0), v0, n, (const double*)(ks + KS_NRM));
  LAUNCHCHK("k_kscale");
  std::vector<zd> H((size_t)(ncv + 1) * ncv, zd(0.0));
  auto Hm = [&](int i, int j) -> zd& { return H[(size_t)i * ncv + j]; };
  std::vector<double> hh(4 * (ncv + 1) + 1), cbuf(2 * ncv);
  std::vector<double> theta;
  std::vector<zd> S;
  int k = 0, total_inner = 0, cycle = 0, m = ncv;
  bool done = false;
  double beta_last = 0.0;
  std::vector<int> order(ncv);
  // u = sum_i c_i basis(i) for i < m (c on the host, complex), written to out
  auto combine = [&](const zd* c, int stride_c, C* out) -> int {
    for (int i = 0; i < m; ++i) {
      cbuf[2 * i] = c[(size_t)i * stride_c].real();
      cbuf[2 * i + 1] = c[(size_t)i * stride_c].imag();
    }
    HIPCHK(hipMemcpyAsync(coef, cbuf.data(), sizeof(double) * 2 * m, hipMemcpyHostToDevice, op->st));
    HIPCHK(hipMemsetAsync(out, 0, sizeof(C) * n, op->st));
    hipLaunchKernelGGL(k_maxpy<C>, dim3(vb), dim3(256), 0, op->st, out, (const C*)V, stride, n, m, (const double*)coef,
                       1.0, (double*)nullptr);
    LAUNCHCHK("k_maxpy");
    HIPCHK(hipStreamSynchronize(op->st));   // cbuf is reused by the next call
    return 0;
  };
  // the inner solves share the operator and the tolerance, so they take
  // similar iteration counts: the true residual is checked every 5
  // iterations from 4 before the previous solve's count (every 10 for the first)
  int prev_its = 0;
  for (cycle = 0; cycle <= max_restarts && !done; ++cycle) {
    m = ncv;
    for (int j = k; j < ncv; ++j) {
      // w = A^-1 v_j (CG on P w = B (L + I)^-1 v_j from w = 0)
      Monitor imon{nullptr, 0, nullptr, 0};
      int its = 0;
      rc = prev_its > 0 ? solve_cg<C>(op, basis(j), w, 0, inner_tol, inner_maxit, 5, kw, &its, imon,
                                      std::max(5, prev_its - 4))
                        : solve_cg<C>(op, basis(j), w, 0, inner_tol, inner_maxit, 10, kw, &its, imon);
      total_inner += its;
      if (rc == USP_OK) prev_its = its;
      if (rc < 0) return rc;
      // classical Gram-Schmidt against v_0 .. v_j, twice
      for (int pass = 0; pass < 2; ++pass) {
        double* hc = pass == 0 ? h1 : h2;
        hipLaunchKernelGGL((k_mdot<C, kMdotKE>), dim3(mb), dim3(256), 0, op->st, (const C*)V, stride, n, j + 1,
                           (const C*)w, kw.rows, kw.pitch);
        if ((rc = ksum(op, kw, 0, 2 * (j + 1), mb, hc))) return rc;
        hipLaunchKernelGGL(k_maxpy<C>, dim3(vb), dim3(256), 0, op->st, w, (const C*)V, stride, n, j + 1,
                           (const double*)hc, -1.0, pass == 1 ? kw.rows : nullptr);
      }
      LAUNCHCHK("lanczos orthogonalisation");
      if ((rc = ksum(op, kw, 0, 1, vb, ks + KS_NRM))) return rc;
      HIPCHK(hipMemcpyAsync(hh.data(), h1, sizeof(double) * 4 * (ncv + 1), hipMemcpyDeviceToHost, op->st));
      HIPCHK(hipMemcpyAsync(hh.data() + 4 * (ncv + 1), ks + KS_NRM, sizeof(double), hipMemcpyDeviceToHost, op->st));
      HIPCHK(hipStreamSynchronize(op->st));
      for (int i = 0; i <= j; ++i)
        Hm(i, j) = zd(hh[2 * i] + hh[2 * (ncv + 1) + 2 * i], hh[2 * i + 1] + hh[2 * (ncv + 1) + 2 * i + 1]);
      const double bn = std::sqrt(hh[4 * (ncv + 1)]);
      if (!(bn == bn)) return fail(USP_ERR_NAN, "non-finite values in the Lanczos basis");
      Hm(j + 1, j) = bn;
      beta_last = bn;
      if (bn <= 1e-14 * std::abs(Hm(j, j))) {   // invariant subspace: the Ritz pairs are exact
        m = j + 1;
        beta_last = 0.0;
        break;
      }
      hipLaunchKernelGGL(k_kscale<C>, dim3(vb), dim3(256), 0, op->st, basis(j + 1), (const C*)w, n,
                         (const double*)(ks + KS_NRM));
      LAUNCHCHK("k_kscale");
    }
    if (m < nev) return fail(USP_ERR_INVALID, "the start vector spans fewer than nev eigenvectors");
    // Rayleigh-Ritz: eigenpairs of the Hermitian part of the projected matrix
    std::vector<zd> Tm((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) Tm[(size_t)i * m + j] = 0.5 * (Hm(i, j) + std::conj(Hm(j, i)));
    hermitian_jacobi(m, Tm, theta, S);
    // wanted: the largest theta (A^-1), i.e. the smallest eigenvalues of A
    order.resize(m);
    for (int i = 0; i < m; ++i) order[i] = m - 1 - i;
    // Ritz vectors and their true residuals ||A u - lam u|| / ||lam u||
    done = true;
    for (int i = 0; i < nev; ++i) {
      const int c = order[i];
      C* u = evecs + (size_t)i * n;
      if ((rc = combine(&S[c], m, u))) return rc;
      const double lam = 1.0 / theta[c];
      evals[i] = lam;
      cbuf[0] = lam;
      cbuf[1] = 0.0;
      HIPCHK(hipMemcpyAsync(coef, cbuf.data(), sizeof(double) * 2, hipMemcpyHostToDevice, op->st));
      HIPCHK(hipMemsetAsync(w, 0, sizeof(C) * n, op->st));
      hipLaunchKernelGGL(k_maxpy<C>, dim3(vb), dim3(256), 0, op->st, w, (const C*)u, stride, n, 1,
                         (const double*)coef, 1.0, (double*)nullptr);   // w = lam u
      LAUNCHCHK("k_maxpy");
      if ((rc = norm2(op, (const C*)w, op->scal + 1))) return rc;
      if ((rc = residual_passes<C>(op, u, (const C*)w, B, nullptr, nullptr))) return rc;
      double hs[2];
      HIPCHK(hipMemcpyAsync(hs, op->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, op->st));
      HIPCHK(hipStreamSynchronize(op->st));
      resid[i] = std::sqrt(hs[0] / hs[1]);
      if (!(resid[i] == resid[i])) return fail(USP_ERR_NAN, "non-finite Ritz vector");
      if (!(resid[i] < tol)) done = false;
    }
    if (done || cycle == max_restarts || beta_last == 0.0) {
      done = true;
      break;
    }
    // thick restart: keep kk Ritz vectors and the next Lanczos vector
    const int kk = std::min(ncv - 1, nev + (ncv - nev) / 2);
    for (int i = 0; i < kk; ++i)
      if ((rc = combine(&S[order[i]], m, tmpv(i)))) return rc;
    for (int i = 0; i < kk; ++i)
      HIPCHK(hipMemcpyAsync(basis(i), tmpv(i), sizeof(C) * n, hipMemcpyDeviceToDevice, op->st));
    HIPCHK(hipMemcpyAsync(basis(kk), basis(ncv), sizeof(C) * n, hipMemcpyDeviceToDevice, op->st));
    std::fill(H.begin(), H.end(), zd(0.0));
    for (int i = 0; i < kk; ++i) {
      Hm(i, i) = theta[order[i]];
      Hm(kk, i) = beta_last * S[(size_t)(m - 1) * m + order[i]];
    }
    k = kk;
  }
  // ascending eigenvalues of A (the order of the loop above already is)
  if (restarts_out) *restarts_out = cycle;
  if (inner_out) *inner_out = total_inner;
  HIPCHK(hipStreamSynchronize(op->st));
  bool conv = true;
  for (int i = 0; i < nev; ++i) conv = conv && resid[i] < tol;
  return conv ? USP_OK : USP_MAXIT;
}

void cmulh(const double a[2], const double b[2], double out[2]) {
  const double r = a[0] * b[0] - a[1] * b[1], i = a[0] * b[1] + a[1] * b[0];
  out[0] = r;
  out[1] = i;
}

}  // namespace

// ---- static device scratch (callers that cannot allocate device memory) ----
//
// usp_residual_static keeps everything it needs besides its inputs in this
// array: the twiddle tables of every length 8 .. 1024 (written once per
// device), the per-block partial rows, two scalars and the FP64 spectrum of
// A x.  Each GPU the library runs on holds its own copy until the process
// ends.  In host code `scratch` only stands in for the symbol: its device
// address, different on every GPU, comes from hipGetSymbolAddress with that
// device current and is the only pointer passed to kernels.
static __device__ __align__(256) char scratch[USP_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kTwdBytes = sizeof(double2) * 2040;   // lengths 8 .. 1024: sum = 2040 entries
constexpr size_t kTwfBytes = sizeof(float2) * 2040;
constexpr size_t kTwRegion = 49152;                    // both tables, 256-byte aligned
static_assert(kTwdBytes + kTwfBytes <= kTwRegion, "twiddle region");

std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxDevices] = {nullptr};

// offset of the length-n table (n = 2^l, 3 <= l <= 10) in entries: 8 + 16 + ... + n/2 = n - 8
inline size_t tw_entry(int n) { return (size_t)n - 8; }

// the current device's scratch address; on the first call for a device its
// address is looked up and the twiddle tables exp(-2 pi i k / n), computed in
// long double, are copied in
int static_scratch(char** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(USP_ERR_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(USP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    static double2 td[2040];
    static float2 tf[2040];
    for (int l = 3; l <= 10; ++l) {
      const int n = 1 << l;
      for (int k = 0; k < n; ++k) {
        const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)k / (long double)n;
        const long double c = cosl(a), sn = sinl(a);
        td[tw_entry(n) + k].x = (double)c;
        td[tw_entry(n) + k].y = (double)sn;
        tf[tw_entry(n) + k].x = (float)c;
        tf[tw_entry(n) + k].y = (float)sn;
      }
    }
    char* base = (char*)p;
    if (hipMemcpy(base, td, kTwdBytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + kTwdBytes, tf, kTwfBytes, hipMemcpyHostToDevice) != hipSuccess)
      return fail(USP_ERR_HIP, "twiddle upload to the static scratch failed");
    g_scratch_dev[dev] = base;
  }
  *out = g_scratch_dev[dev];
  return 0;
}

}  // namespace

extern "C" {

const char* usp_last_error(void) { return g_err.c_str(); }

int usp_workspace_bytes(const usp_symbol* L, int dtype, int flags, size_t* bytes) {
  Layout lay;
  Dims d;
  int rc = make_layout(L, dtype, flags, &lay, &d);
  if (rc) return rc;
  if (!bytes) return fail(USP_ERR_INVALID, "bytes is NULL");
  *bytes = lay.total;
  return 0;
}

int usp_prepare_operator(const usp_symbol* L, int dtype, int flags, const void* B_dev, const usp_gather* gather,
                         void* workspace_dev, size_t workspace_bytes, void* stream, usp_op* out) {
  if (!out) return fail(USP_ERR_INVALID, "out is NULL");
  *out = nullptr;
  Layout lay;
  Dims d;
  int rc = make_layout(L, dtype, flags, &lay, &d);
  if (rc) return rc;
  if (!B_dev) return fail(USP_ERR_INVALID, "B_dev is NULL");
  if (!workspace_dev || workspace_bytes < lay.total)
    return fail(USP_ERR_WORKSPACE, "workspace too small: need " + std::to_string(lay.total) + " bytes");
  if (((uintptr_t)workspace_dev) & 255) return fail(USP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (gather && d.ndim != 1) return fail(USP_ERR_INVALID, "a gather term needs ndim == 1");
  if (gather && (!gather->idx_dev || !gather->g0_dev || !gather->g1_dev))
    return fail(USP_ERR_INVALID, "gather arrays must be non-NULL");

  usp_op op = new usp_op_s();
  op->d = d;
  op->dtype = dtype;
  op->flags = flags;
  op->refine = (flags & USP_FLAG_REFINE) != 0;
  op->st = (hipStream_t)stream;
  op->sym = *L;
  op->B = B_dev;
  op->has_gather = gather != nullptr;
  if (gather) op->g = *gather;
  op->ws = (char*)workspace_dev;
  op->lay = lay;
  char* w = op->ws;
  if (d.ndim >= 2) {
    op->t = w + lay.t;
    op->S = (double2*)(w + lay.S);
    if (op->refine) {
      op->B32 = (float2*)(w + lay.B32);
      op->r32 = (float2*)(w + lay.r32);
      op->d32 = (float2*)(w + lay.d32);
    }
  }
  op->partials = (double*)(w + lay.partials);
  op->pitch = lay.nblk;
  op->hist = (double*)(w + lay.hist);
  op->scal = (double*)(w + lay.scal);
  op->hist_true = (double*)(w + lay.hist_true);
  op->info = (Solve1DInfo*)(w + lay.info);
  op->antisym = (flags & USP_FLAG_ANTISYM) != 0;
  if (op->antisym) {
    op->adj_j = (int*)(w + lay.adj_j);
    op->adj_w = w + lay.adj_w;
  }
  cmulh(L->s, L->a0, op->sa0);
  cmulh(L->s, L->a1, op->sa1);
  cmulh(L->s, L->a2, op->sa2);

  auto cleanup = [&](int code) {
    delete op;
    return code;
  };
  // twiddle tables exp(-2 pi i k / n), computed in long double
  for (int l = 3; l <= 10; ++l) {
    const int n = 1 << l;
    if (!lay.twd[l]) continue;
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
    op->twf[l] = (float2*)(w + lay.twf[l]);
    op->twd[l] = (double2*)(w + lay.twd[l]);
    if (hipMemcpyAsync(op->twf[l], tf.data(), n * sizeof(float2), hipMemcpyHostToDevice, op->st) != hipSuccess ||
        hipMemcpyAsync(op->twd[l], td.data(), n * sizeof(double2), hipMemcpyHostToDevice, op->st) != hipSuccess ||
        hipStreamSynchronize(op->st) != hipSuccess)
      return cleanup(fail(USP_ERR_HIP, "twiddle upload failed"));
  }
  if (op->antisym) {
    // table of the adjoint gather G*: row k lists (j, conj(g)) for every G[j][k] = g
    const long n = d.N;
    const size_t es = dtype == USP_C64 ? 8 : 16;
    std::vector<int> aj(n * kAdjMax, -1);
    std::vector<char> aw(n * kAdjMax * es, 0);
    if (gather) {
      std::vector<int> gi(n);
      std::vector<char> g0(n * es), g1(n * es);
      if (hipStreamSynchronize(op->st) != hipSuccess ||
          hipMemcpy(gi.data(), gather->idx_dev, n * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(g0.data(), gather->g0_dev, n * es, hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(g1.data(), gather->g1_dev, n * es, hipMemcpyDeviceToHost) != hipSuccess)
        return cleanup(fail(USP_ERR_HIP, "gather readback failed"));
      std::vector<int> cnt(n, 0);
      bool wide = false;
      auto add = [&](long k, long j, const char* g) {
        bool zero;  // by value: weights of empty rows may be -0.0
        if (es == 8) {
          float2 v;
          std::memcpy(&v, g, 8);
          zero = v.x == 0.0f && v.y == 0.0f;
        } else {
          double2 v;
          std::memcpy(&v, g, 16);
          zero = v.x == 0.0 && v.y == 0.0;
        }
        if (zero) return;
        if (cnt[k] >= kAdjMax) {
          wide = true;
          return;
        }
        const int a = cnt[k]++;
        aj[k * kAdjMax + a] = (int)j;
        char* dst = aw.data() + (k * kAdjMax + a) * es;
        std::memcpy(dst, g, es);
        if (es == 8) {  // conjugate
          float im;
          std::memcpy(&im, dst + 4, 4);
          im = -im;
          std::memcpy(dst + 4, &im, 4);
        } else {
          double im;
          std::memcpy(&im, dst + 8, 8);
          im = -im;
          std::memcpy(dst + 8, &im, 8);
        }
      };
      for (long j = 0; j < n; ++j) {
        const long i0 = std::min<long>(std::max(gi[j], 0), n - 1);
        const long i1 = std::min<long>(i0 + 1, n - 1);
        add(i0, j, g0.data() + j * es);
        add(i1, j, g1.data() + j * es);
      }
      if (wide) return cleanup(fail(USP_ERR_UNSUPPORTED_SHAPE, "the adjoint gather has more than 8 entries per row"));
    }
    if (hipMemcpyAsync(op->adj_j, aj.data(), aj.size() * sizeof(int), hipMemcpyHostToDevice, op->st) != hipSuccess ||
        hipMemcpyAsync(op->adj_w, aw.data(), aw.size(), hipMemcpyHostToDevice, op->st) != hipSuccess ||
        hipStreamSynchronize(op->st) != hipSuccess)
      return cleanup(fail(USP_ERR_HIP, "adjoint table upload failed"));
  }
  if (op->refine) {
    hipLaunchKernelGGL(k_to_c64, dim3(1024), dim3(256), 0, op->st, (const double2*)B_dev, op->B32, d.N);
    if (hipGetLastError() != hipSuccess) return cleanup(fail(USP_ERR_HIP, "k_to_c64 launch failed"));
  }
  // ||V|| < 1 (diagonal part): max |1 - B|
  {
    const int blocks = (int)std::min<long>((d.N + 255) / 256, 1024);
    if (dtype == USP_C64)
      hipLaunchKernelGGL((k_max_v<float2>), dim3(blocks), dim3(256), 0, op->st, (const float2*)B_dev, d.N, op->partials);
    else
      hipLaunchKernelGGL((k_max_v<double2>), dim3(blocks), dim3(256), 0, op->st, (const double2*)B_dev, d.N,
                         op->partials);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, op->st, op->partials, blocks, op->scal + 2);
    if (hipGetLastError() != hipSuccess) return cleanup(fail(USP_ERR_HIP, "k_max_v launch failed"));
    double vmax = 0;
    if (hipMemcpyAsync(&vmax, op->scal + 2, sizeof(double), hipMemcpyDeviceToHost, op->st) != hipSuccess ||
        hipStreamSynchronize(op->st) != hipSuccess)
      return cleanup(fail(USP_ERR_HIP, "max|v| readback failed"));
    if (!(vmax < 1.0))
      return cleanup(fail(USP_ERR_NOT_CONTRACTIVE, "max|v| = " + std::to_string(vmax) + " is not < 1"));
  }
  *out = op;
  return 0;
}

int usp_destroy(usp_op op) {
  delete op;
  return 0;
}

int usp_solve(usp_op op, const void* y_dev, void* x_dev, int x_is_guess, double alpha, double tol, int maxit,
              int check_every, int* iters_out, double* hist_pre, int hist_pre_cap, double* hist_true,
              int hist_true_cap, int* n_true_out) {
  if (!op || !y_dev || !x_dev) return fail(USP_ERR_INVALID, "NULL argument");
  if (!(alpha > 0.0) || maxit < 0 || check_every < 1) return fail(USP_ERR_INVALID, "alpha > 0, maxit >= 0, check_every >= 1");
  Monitor mon{hist_pre, hist_pre_cap, hist_true, hist_true_cap};
  int rc;
  if (op->d.ndim == 1) {
    if (op->dtype == USP_C64)
      rc = solve_1d<float2>(op, (const float2*)y_dev, (float2*)x_dev, x_is_guess, alpha, tol, maxit, check_every,
                            iters_out, mon);
    else
      rc = solve_1d<double2>(op, (const double2*)y_dev, (double2*)x_dev, x_is_guess, alpha, tol, maxit,
                             check_every, iters_out, mon);
  } else if (op->refine) {
    rc = solve_refined(op, (const double2*)y_dev, (double2*)x_dev, x_is_guess, alpha, tol, maxit, check_every,
                       iters_out, mon);
  } else if (op->dtype == USP_C64) {
    rc = solve_plain<float2>(op, (const float2*)y_dev, (float2*)x_dev, x_is_guess, alpha, tol, maxit, check_every,
                             iters_out, mon, true);
  } else {
    rc = solve_plain<double2>(op, (const double2*)y_dev, (double2*)x_dev, x_is_guess, alpha, tol, maxit,
                              check_every, iters_out, mon, true);
  }
  if (n_true_out) *n_true_out = mon.n_true;
  return rc;
}

int usp_apply_precond(usp_op op, const void* v_dev, void* w_dev, int rhs, void* ws_dev, size_t ws_bytes) {
  if (!op || !v_dev || !w_dev) return fail(USP_ERR_INVALID, "NULL argument");
  KWork kw;
  int rc = krylov_layout(op, USP_KRYLOV_BICGSTAB, 0, &kw);
  if (rc) return rc;
  if ((rc = krylov_bind(&kw, ws_dev, ws_bytes))) return rc;
  rc = op->dtype == USP_C64 ? kapply<float2>(op, (const float2*)v_dev, (float2*)w_dev, rhs != 0, nullptr, 0, kw)
                            : kapply<double2>(op, (const double2*)v_dev, (double2*)w_dev, rhs != 0, nullptr, 0, kw);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(op->st));
  return 0;
}

int usp_krylov_workspace_bytes(usp_op op, int method, int restart, size_t* bytes) {
  if (!op || !bytes) return fail(USP_ERR_INVALID, "NULL argument");
  KWork kw;
  int rc = krylov_layout(op, method, restart, &kw);
  if (rc) return rc;
  *bytes = kw.total;
  return 0;
}

int usp_hermitian_eig(int n, const double* a, double* w_out, double* z_out) {
  if (n < 1 || n > 256 || !a || !w_out || !z_out) return fail(USP_ERR_INVALID, "n in [1, 256] and non-NULL arrays");
  std::vector<zd> A((size_t)n * n);
  for (size_t i = 0; i < A.size(); ++i) {
    if (!std::isfinite(a[2 * i]) || !std::isfinite(a[2 * i + 1])) return fail(USP_ERR_NAN, "non-finite matrix entry");
    A[i] = zd(a[2 * i], a[2 * i + 1]);
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      A[(size_t)i * n + j] = 0.5 * (A[(size_t)i * n + j] + std::conj(A[(size_t)j * n + i]));
  std::vector<double> w;
  std::vector<zd> Z;
  hermitian_jacobi(n, A, w, Z);
  for (int i = 0; i < n; ++i) w_out[i] = w[i];
  for (size_t i = 0; i < Z.size(); ++i) {
    z_out[2 * i] = Z[i].real();
    z_out[2 * i + 1] = Z[i].imag();
  }
  return 0;
}

int usp_eigs_workspace_bytes(usp_op op, int nev, int ncv, size_t* bytes) {
  if (!op || !bytes) return fail(USP_ERR_INVALID, "NULL argument");
  EigWork ew;
  int rc = eigs_layout(op, nev, ncv, &ew);
  if (rc) return rc;
  *bytes = ew.total;
  return 0;
}

int usp_eigs(usp_op op, int nev, int ncv, const void* v0_dev, double tol, int max_restarts, double inner_tol,
             int inner_maxit, void* evecs_dev, double* evals_out, double* resid_out, void* ws_dev, size_t ws_bytes,
             int* restarts_out, int* inner_iters_out) {
  if (!op || !v0_dev || !evecs_dev || !evals_out || !resid_out) return fail(USP_ERR_INVALID, "NULL argument");
  if (!(tol > 0.0) || max_restarts < 0 || !(inner_tol > 0.0) || inner_maxit < 1)
    return fail(USP_ERR_INVALID, "tol > 0, max_restarts >= 0, inner_tol > 0, inner_maxit >= 1");
  EigWork ew;
  int rc = eigs_layout(op, nev, ncv, &ew);
  if (rc) return rc;
  if (!ws_dev || ws_bytes < ew.total)
    return fail(USP_ERR_WORKSPACE, "eigs workspace too small: need " + std::to_string(ew.total) + " bytes");
  if ((rc = krylov_bind(&ew.kw, ws_dev, ws_bytes))) return rc;
  if (op->dtype == USP_C64)
    return eigs_run<float2>(op, nev, ncv, (const float2*)v0_dev, tol, max_restarts, inner_tol, inner_maxit,
                            (float2*)evecs_dev, evals_out, resid_out, (char*)ws_dev, ew, restarts_out,
                            inner_iters_out);
  return eigs_run<double2>(op, nev, ncv, (const double2*)v0_dev, tol, max_restarts, inner_tol, inner_maxit,
                           (double2*)evecs_dev, evals_out, resid_out, (char*)ws_dev, ew, restarts_out,
                           inner_iters_out);
}

int usp_solve_krylov(usp_op op, int method, int restart, const void* y_dev, void* x_dev, int x_is_guess, double tol,
                     int maxit, int check_every, void* ws_dev, size_t ws_bytes, int* iters_out, double* hist_est,
                     int hist_est_cap, double* hist_true, int hist_true_cap, int* n_true_out) {
  if (!op || !y_dev || !x_dev) return fail(USP_ERR_INVALID, "NULL argument");
  if (maxit < 0 || check_every < 1) return fail(USP_ERR_INVALID, "maxit >= 0, check_every >= 1");
  KWork kw;
  int rc = krylov_layout(op, method, restart, &kw);
  if (rc) return rc;
  if ((rc = krylov_bind(&kw, ws_dev, ws_bytes))) return rc;
  Monitor mon{hist_est, hist_est_cap, hist_true, hist_true_cap};
  if (method == USP_KRYLOV_CG) {
    rc = op->dtype == USP_C64
             ? solve_cg<float2>(op, (const float2*)y_dev, (float2*)x_dev, x_is_guess, tol, maxit, check_every, kw,
                                iters_out, mon)
             : solve_cg<double2>(op, (const double2*)y_dev, (double2*)x_dev, x_is_guess, tol, maxit, check_every, kw,
                                 iters_out, mon);
  } else if (method == USP_KRYLOV_BICGSTAB) {
    rc = op->dtype == USP_C64
             ? solve_bicgstab<float2>(op, (const float2*)y_dev, (float2*)x_dev, x_is_guess, tol, maxit, check_every,
                                      kw, iters_out, mon)
             : solve_bicgstab<double2>(op, (const double2*)y_dev, (double2*)x_dev, x_is_guess, tol, maxit,
                                       check_every, kw, iters_out, mon);
  } else {
    rc = op->dtype == USP_C64
             ? solve_gmres<float2>(op, (const float2*)y_dev, (float2*)x_dev, x_is_guess, restart, tol, maxit, kw,
                                   iters_out, mon)
             : solve_gmres<double2>(op, (const double2*)y_dev, (double2*)x_dev, x_is_guess, restart, tol, maxit, kw,
                                    iters_out, mon);
  }
  if (n_true_out) *n_true_out = mon.n_true;
  return rc;
}

int usp_iterate(usp_op op, const void* y_dev, void* x_dev, int x_is_guess, double alpha, int K, double* hist_pre,
                int hist_pre_cap) {
  if (!op || !y_dev || !x_dev) return fail(USP_ERR_INVALID, "NULL argument");
  if (op->refine) return fail(USP_ERR_INVALID, "usp_iterate is not available in refined mode");
  if (K < 0) return fail(USP_ERR_INVALID, "K >= 0");
  Monitor mon{hist_pre, hist_pre_cap, nullptr, 0};
  int it = 0, rc;
  if (op->d.ndim == 1) {
    if (op->dtype == USP_C64)
      rc = solve_1d<float2>(op, (const float2*)y_dev, (float2*)x_dev, x_is_guess, alpha, -1.0, K, K + 1, &it, mon);
    else
      rc = solve_1d<double2>(op, (const double2*)y_dev, (double2*)x_dev, x_is_guess, alpha, -1.0, K, K + 1, &it,
                             mon);
  } else if (op->dtype == USP_C64) {
    rc = solve_plain<float2>(op, (const float2*)y_dev, (float2*)x_dev, x_is_guess, alpha, -1.0, K, K + 1, &it, mon,
                             false);
  } else {
    rc = solve_plain<double2>(op, (const double2*)y_dev, (double2*)x_dev, x_is_guess, alpha, -1.0, K, K + 1, &it,
                              mon, false);
  }
  if (rc < 0) return rc;
  return 0;
}

int usp_residual(usp_op op, const void* y_dev, const void* x_dev, double* rel_out, double* rnorm_out,
                 double* ynorm_out) {
  if (!op || !y_dev || !x_dev) return fail(USP_ERR_INVALID, "NULL argument");
  double host[2];
  int rc;
  if (op->d.ndim == 1) {
    rc = op->dtype == USP_C64 ? residual_1d<float2>(op, (const float2*)y_dev, (const float2*)x_dev, host)
                              : residual_1d<double2>(op, (const double2*)y_dev, (const double2*)x_dev, host);
    if (rc) return rc;
  } else {
    if (op->dtype == USP_C64 && !op->refine) {
      if ((rc = norm2(op, (const float2*)y_dev, op->scal + 1))) return rc;
      rc = residual_passes<float2>(op, (float2*)x_dev, (const float2*)y_dev, (const float2*)op->B, nullptr, nullptr);
    } else {
      if ((rc = norm2(op, (const double2*)y_dev, op->scal + 1))) return rc;
      rc = residual_passes<double2>(op, (double2*)x_dev, (const double2*)y_dev, (const double2*)op->B, nullptr,
                                    nullptr);
    }
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(host, op->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, op->st));
    HIPCHK(hipStreamSynchronize(op->st));
  }
  if (rel_out) *rel_out = std::sqrt(host[0] / host[1]);
  if (rnorm_out) *rnorm_out = std::sqrt(host[0]);
  if (ynorm_out) *ynorm_out = std::sqrt(host[1]);
  return 0;
}

int usp_profile(usp_op op, const void* y_dev, void* x_dev, double alpha, int K, double* pass_ms, double* iter_ms) {
  if (!op || !y_dev || !x_dev || !pass_ms || K < 1) return fail(USP_ERR_INVALID, "invalid argument");
  if (op->d.ndim < 2) return fail(USP_ERR_INVALID, "usp_profile is for 2-D / 3-D grids");
  std::vector<hipEvent_t> ev[USP_NPASS];
  op->prof = ev;
  int rc = 0;
  auto run = [&]() -> int {
    int r;
    if (op->refine) {
      if ((r = norm2(op, (const double2*)y_dev, op->scal + 1))) return r;
      if ((r = residual_passes<double2>(op, (double2*)x_dev, (const double2*)y_dev, (const double2*)op->B, nullptr,
                                        op->r32)))
        return r;
      HIPCHK(hipMemsetAsync(op->d32, 0, sizeof(float2) * op->d.N, op->st));
      if ((r = first_pass<float2>(op, op->d32, op->r32, op->B32, 0))) return r;
      for (int j = 0; j < K; ++j)
        if ((r = iteration<float2>(op, op->d32, op->r32, op->B32, alpha))) return r;
    } else if (op->dtype == USP_C64) {
      const float2 *y = (const float2*)y_dev, *B = (const float2*)op->B;
      float2* x = (float2*)x_dev;
      if ((r = norm2(op, y, op->scal + 1))) return r;
      HIPCHK(hipMemsetAsync(x, 0, sizeof(float2) * op->d.N, op->st));
      if ((r = first_pass<float2>(op, x, y, B, 0))) return r;
      for (int j = 0; j < K; ++j)
        if ((r = iteration<float2>(op, x, y, B, alpha))) return r;
      if ((r = residual_passes<float2>(op, x, y, B, nullptr, nullptr))) return r;
    } else {
      const double2 *y = (const double2*)y_dev, *B = (const double2*)op->B;
      double2* x = (double2*)x_dev;
      if ((r = norm2(op, y, op->scal + 1))) return r;
      HIPCHK(hipMemsetAsync(x, 0, sizeof(double2) * op->d.N, op->st));
      if ((r = first_pass<double2>(op, x, y, B, 0))) return r;
      for (int j = 0; j < K; ++j)
        if ((r = iteration<double2>(op, x, y, B, alpha))) return r;
      if ((r = residual_passes<double2>(op, x, y, B, nullptr, nullptr))) return r;
    }
    return 0;
  };
  op->pending = op->pending_first = 0;
  rc = run();
  if (!rc) rc = finalize_hist(op);
  op->prof = nullptr;
  if (hipStreamSynchronize(op->st) != hipSuccess && !rc) rc = fail(USP_ERR_HIP, "synchronize failed");
  for (int k = 0; k < USP_NPASS; ++k) {
    double tot = 0.0;
    const size_t n = ev[k].size() / 2;
    for (size_t i = 0; i < n; ++i) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, ev[k][2 * i], ev[k][2 * i + 1]);
      tot += ms;
    }
    pass_ms[k] = n ? tot / n : 0.0;
    for (hipEvent_t e : ev[k]) hipEventDestroy(e);
  }
  if (rc) return rc;
  if (iter_ms) {
    // whole iterations, no per-pass events
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int r = 0;
    HIPCHK(hipEventRecord(e0, op->st));
    for (int j = 0; j < K && !r; ++j) {
      if (op->refine) r = iteration<float2>(op, op->d32, op->r32, op->B32, alpha);
      else if (op->dtype == USP_C64)
        r = iteration<float2>(op, (float2*)x_dev, (const float2*)y_dev, (const float2*)op->B, alpha);
      else
        r = iteration<double2>(op, (double2*)x_dev, (const double2*)y_dev, (const double2*)op->B, alpha);
    }
    HIPCHK(hipEventRecord(e1, op->st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (r) return r;
    *iter_ms = ms / K;
  }
  return 0;
}

int usp_residual_static(const usp_symbol* L, int dtype, const void* B_dev, const void* y_dev, const void* x_dev,
                        double* rel_out, double* rnorm_out, double* ynorm_out, void* stream) {
  if (!L || !B_dev || !y_dev || !x_dev) return fail(USP_ERR_INVALID, "NULL argument");
  Layout lay;
  Dims d;
  int rc = make_layout(L, dtype, 0, &lay, &d);   // validates the symbol and dtype
  if (rc) return rc;
  // scratch: twiddles | scalars | partial rows | FP64 spectrum (2-D / 3-D)
  const long nblk = (long)d.n0 * d.n1 + 4096;
  const size_t off_scal = kTwRegion;
  const size_t off_part = align_up(off_scal + 64 * sizeof(double));
  const size_t off_S = align_up(off_part + sizeof(double) * nblk * (kRows + 2));
  const size_t need = d.ndim >= 2 ? align_up(off_S + (size_t)d.N * 16) : off_S;
  if (need > (size_t)USP_STATIC_SCRATCH_BYTES)
    return fail(USP_ERR_WORKSPACE, "grid too large for the static scratch: needs " + std::to_string(need) +
                                       " bytes of " + std::to_string((size_t)USP_STATIC_SCRATCH_BYTES));
  char* base = nullptr;
  if ((rc = static_scratch(&base))) return rc;
  // an operator record on the stack over the scratch (no allocation)
  usp_op_s o;
  o.d = d;
  o.dtype = dtype;
  o.st = (hipStream_t)stream;
  o.sym = *L;
  o.B = B_dev;
  o.S = d.ndim >= 2 ? (double2*)(base + off_S) : nullptr;
  o.partials = (double*)(base + off_part);
  o.pitch = nblk;
  o.scal = (double*)(base + off_scal);
  for (int l = 3; l <= 10; ++l) {
    o.twd[l] = (double2*)base + tw_entry(1 << l);
    o.twf[l] = (float2*)(base + kTwdBytes) + tw_entry(1 << l);
  }
  cmulh(L->s, L->a0, o.sa0);
  cmulh(L->s, L->a1, o.sa1);
  cmulh(L->s, L->a2, o.sa2);
  double host[2];
  if (d.ndim == 1) {
    rc = dtype == USP_C64 ? residual_1d<float2>(&o, (const float2*)y_dev, (const float2*)x_dev, host)
                          : residual_1d<double2>(&o, (const double2*)y_dev, (const double2*)x_dev, host);
    if (rc) return rc;
  } else {
    if (dtype == USP_C64) {
      if ((rc = norm2(&o, (const float2*)y_dev, o.scal + 1))) return rc;
      rc = residual_passes<float2>(&o, (float2*)x_dev, (const float2*)y_dev, (const float2*)B_dev, nullptr, nullptr);
    } else {
      if ((rc = norm2(&o, (const double2*)y_dev, o.scal + 1))) return rc;
      rc = residual_passes<double2>(&o, (double2*)x_dev, (const double2*)y_dev, (const double2*)B_dev, nullptr,
                                    nullptr);
    }
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(host, o.scal, 2 * sizeof(double), hipMemcpyDeviceToHost, o.st));
    HIPCHK(hipStreamSynchronize(o.st));
  }
  if (rel_out) *rel_out = std::sqrt(host[0] / host[1]);
  if (rnorm_out) *rnorm_out = std::sqrt(host[0]);
  if (ynorm_out) *ynorm_out = std::sqrt(host[1]);
  return 0;
}

int usp_get_plan(usp_op op, usp_plan* out) {
  if (!op || !out) return fail(USP_ERR_INVALID, "NULL argument");
  *out = op->plan;
  return 0;
}

int usp_set_plan(usp_op op, const usp_plan* plan) {
  if (!op || !plan) return fail(USP_ERR_INVALID, "NULL argument");
  for (int w : {plan->w_mid, plan->w_sym})
    if (!(w == 0 || w == 4 || w == 8 || w == 16 || w == 32)) return fail(USP_ERR_INVALID, "tile width must be 0, 4, 8, 16 or 32");
  if (plan->r_load < 0 || plan->r_load > 3) return fail(USP_ERR_INVALID, "r_load must be 0 to 3");
  op->plan = *plan;
  return 0;
}

int usp_autotune(usp_op op, const void* y_dev, void* x_dev, double alpha, int reps, usp_plan* best_out) {
  if (!op || !y_dev || !x_dev || reps < 1) return fail(USP_ERR_INVALID, "invalid argument");
  if (op->d.ndim < 2) {
    if (best_out) *best_out = op->plan;
    return 0;
  }
  const bool c64 = op->refine || op->dtype == USP_C64;
  const int ws_c64[] = {8, 16, 32}, ws_c128[] = {4, 8, 16};
  const int* ws = c64 ? ws_c64 : ws_c128;
  std::vector<usp_plan> cands;
  for (int fl = 0; fl < 4; ++fl)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        usp_plan p = op->plan;
        p.x_prefetch = fl & 1;
        p.x_stream = (fl >> 1) & 1;
        p.w_mid = op->d.ndim == 3 ? ws[a] : 0;
        p.w_sym = ws[b];
        if (op->d.ndim == 2 && a > 0) continue;
        if ((p.w_mid && !(c64 ? width_ok<float2>(op->d.n1, p.w_mid) : width_ok<double2>(op->d.n1, p.w_mid))) ||
            !(c64 ? width_ok<float2>(op->d.n0, p.w_sym) : width_ok<double2>(op->d.n0, p.w_sym)))
          continue;
        cands.push_back(p);
      }
  const usp_plan saved = op->plan;
  double best_ms = INFINITY;
  usp_plan best = saved;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (const usp_plan& p : cands) {
    op->plan = p;
    double ms_min = INFINITY;
    for (int rep = 0; rep < 2; ++rep) {
      int r = 0;
      HIPCHK(hipEventRecord(e0, op->st));
      for (int j = 0; j < reps && !r; ++j) {
        if (op->refine) r = iteration<float2>(op, op->d32, op->r32, op->B32, alpha);
        else if (op->dtype == USP_C64)
          r = iteration<float2>(op, (float2*)x_dev, (const float2*)y_dev, (const float2*)op->B, alpha);
        else
          r = iteration<double2>(op, (double2*)x_dev, (const double2*)y_dev, (const double2*)op->B, alpha);
      }
      HIPCHK(hipEventRecord(e1, op->st));
      HIPCHK(hipEventSynchronize(e1));
      if (r) {
        op->plan = saved;
        return r;
      }
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      ms_min = std::min(ms_min, (double)ms);
    }
    if (ms_min < best_ms) {
      best_ms = ms_min;
      best = p;
    }
  }
  // the FP64 residual's load plan: one residual evaluation per candidate
  for (int rl = 0; rl < 4; ++rl) {
    usp_plan p = best;
    p.r_load = rl;
    op->plan = p;
    double ms_min = INFINITY;
    for (int rep = 0; rep < 3; ++rep) {
      int r = 0;
      HIPCHK(hipEventRecord(e0, op->st));
      if (op->refine || op->dtype == USP_C128)
        r = residual_passes<double2>(op, (double2*)x_dev, (const double2*)y_dev, (const double2*)op->B, nullptr,
                                     nullptr);
      else
        r = residual_passes<float2>(op, (float2*)x_dev, (const float2*)y_dev, (const float2*)op->B, nullptr,
                                    nullptr);
      HIPCHK(hipEventRecord(e1, op->st));
      HIPCHK(hipEventSynchronize(e1));
      if (r) {
        op->plan = saved;
        return r;
      }
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      ms_min = std::min(ms_min, (double)ms);
    }
    if (rl == 0 || ms_min < best_ms) {
      best_ms = ms_min;
      best.r_load = rl;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  op->pending = op->pending_first = 0;
  op->plan = best;
  if (best_out) *best_out = best;
  return 0;
}

int usp_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream) {
  if (!src_dev || !dst_dev) return fail(USP_ERR_INVALID, "NULL argument");
  if ((((uintptr_t)src_dev) | ((uintptr_t)dst_dev) | bytes) & 15)
    return fail(USP_ERR_INVALID, "pointers and size must be multiples of 16 bytes");
  const char *s = (const char*)src_dev, *d = (const char*)dst_dev;
  if (s < d + bytes && d < s + bytes) return fail(USP_ERR_INVALID, "buffers overlap");
  const long n = (long)(bytes / 16);
  if (n == 0) return 0;
  const long chunk = 256L * kCopyUnroll;
  const long blocks = (n + chunk - 1) / chunk;
  if (blocks > 0x7fffffffL) return fail(USP_ERR_INVALID, "copy too large");
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     (const double2*)src_dev, (double2*)dst_dev, n);
  LAUNCHCHK("k_stream_copy");
  return 0;
}

int usp_canonical_fields(const void* q_dev, const void* S_dev, size_t n, const double* bias, const double* c,
                         double src_scale, int dtype, void* B_dev, void* y_dev, void* stream) {
  if (!q_dev || !S_dev || !bias || !c) return fail(USP_ERR_INVALID, "NULL argument");
  if (c[0] == 0.0 && c[1] == 0.0) return fail(USP_ERR_INVALID, "c must be non-zero");
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  if (dtype == USP_C64)
    hipLaunchKernelGGL((k_canonical_fields<float2>), dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const double2*)q_dev, (const double2*)S_dev, (long)n, bias[0], bias[1], c[0], c[1],
                       src_scale, (float2*)B_dev, (float2*)y_dev);
  else if (dtype == USP_C128)
    hipLaunchKernelGGL((k_canonical_fields<double2>), dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const double2*)q_dev, (const double2*)S_dev, (long)n, bias[0], bias[1], c[0], c[1],
                       src_scale, (double2*)B_dev, (double2*)y_dev);
  else
    return fail(USP_ERR_INVALID, "dtype");
  LAUNCHCHK("k_canonical_fields");
  return 0;
}

}  // extern "C"
