// Single-workgroup solver for 1-D problems (N <= 1024): the whole of Algorithm 1
// (Sec. 2.1) -- iterations, residual checks and the stopping decision -- runs in
// one launch with the field held in registers and LDS.  It also carries the
// pantograph's non-diagonal V (Sec. 3.3): V = diag(v) + G with the dilation
// gather (G x)_j = g0_j x[gi_j] + g1_j x[gi_j + 1].
//
// Symbol: l(p) = c0 + c2 p^2 + c1 i p with p = pscale * (k or k - N); the
// first-derivative part i p is set to zero at the Nyquist index when nyq_zero.
#pragma once
#include "fft.hpp"

namespace usp {

struct Sym1D {
  double c0r, c0i, c1r, c1i, c2r, c2i;  // s*a0, s*a1, s*a2
  double pscale;                        // 2 pi / (N h)
  int nyq_zero;
};

struct Solve1DInfo {
  int iterations;
  int status;    // 0 converged, 1 maxit, 3 diverged, -5 NaN
  int n_true;
  int pad;
};

template <class C, int N>
__device__ __forceinline__ C sym1d_mult(const Sym1D& s, int k, bool inverse_of_l_plus_1) {
  using Rr = typename real_of<C>::type;
  const int kk = (k < N / 2) ? k : k - N;
  const double p = s.pscale * kk;
  const double pl = (s.nyq_zero && k == N / 2) ? 0.0 : p;
  // l(p) = c0 + c2 p^2 + c1 * i * p
  double lr = s.c0r + s.c2r * p * p - s.c1i * pl;
  double li = s.c0i + s.c2i * p * p + s.c1r * pl;
  C m;
  if (inverse_of_l_plus_1) {
    lr += 1.0;
    const double den = lr * lr + li * li;
    m.x = (Rr)(lr / den / N);
    m.y = (Rr)(-li / den / N);
  } else {
    m.x = (Rr)(lr / N);
    m.y = (Rr)(li / N);
  }
  return m;
}

template <class C, int N>
__global__ void __launch_bounds__(N / LinePlan<N>::E)
k_solve1d(C* __restrict__ x, const C* __restrict__ y, const C* __restrict__ B, const int* __restrict__ gi,
          const C* __restrict__ g0, const C* __restrict__ g1, const C* __restrict__ tw, Sym1D sym, double alpha,
          double tol, int maxit, int check_every, int x_is_guess, double* __restrict__ hist_pre,
          double* __restrict__ hist_true, int hist_cap, Solve1DInfo* __restrict__ info) {
  using Rr = typename real_of<C>::type;
  using LP = LinePlan<N>;
  constexpr int E = LP::E, T = N / E;
  __shared__ C lds[LdsRow<C>::padded(N)];
  __shared__ C xs[N];
  __shared__ double scratch[64];
  const int t = threadIdx.x;
  LdsRow<C> row{lds};
  const bool gather = (gi != nullptr);

  C xv[E], yv[E], bv[E], gsym[E], lsym[E];
  C h0[E], h1[E];
  int gidx[E];
  double yy = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = t + T * e;
    xv[e] = x_is_guess ? x[p] : mk<C>(0.0, 0.0);
    yv[e] = y[p];
    bv[e] = B[p];
    gsym[e] = sym1d_mult<C, N>(sym, p, true);
    lsym[e] = sym1d_mult<C, N>(sym, p, false);
    if (gather) {
      gidx[e] = min(max(gi[p], 0), N - 1);
      h0[e] = g0[p];
      h1[e] = g1[p];
    } else {
      gidx[e] = 0;
      h0[e] = h1[e] = mk<C>(0.0, 0.0);
    }
    yy += cabs2(yv[e]);
  }
  yy = block_sum(yy, scratch);

  // G applied to a field held in registers (through LDS)
  auto apply_gather = [&](const C (&f)[E], C (&out)[E]) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) xs[t + T * e] = f[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i0 = gidx[e];
      const int i1 = (i0 + 1 < N) ? i0 + 1 : N - 1;
      out[e] = cadd(cmul(h0[e], xs[i0]), cmul(h1[e], xs[i1]));
    }
  };

  int status = 1, it = 0, ntrue = 0, grow = 0;
  double d0 = -1.0, dprev = -1.0;
  const Rr a = (Rr)alpha;
  for (it = 0; it < maxit;) {
    C v[E], gx[E];
    // t = B x + y  (B x = diag(B) x - G x)
    if (gather) apply_gather(xv, gx);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      v[e] = cadd(cmul(bv[e], xv[e]), yv[e]);
      if (gather) v[e] = csub(v[e], gx[e]);
    }
    FftRun<C, N, E, -1, 1, typename LP::P>::run(v, t, row, tw, BlockSync{});
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cmul(v[e], gsym[e]);
    FftRun<C, N, E, +1, 1, typename LP::P>::run(v, t, row, tw, BlockSync{});
    // Delta = B (u - x)
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = csub(v[e], xv[e]);
    if (gather) apply_gather(v, gx);
    double dd = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      C dl = cmul(bv[e], v[e]);
      if (gather) dl = csub(dl, gx[e]);
      xv[e] = cadd(xv[e], cscale(dl, a));
      dd += cabs2(dl);
    }
    dd = block_sum(dd, scratch);
    if (t == 0 && it < hist_cap) hist_pre[it] = dd;
    ++it;
    // divergence: ||Delta|| grew three times in a row and exceeds its first value
    if (d0 < 0.0) d0 = dd;
    grow = (dprev >= 0.0 && dd > dprev) ? grow + 1 : 0;
    dprev = dd;
    if (!(dd == dd)) { status = -5; break; }
    if (grow >= 3 && dd > d0) { status = 3; break; }

    if (it % check_every == 0 || it == maxit) {
      // r = y - L x - (1 - B) x - G x
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = xv[e];
      FftRun<C, N, E, -1, 1, typename LP::P>::run(v, t, row, tw, BlockSync{});
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = cmul(v[e], lsym[e]);
      FftRun<C, N, E, +1, 1, typename LP::P>::run(v, t, row, tw, BlockSync{});
      if (gather) apply_gather(xv, gx);
      double rr = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        C r = cadd(csub(csub(yv[e], v[e]), xv[e]), cmul(bv[e], xv[e]));
        if (gather) r = csub(r, gx[e]);
        rr += cabs2(r);
      }
      rr = block_sum(rr, scratch);
      const double rho = sqrt(rr / yy);
      if (t == 0 && ntrue < hist_cap) {
        hist_true[2 * ntrue] = (double)it;
        hist_true[2 * ntrue + 1] = rho;
      }
      ++ntrue;
      if (!(rho == rho)) { status = -5; break; }
      if (rho < tol) { status = 0; break; }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) x[t + T * e] = xv[e];
  if (t == 0) {
    info->iterations = it;
    info->status = status;
    info->n_true = ntrue;
  }
}

}  // namespace usp
