// Single-workgroup solver for the antisymmetrised canonical form of a 1-D
// problem (Sec. 2.2, Eq. antisymmetrised), for systems that are not
// accretive.  From A~ = L~ + V~ (scale c real) the larger system on
// x = [x~; x~'] (2N unknowns, component-major) is
//     A = [[0, -A~*], [A~, 0]],  L = [[0, -L~*], [L~, 0]],  V = [[0, -V~*], [V~, 0]],
// skew-Hermitian with ||V|| = ||V~|| < 1, and Algorithm 1 runs on it:
//     B x + y = [x1 + V~* x2 + y1;  x2 - V~ x1 + y2],
//     (L + I)^-1 per Fourier mode = [[1, conj(l)], [-l, 1]] / (1 + |l|^2),
//     Delta = B (u - x).
// V~ = diag(1 - B~) + G with the dilation gather G; its adjoint
// V~* = diag(conj(1 - B~)) + G* uses a precomputed table of G* (row k lists
// the pairs (j, conj(g)) with G[j][k] = g; at most kAdjMax per row).
#pragma once
#include "solve1d.hpp"

namespace usp {

constexpr int kAdjMax = 8;

// l(p) of the 1-D symbol (no 1/N)
template <int N>
__device__ __forceinline__ void sym1d_l(const Sym1D& s, int k, double& lr, double& li) {
  const int kk = (k < N / 2) ? k : k - N;
  const double p = s.pscale * kk;
  const double pl = (s.nyq_zero && k == N / 2) ? 0.0 : p;
  lr = s.c0r + s.c2r * p * p - s.c1i * pl;
  li = s.c0i + s.c2i * p * p + s.c1r * pl;
}

// res_out != NULL: only ||y - A x||^2 and ||y||^2 -> res_out[0..1] (x read as given)
template <class C, int N>
__global__ void __launch_bounds__(N / LinePlan<N>::E)
k_solve1d_as(C* __restrict__ x, const C* __restrict__ y, const C* __restrict__ B, const int* __restrict__ gi,
             const C* __restrict__ g0, const C* __restrict__ g1, const int* __restrict__ aj,
             const C* __restrict__ aw, const C* __restrict__ tw, Sym1D sym, double alpha, double tol, int maxit,
             int check_every, int x_is_guess, double* __restrict__ hist_pre, double* __restrict__ hist_true,
             int hist_cap, Solve1DInfo* __restrict__ info, double* __restrict__ res_out) {
  using Rr = typename real_of<C>::type;
  using LP = LinePlan<N>;
  constexpr int E = LP::E, T = N / E;
  __shared__ C lds[LdsRow<C>::padded(N)];
  __shared__ C fs[N];
  __shared__ double scratch[64];
  const int t = threadIdx.x;
  LdsRow<C> row{lds};
  const bool gather = (gi != nullptr);

  C x1[E], x2[E];
  double yy = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = t + T * e;
    const bool g = x_is_guess || res_out;
    x1[e] = g ? x[p] : mk<C>(0.0, 0.0);
    x2[e] = g ? x[N + p] : mk<C>(0.0, 0.0);
    yy += cabs2(y[p]) + cabs2(y[N + p]);
  }
  yy = block_sum(yy, scratch);

  // out = V~ f = (1 - B) f + G f
  auto v_apply = [&](const C (&f)[E], C (&out)[E]) {
    if (gather) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E; ++e) fs[t + T * e] = f[e];
      __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = t + T * e;
      const C vb = csub(mk<C>(1.0, 0.0), B[p]);
      C o = cmul(vb, f[e]);
      if (gather) {
        const int i0 = min(max(gi[p], 0), N - 1);
        const int i1 = (i0 + 1 < N) ? i0 + 1 : N - 1;
        o = cadd(o, cadd(cmul(g0[p], fs[i0]), cmul(g1[p], fs[i1])));
      }
      out[e] = o;
    }
  };
  // out = V~* f = conj(1 - B) f + G* f
  auto vh_apply = [&](const C (&f)[E], C (&out)[E]) {
    if (gather) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < E; ++e) fs[t + T * e] = f[e];
      __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = t + T * e;
      const C vb = csub(mk<C>(1.0, 0.0), B[p]);
      C o = cmul(mk<C>(vb.x, -vb.y), f[e]);
      if (gather) {
#pragma unroll
        for (int a = 0; a < kAdjMax; ++a) {
          const int j = aj[p * kAdjMax + a];
          if (j >= 0) o = cadd(o, cmul(aw[p * kAdjMax + a], fs[j]));
        }
      }
      out[e] = o;
    }
  };
  // residual r = y - A x = [y1 + L~* x2 + V~* x2;  y2 - L~ x1 - V~ x1]; returns ||r||^2
  auto residual = [&]() -> double {
    C a[E], b[E], w1[E], w2[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      a[e] = x1[e];
      b[e] = x2[e];
    }
    FftRun<C, N, E, -1, 1, typename LP::P>::run(a, t, row, tw, BlockSync{});
    FftRun<C, N, E, -1, 1, typename LP::P>::run(b, t, row, tw, BlockSync{});
#pragma unroll
    for (int e = 0; e < E; ++e) {
      double lr, li;
      sym1d_l<N>(sym, t + T * e, lr, li);
      a[e] = cmul(a[e], mk<C>(lr / N, li / N));
      b[e] = cmul(b[e], mk<C>(lr / N, -li / N));
    }
    FftRun<C, N, E, +1, 1, typename LP::P>::run(a, t, row, tw, BlockSync{});
    FftRun<C, N, E, +1, 1, typename LP::P>::run(b, t, row, tw, BlockSync{});
    vh_apply(x2, w1);
    v_apply(x1, w2);
    double rr = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = t + T * e;
      const C r1 = cadd(cadd(y[p], b[e]), w1[e]);
      const C r2 = csub(csub(y[N + p], a[e]), w2[e]);
      rr += cabs2(r1) + cabs2(r2);
    }
    return block_sum(rr, scratch);
  };

  if (res_out) {
    const double rr = residual();
    if (t == 0) {
      res_out[0] = rr;
      res_out[1] = yy;
    }
    return;
  }

  int status = 1, it = 0, ntrue = 0, grow = 0;
  double d0 = -1.0, dprev = -1.0;
  const Rr al = (Rr)alpha;
  for (it = 0; it < maxit;) {
    C t1[E], t2[E], w1[E], w2[E];
    vh_apply(x2, w1);
    v_apply(x1, w2);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int p = t + T * e;
      t1[e] = cadd(cadd(x1[e], w1[e]), y[p]);
      t2[e] = cadd(csub(x2[e], w2[e]), y[N + p]);
    }
    FftRun<C, N, E, -1, 1, typename LP::P>::run(t1, t, row, tw, BlockSync{});
    FftRun<C, N, E, -1, 1, typename LP::P>::run(t2, t, row, tw, BlockSync{});
#pragma unroll
    for (int e = 0; e < E; ++e) {
      double lr, li;
      sym1d_l<N>(sym, t + T * e, lr, li);
      const double s = 1.0 / ((1.0 + lr * lr + li * li) * N);
      const C a = t1[e], b = t2[e];
      t1[e] = cscale(cadd(a, cmul(mk<C>(lr, -li), b)), (Rr)s);
      t2[e] = cscale(csub(b, cmul(mk<C>(lr, li), a)), (Rr)s);
    }
    FftRun<C, N, E, +1, 1, typename LP::P>::run(t1, t, row, tw, BlockSync{});
    FftRun<C, N, E, +1, 1, typename LP::P>::run(t2, t, row, tw, BlockSync{});
#pragma unroll
    for (int e = 0; e < E; ++e) {
      t1[e] = csub(t1[e], x1[e]);   // u1 - x1
      t2[e] = csub(t2[e], x2[e]);   // u2 - x2
    }
    vh_apply(t2, w1);
    v_apply(t1, w2);
    double dd = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const C d1 = cadd(t1[e], w1[e]);
      const C d2 = csub(t2[e], w2[e]);
      x1[e] = cadd(x1[e], cscale(d1, al));
      x2[e] = cadd(x2[e], cscale(d2, al));
      dd += cabs2(d1) + cabs2(d2);
    }
    dd = block_sum(dd, scratch);
    if (t == 0 && it < hist_cap) hist_pre[it] = dd;
    ++it;
    if (d0 < 0.0) d0 = dd;
    grow = (dprev >= 0.0 && dd > dprev) ? grow + 1 : 0;
    dprev = dd;
    if (!(dd == dd)) { status = -5; break; }
    if (grow >= 3 && dd > d0) { status = 3; break; }
    if (it % check_every == 0 || it == maxit) {
      const double rho = sqrt(residual() / yy);
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
  for (int e = 0; e < E; ++e) {
    x[t + T * e] = x1[e];
    x[N + t + T * e] = x2[e];
  }
  if (t == 0) {
    info->iterations = it;
    info->status = status;
    info->n_true = ntrue;
  }
}

}  // namespace usp
