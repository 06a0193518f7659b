// Pass kernels of one fixed-point iteration on a 2-D / 3-D periodic grid, and the
// FP64 true-residual passes.  Grid layout: C order [n0][n1][n2], n2 contiguous;
// 2-D problems use n1 = 1.
//
// One iteration of Algorithm 1 (Sec. 2.1),
//     Delta = B [ (L + I)^-1 (B x + y) - x ],   x <- x + alpha Delta,
// with (L + I)^-1 = F^-1 diag(1/(l(p) + 1)) F (Eq. laplacian_inverse), runs as
//   X (fused)  : inverse FFT along n2 of the previous spectrum -> u, Delta, update x,
//                ||Delta||^2, then t = B x + y and its forward FFT along n2
//   M fwd      : forward FFT along n1 (3-D only)
//   S (symbol) : forward FFT along n0, multiply by 1/(N (l(p) + 1)), inverse FFT along n0
//   M inv      : inverse FFT along n1 (3-D only)
// so each iteration streams x, y, B once, reads+writes x once and t (the single
// temporary vector) three times (3-D).
//
// The true residual r = y - A x = y - L x - (1 - B) x (Sec. 2.2 canonical form)
// is evaluated in FP64 by the same pass structure with the spectral multiplier
// l(p)/N: X_RFWD (x -> FFT along n2, FP64), M fwd/inv (FP64), S_SYMA (FP64),
// X_RINV (inverse FFT along n2, r, ||r||^2, optional complex64 copy of r).
#pragma once
#include "fft.hpp"

namespace usp {

enum XMode { X_FIRST = 0, X_FUSED = 1, X_RFWD = 2, X_RINV = 3 };
enum SMode { S_FWD = 0, S_INV = 1, S_SYM = 2, S_SYMA = 3 };

struct RedArgs {
  double* row;  // per-block partial sums of this launch (NULL: none)
};

template <class C> constexpr int x_threads() { return sizeof(C) == 8 ? 256 : 128; }

// Contiguous-axis pass.  Cc: compute (and spectrum storage) type; Cx: storage
// type of x, y, B.
template <class Cc, class Cx, int N, int MODE>
__global__ void __launch_bounds__(x_threads<Cc>())
k_xpass(Cc* __restrict__ t, Cx* __restrict__ x, const Cx* __restrict__ y, const Cx* __restrict__ B,
        const float2* __restrict__ d, float2* __restrict__ r32, const Cc* __restrict__ tw, double alpha,
        int nlines, int has_x, RedArgs red) {
  using Rr = typename real_of<Cc>::type;
  using PP = PassPlan<N>;
  constexpr int E = PP::E, T = N / E;
  constexpr int TPB = x_threads<Cc>();
  constexpr int LPB = (TPB / T) > 0 ? (TPB / T) : 1;
  constexpr int PADN = LdsRow<Cc>::padded(N);
  __shared__ Cc lds[LPB * PADN];
  __shared__ double scratch[64];

  const int tid = threadIdx.x;
  const int tt = tid % T, li = tid / T;
  const long line = (long)blockIdx.x * LPB + li;
  const bool active = (li < LPB) && (line < nlines);
  const long base = line * N;
  LdsRow<Cc> row{lds + (li < LPB ? li : 0) * PADN};
  Cc v[E];
  double acc = 0.0;

  if (MODE == X_FIRST) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const long p = base + tt + T * e;
      Cc val = mk<Cc>(0.0, 0.0);
      if (active) {
        val = cvt<Cc>(y[p]);
        if (has_x) val = cadd(val, cmul(cvt<Cc>(B[p]), cvt<Cc>(x[p])));
      }
      v[e] = val;
    }
    FftRun<Cc, N, E, -1, 1, typename PP::P>::run(v, tt, row, tw, BlockSync{});
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) t[base + tt + T * e] = v[e];
    }
    return;
  }

  if (MODE == X_FUSED || MODE == X_RINV) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = active ? t[base + tt + T * e] : mk<Cc>(0.0, 0.0);
    FftRun<Cc, N, E, +1, 1, typename PP::P>::run(v, tt, row, tw, BlockSync{});
  }

  if (MODE == X_FUSED) {
    const Rr a = (Rr)alpha;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (active) {
        const long p = base + tt + T * e;
        const Cc xx = cvt<Cc>(x[p]);
        const Cc bb = cvt<Cc>(B[p]);
        const Cc yy = cvt<Cc>(y[p]);
        const Cc dl = cmul(bb, csub(v[e], xx));     // Delta = B (u - x)
        const Cc xn = cadd(xx, cscale(dl, a));      // x + alpha Delta
        acc += cabs2(dl);
        x[p] = cvt<Cx>(xn);
        v[e] = cadd(cmul(bb, xn), yy);              // next t = B x + y
      } else {
        v[e] = mk<Cc>(0.0, 0.0);
      }
    }
    FftRun<Cc, N, E, -1, 1, typename PP::P>::run(v, tt, row, tw, BlockSync{});
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) t[base + tt + T * e] = v[e];
    }
    block_partial(acc, scratch, red.row);
    return;
  }

  if (MODE == X_RFWD) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      Cc val = mk<Cc>(0.0, 0.0);
      if (active) {
        const long p = base + tt + T * e;
        val = cvt<Cc>(x[p]);
        if (d) {
          val = cadd(val, cvt<Cc>(d[p]));
          x[p] = cvt<Cx>(val);
        }
      }
      v[e] = val;
    }
    FftRun<Cc, N, E, -1, 1, typename PP::P>::run(v, tt, row, tw, BlockSync{});
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) t[base + tt + T * e] = v[e];
    }
    return;
  }

  if (MODE == X_RINV) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (active) {
        const long p = base + tt + T * e;
        const Cc xx = cvt<Cc>(x[p]);
        const Cc bb = cvt<Cc>(B[p]);
        const Cc yy = cvt<Cc>(y[p]);
        // r = y - L x - (1 - B) x
        const Cc r = cadd(csub(csub(yy, v[e]), xx), cmul(bb, xx));
        acc += cabs2(r);
        if (r32) r32[p] = cvt<float2>(r);
      }
    }
    block_partial(acc, scratch, red.row);
    return;
  }
}

// Strided-axis pass over a tile of W adjacent columns.  Element (pos, col, b)
// lives at b*N*S + pos*S + col.  blockIdx.x: column tile, blockIdx.y: batch.
struct SymArgs {
  const double* qa;  // (p_axis)^2 along the transformed axis, N entries
  const double* qm;  // (p)^2 along n1 (3-D) or a single 0 (2-D)
  const double* qx;  // (p)^2 along n2
  int log2_n2;
  double c0r, c0i, c2r, c2i;  // multiplier base: c0 + c2 |p|^2
  double scale;               // 1/Ntotal
};

template <class C> constexpr int s_lds_ok(int N, int W) { return N * (W + 1) * (int)sizeof(C) <= 150 * 1024; }

template <class C, int N, int W, int MODE>
__global__ void __launch_bounds__(W * (N / PassPlan<N>::E))
k_spass(C* __restrict__ data, const C* __restrict__ tw, long S, SymArgs sym) {
  using Rr = typename real_of<C>::type;
  using PP = PassPlan<N>;
  constexpr int E = PP::E, T = N / E;
  __shared__ C lds[N * (W + 1)];
  const int tid = threadIdx.x;
  const int c = tid % W, tt = tid / W;
  const long col = (long)blockIdx.x * W + c;
  const long base = (long)blockIdx.y * N * S + col;
  LdsCol<C, W> line{lds + c};
  C v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = data[base + (long)(tt + T * e) * S];

  if (MODE == S_INV) {
    FftRun<C, N, E, +1, 1, typename PP::P>::run(v, tt, line, tw, BlockSync{});
  } else {
    FftRun<C, N, E, -1, 1, typename PP::P>::run(v, tt, line, tw, BlockSync{});
  }
  if (MODE == S_SYM || MODE == S_SYMA) {
    const long n2m = (1L << sym.log2_n2) - 1;
    const double qc = sym.qm[col >> sym.log2_n2] + sym.qx[col & n2m];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const Rr p2 = (Rr)(sym.qa[tt + T * e] + qc);
      C m;
      m.x = (Rr)sym.c0r + (Rr)sym.c2r * p2;
      m.y = (Rr)sym.c0i + (Rr)sym.c2i * p2;
      if (MODE == S_SYM) m = crecip(m);
      v[e] = cmul(v[e], cscale(m, (Rr)sym.scale));
    }
    FftRun<C, N, E, +1, 1, typename PP::P>::run(v, tt, line, tw, BlockSync{});
  }
#pragma unroll
  for (int e = 0; e < E; ++e) data[base + (long)(tt + T * e) * S] = v[e];
}

}  // namespace usp
