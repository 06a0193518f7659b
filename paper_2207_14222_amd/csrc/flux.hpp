// Kernels of steady diffusion in flux form with a tensor coefficient
// (Sec. 3.2, Eq. diffusion-equation-matrix-form) on a 2-D periodic grid.
// The unknown x = [u; Jx; Jy] is stored component-major, [3][n0][n1] (n1
// contiguous, the x axis).  Per voxel B = I - V is block diagonal: b_u and the
// 2 x 2 block [[b_xx, b_xy], [b_yx, b_yy]] acting on (Jx, Jy).  L's symbol is a
// 3 x 3 block per Fourier mode,
//     L(p) = S [[mubar, i p1, i p0], [i p1, Di_xx, Di_xy], [i p0, Di_yx, Di_yy]] S / c,
// (p the spectral-derivative wavenumbers, Nyquist mode zero; S = diag(s)).
//
// One iteration of Algorithm 1 is two launches:
//   k_fx_col (y axis)  column tiles of the three planes: forward FFT along n0,
//                      per mode the 3 x 3 block (L + I)^-1 / (n0 n1) applied
//                      across the planes (exchanged through LDS), inverse FFT;
//   k_fx_row (x axis)  the three planes' lines of a grid row in one block:
//                      inverse FFT along n1 -> u, Delta = B (u - x) (the 2 x 2
//                      flux block exchanged through LDS), x += alpha Delta,
//                      ||Delta||^2 partial, next t = B x + y, forward FFT.
// The FP64 residual uses the same two kernels: k_fx_row (RFWD) transforms x,
// k_fx_col applies L / (n0 n1), k_fx_row (RINV) forms y - L x - (x - B x).
#pragma once
#include <type_traits>

#include "passes.hpp"

namespace usp {

// Per-mode block M(p) = I + S L~(p) S / c written as
//     [[A, i b1, i b2], [i b1, E_xx, E_xy], [i b2, E_yx, E_yy]],
// b1 = q1 p1, b2 = q2 p0 (q1 = s0 s1 / c, q2 = s0 s2 / c), A = 1 + s0^2 mubar / c,
// E = I + S' Dibar S' / c; dE = E_xx E_yy - E_xy E_yx.
struct FluxSym {
  double A[2];
  double E[4][2];       // xx, xy, yx, yy
  double dE[2];
  double q1, q2;
  double pscale0, pscale1;  // 2 pi / (n h) per axis
  int n0, n1;
};

enum FxMode { FX_FIRST = 0, FX_FUSED = 1, FX_RFWD = 2, FX_RINV = 3 };

// Row kernel geometry: E = 4 elements per thread (T = N/4 threads per line),
// LPB rows per block so that each plane's thread group fills at least a wave.
template <int N> struct FxRow {
  using PL = LinePlan<N>;
  static constexpr int E = PL::E, T = N / E;
  static constexpr int LPB = (64 / T) > 1 ? 64 / T : 1;
  static constexpr int G = LPB * T;   // threads per plane
};

// Column kernel FFT plans with 8 elements per thread (long columns, where
// 4 per thread would need more than 1024 threads).
template <int N> struct FxColPlan;
template <> struct FxColPlan<8> { using P = Plan<8>; };
template <> struct FxColPlan<16> { using P = Plan<8, 2>; };
template <> struct FxColPlan<32> { using P = Plan<8, 4>; };
template <> struct FxColPlan<64> { using P = Plan<8, 8>; };
template <> struct FxColPlan<128> { using P = Plan<8, 8, 2>; };
template <> struct FxColPlan<256> { using P = Plan<8, 8, 4>; };
template <> struct FxColPlan<512> { using P = Plan<8, 8, 8>; };
template <> struct FxColPlan<1024> { using P = Plan<8, 8, 4, 4>; };

// Column kernel geometry: W = 2 columns of the 3 planes per block (more
// blocks in flight beat wider row segments at these sizes; measured), fewer
// where three [N][W+1] tiles exceed LDS; 4 elements per thread when 3 W N/4
// threads fit a block, else 8; twiddles in LDS when they fit beside the tiles.
template <class C, int N> struct FxCol {
  static constexpr int tile_bytes(int w) { return 3 * N * (w + 1) * (int)sizeof(C); }
  static constexpr int W = tile_bytes(2) <= 160 * 1024 ? 2 : 1;
  static constexpr bool LINE = 3 * W * (N / 4) <= 1024;
  static constexpr int E = LINE ? 4 : 8, T = N / E;
  using P = typename std::conditional<LINE, typename LinePlan<N>::P, typename FxColPlan<N>::P>::type;
  static constexpr int THREADS = 3 * W * T;
  static constexpr bool TWL = tile_bytes(W) + N * (int)sizeof(C) <= 160 * 1024;
};



// z <- M(p)^-1 z (INV, adjugate over the closed-form determinant) or
// (M(p) - I) z, times sc, for one mode's three plane values (FP64)
template <bool INV>
__device__ __forceinline__ void fx_apply_block(const FluxSym& fs, double p0, double p1, double sc, double (&z)[3][2]) {
  const double b1 = fs.q1 * p1, b2 = fs.q2 * p0;
  const double* A = fs.A;
  const double* Exx = fs.E[0];
  const double* Exy = fs.E[1];
  const double* Eyx = fs.E[2];
  const double* Eyy = fs.E[3];
  double m[3][3][2];   // the matrix applied (before the common factor)
  auto set = [&](int i, int j, double re, double im) {
    m[i][j][0] = re;
    m[i][j][1] = im;
  };
  double fr = sc, fi = 0.0;   // common factor
  if (!INV) {
    set(0, 0, A[0] - 1.0, A[1]);      set(0, 1, 0.0, b1);              set(0, 2, 0.0, b2);
    set(1, 0, 0.0, b1);               set(1, 1, Exx[0] - 1.0, Exx[1]); set(1, 2, Exy[0], Exy[1]);
    set(2, 0, 0.0, b2);               set(2, 1, Eyx[0], Eyx[1]);       set(2, 2, Eyy[0] - 1.0, Eyy[1]);
  } else {
    const double bb = b1 * b2, b11 = b1 * b1, b22 = b2 * b2;
    // det = A dE + b1^2 E_yy - b1 b2 (E_xy + E_yx) + b2^2 E_xx
    const double dr = A[0] * fs.dE[0] - A[1] * fs.dE[1] + b11 * Eyy[0] - bb * (Exy[0] + Eyx[0]) + b22 * Exx[0];
    const double di = A[0] * fs.dE[1] + A[1] * fs.dE[0] + b11 * Eyy[1] - bb * (Exy[1] + Eyx[1]) + b22 * Exx[1];
    const double dd = dr * dr + di * di;
    fr = sc * dr / dd;
    fi = -sc * di / dd;
    // adjugate (transposed cofactors) of [[A, i b1, i b2], [i b1, Exx, Exy], [i b2, Eyx, Eyy]]
    set(0, 0, fs.dE[0], fs.dE[1]);
    set(0, 1, b1 * Eyy[1] - b2 * Eyx[1], -(b1 * Eyy[0] - b2 * Eyx[0]));     // -i (b1 Eyy - b2 Eyx)
    set(0, 2, -(b1 * Exy[1] - b2 * Exx[1]), b1 * Exy[0] - b2 * Exx[0]);     //  i (b1 Exy - b2 Exx)
    set(1, 0, b1 * Eyy[1] - b2 * Exy[1], -(b1 * Eyy[0] - b2 * Exy[0]));     // -i (b1 Eyy - b2 Exy)
    set(1, 1, A[0] * Eyy[0] - A[1] * Eyy[1] + b22, A[0] * Eyy[1] + A[1] * Eyy[0]);
    set(1, 2, -(A[0] * Exy[0] - A[1] * Exy[1] + bb), -(A[0] * Exy[1] + A[1] * Exy[0]));
    set(2, 0, -(b1 * Eyx[1] - b2 * Exx[1]), b1 * Eyx[0] - b2 * Exx[0]);     //  i (b1 Eyx - b2 Exx)
    set(2, 1, -(A[0] * Eyx[0] - A[1] * Eyx[1] + bb), -(A[0] * Eyx[1] + A[1] * Eyx[0]));
    set(2, 2, A[0] * Exx[0] - A[1] * Exx[1] + b11, A[0] * Exx[1] + A[1] * Exx[0]);
  }
  double o[3][2];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      re += m[i][j][0] * z[j][0] - m[i][j][1] * z[j][1];
      im += m[i][j][0] * z[j][1] + m[i][j][1] * z[j][0];
    }
    o[i][0] = re * fr - im * fi;
    o[i][1] = re * fi + im * fr;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    z[i][0] = o[i][0];
    z[i][1] = o[i][1];
  }
}

// spectral-derivative wavenumber of frequency index k on an n-point axis (Nyquist zero)
__device__ __forceinline__ double fx_wavenumber(int k, int n, double scale) {
  if ((n % 2) == 0 && k == n / 2) return 0.0;
  return scale * (double)(k < (n + 1) / 2 ? k : k - n);
}

// y-axis pass over W columns of the three planes: forward FFT along n0, the
// per-mode 3 x 3 block ((L + I)^-1 if INV, else L) times 1/(n0 n1), inverse FFT.
// Plane k of column col, position p lives at data[k n + p n1 + col]; the grid
// has n1 / W blocks of FxCol::THREADS threads.
template <class C, int N, bool INV>
__global__ void __launch_bounds__((FxCol<C, N>::THREADS))
k_fx_col(C* __restrict__ data, const C* __restrict__ tw, FluxSym fs) {
  using G = FxCol<C, N>;
  constexpr int W = G::W, E = G::E, T = G::T;
  __shared__ C tiles[3 * N * (W + 1)];
  __shared__ C tws[G::TWL ? N : 1];
  const C* twp = tw;
  if (G::TWL) {
    load_twiddles<C, N>(tws, tw);
    twp = tws;
  }
  const int tid = threadIdx.x;
  const int k = tid / (W * T), g = tid % (W * T), c = g % W, tt = g / W;
  const long n1 = fs.n1, n = (long)N * n1;
  // consecutive column tiles on one XCD (blocks are dealt to the 8 XCDs in
  // turn), so that the row segments they share meet in that XCD's L2
  const int nb = gridDim.x, bb = blockIdx.x;
  const long bcol = (nb % 8 == 0) ? (long)(bb % 8) * (nb / 8) + bb / 8 : bb;
  const long col = bcol * W + c;
  const long base = k * n + col;
  LdsCol<C, W> line{tiles + k * N * (W + 1) + c};
  C v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = data[base + (long)(tt + T * e) * n1];
  FftRun<C, N, E, -1, 1, typename G::P>::run(v, tt, line, twp, BlockSync{});
  // every plane's spectrum into its tile; then the block's N W modes are
  // shared out over all threads, each mode's three values updated in place
#pragma unroll
  for (int e = 0; e < E; ++e) line[tt + T * e] = v[e];
  __syncthreads();
  const double sc = 1.0 / (double)n;
  for (int m = tid; m < N * W; m += G::THREADS) {
    const int p = m / W, cm = m % W;
    const double p0 = fx_wavenumber(p, N, fs.pscale0);
    const double p1 = fx_wavenumber((int)(bcol * W + cm), (int)n1, fs.pscale1);
    C* q = tiles + p * (W + 1) + cm;
    double z[3][2];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const C a = q[j * N * (W + 1)];
      z[j][0] = (double)a.x;
      z[j][1] = (double)a.y;
    }
    fx_apply_block<INV>(fs, p0, p1, sc, z);
#pragma unroll
    for (int j = 0; j < 3; ++j) q[j * N * (W + 1)] = mk<C>(z[j][0], z[j][1]);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = line[tt + T * e];
  __syncthreads();   // the inverse FFT's first stage rewrites the tile
  FftRun<C, N, E, +1, 1, typename G::P>::run(v, tt, line, twp, BlockSync{});
#pragma unroll
  for (int e = 0; e < E; ++e) data[base + (long)(tt + T * e) * n1] = v[e];
}

// x-axis pass over the three planes' lines of LPB grid rows (ceil(n0 / LPB)
// blocks of 3 G threads; the plane index is threadIdx.x / G).  Cc: compute and
// spectrum type; Cx: storage type of x, y, b_u, b2.
//   FX_FIRST  t = B x + y (x = 0 unless has_x), forward FFT -> spec
//   FX_FUSED  spec -> inverse FFT = u; Delta = B (u - x); x += alpha Delta;
//             ||Delta||^2 block partial -> row0; t = B x + y; forward FFT -> spec
//   FX_RFWD   spec = forward FFT of x
//   FX_RINV   spec (= L x along the rows) -> inverse FFT; r = y - L x - x + B x;
//             ||r||^2 -> row0, ||y||^2 -> row1 (block partials)
// Rows at or beyond n0 compute on zeros and store nothing, so every thread
// takes every barrier.
template <class Cc, class Cx, int N, int MODE>
__global__ void __launch_bounds__(3 * FxRow<N>::G)
k_fx_row(Cc* __restrict__ spec, Cx* __restrict__ x, const Cx* __restrict__ y, const Cx* __restrict__ bu,
         const Cx* __restrict__ b2, const Cc* __restrict__ tw, double alpha, int n0, int has_x,
         double* __restrict__ row0, double* __restrict__ row1) {
  using Rr = typename real_of<Cc>::type;
  using FR = FxRow<N>;
  using P = typename FR::PL::P;
  constexpr int E = FR::E, T = FR::T, LPB = FR::LPB, G = FR::G;
  constexpr int PADN = LdsRow<Cc>::padded(N);
  __shared__ Cc rows[3 * LPB * PADN];
  __shared__ Cc tws[N];
  __shared__ double scratch[64];
  load_twiddles<Cc, N>(tws, tw);
  const int tid = threadIdx.x;
  const int k = tid / G, g = tid % G, li = g / T, tt = g % T;
  const long r = (long)blockIdx.x * LPB + li;
  const bool act = r < n0;
  const long n = (long)n0 * N;
  const long vbase = r * N;              // voxel index of the row start
  const long base = k * n + vbase;       // plane k
  LdsRow<Cc> row{rows + (k * LPB + li) * PADN};
  LdsRow<Cc> prow{rows + (((3 - k) % 3) * LPB + li) * PADN};   // flux partner plane (k = 1, 2)
  // planes 1 and 2 swap values through LDS (plane 0 reads its own); the rows
  // are free on entry and again on exit
  auto exch = [&](const Cc (&mine)[E], Cc (&other)[E]) {
#pragma unroll
    for (int e = 0; e < E; ++e) row[tt + T * e] = mine[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) other[e] = prow[tt + T * e];
    __syncthreads();
  };
  // row k of B at this thread's voxels: own-plane and partner-plane entries
  Cc bk0[E], bk1[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const long v = vbase + tt + T * e;
    if (!act || MODE == FX_RFWD) {
      bk0[e] = mk<Cc>(0.0, 0.0);
      bk1[e] = mk<Cc>(0.0, 0.0);
    } else if (k == 0) {
      bk0[e] = cvt<Cc>(bu[v]);
      bk1[e] = mk<Cc>(0.0, 0.0);
    } else {
      bk0[e] = cvt<Cc>(b2[4 * v + 3 * (k - 1)]);       // b_xx (k = 1) or b_yy (k = 2)
      bk1[e] = cvt<Cc>(b2[4 * v + k]);                 // b_xy (k = 1) or b_yx (k = 2)
    }
  }
  auto bapply = [&](int e, Cc own, Cc partner) { return cadd(cmul(bk0[e], own), cmul(bk1[e], partner)); };

  Cc a[E];
  if (MODE == FX_FIRST) {
    Cc xv[E], xo[E];
#pragma unroll
    for (int e = 0; e < E; ++e) xv[e] = (act && has_x) ? cvt<Cc>(x[base + tt + T * e]) : mk<Cc>(0.0, 0.0);
    exch(xv, xo);
#pragma unroll
    for (int e = 0; e < E; ++e)
      a[e] = cadd(bapply(e, xv[e], xo[e]), act ? cvt<Cc>(y[base + tt + T * e]) : mk<Cc>(0.0, 0.0));
    FftRun<Cc, N, E, -1, 1, P>::run(a, tt, row, tws, BlockSync{});
    if (act) {
#pragma unroll
      for (int e = 0; e < E; ++e) spec[base + tt + T * e] = a[e];
    }
  } else if (MODE == FX_RFWD) {
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = act ? cvt<Cc>(x[base + tt + T * e]) : mk<Cc>(0.0, 0.0);
    FftRun<Cc, N, E, -1, 1, P>::run(a, tt, row, tws, BlockSync{});
    if (act) {
#pragma unroll
      for (int e = 0; e < E; ++e) spec[base + tt + T * e] = a[e];
    }
  } else if (MODE == FX_FUSED) {
    Cc xv[E], yv[E], z[E], zo[E];
    const Rr al = (Rr)alpha;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      a[e] = act ? spec[base + tt + T * e] : mk<Cc>(0.0, 0.0);
      xv[e] = act ? cvt<Cc>(x[base + tt + T * e]) : mk<Cc>(0.0, 0.0);
      yv[e] = act ? cvt<Cc>(y[base + tt + T * e]) : mk<Cc>(0.0, 0.0);
    }
    FftRun<Cc, N, E, +1, 1, P>::run(a, tt, row, tws, BlockSync{});
#pragma unroll
    for (int e = 0; e < E; ++e) z[e] = csub(a[e], xv[e]);
    exch(z, zo);
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const Cc dl = bapply(e, z[e], zo[e]);
      xv[e] = cadd(xv[e], cscale(dl, al));
      acc += cabs2(dl);
    }
    if (act) {
#pragma unroll
      for (int e = 0; e < E; ++e) x[base + tt + T * e] = cvt<Cx>(xv[e]);
    }
    exch(xv, zo);
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = cadd(bapply(e, xv[e], zo[e]), yv[e]);
    FftRun<Cc, N, E, -1, 1, P>::run(a, tt, row, tws, BlockSync{});
    if (act) {
#pragma unroll
      for (int e = 0; e < E; ++e) spec[base + tt + T * e] = a[e];
    }
    block_partial(acc, scratch, row0);
  } else {  // FX_RINV
    Cc xv[E], xo[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      a[e] = act ? spec[base + tt + T * e] : mk<Cc>(0.0, 0.0);
      xv[e] = act ? cvt<Cc>(x[base + tt + T * e]) : mk<Cc>(0.0, 0.0);
    }
    FftRun<Cc, N, E, +1, 1, P>::run(a, tt, row, tws, BlockSync{});
    exch(xv, xo);
    double rr = 0.0, yy = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const Cc yv = act ? cvt<Cc>(y[base + tt + T * e]) : mk<Cc>(0.0, 0.0);
      const Cc res = cadd(csub(csub(yv, a[e]), xv[e]), bapply(e, xv[e], xo[e]));
      rr += cabs2(res);
      yy += cabs2(yv);
    }
    rr = block_sum(rr, scratch);
    yy = block_sum(yy, scratch);
    if (threadIdx.x == 0) {
      row0[blockIdx.x] = rr;
      row1[blockIdx.x] = yy;
    }
  }
}

// block i adds row (first + i) % ring of `part` (ncols partials each, pitch
// apart) in a fixed order into out[(out_first + i) % out_ring]
template <int U = 0>
__global__ void __launch_bounds__(256) k_fx_sum(const double* __restrict__ part, long pitch, int ncols, int first,
                                                int ring, double* __restrict__ out, int out_first, int out_ring) {
  __shared__ double scratch[64];
  const double* row = part + (long)((first + (int)blockIdx.x) % ring) * pitch;
  double acc = 0.0;
  for (int i = threadIdx.x; i < ncols; i += blockDim.x) acc += row[i];
  const double s = block_sum(acc, scratch);
  if (threadIdx.x == 0) out[(out_first + (int)blockIdx.x) % out_ring] = s;
}

}  // namespace usp
