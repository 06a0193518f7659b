// Kernels of steady diffusion in flux form with a tensor coefficient
// (Sec. 3.2, Eq. diffusion-equation-matrix-form) on a periodic 2-D or 3-D
// grid with D = 2 or 3 flux components.  The unknown x = [u; J_1 .. J_D] is
// stored component-major, D + 1 planes of the grid (last axis contiguous);
// flux component k pairs with axis D - k (J_1 = J_x with the contiguous
// axis).  Per voxel B = I - V is block diagonal: b_u and the D x D block b2
// acting on the flux components.  L's symbol is a (D + 1) x (D + 1) block per
// Fourier mode; with M = I + S L~(p) S / c,
//     M = [[A, i b^T], [i b, E]],   b_k = q_k p_(axis D - k),
// A = 1 + s0^2 mubar / c, E = I + S' Dibar S' / c (constant), and its inverse
// by the Schur complement s = A + b^T E^-1 b:
//     out_0 = (z_0 - i h^T z') / s,   out' = E^-1 z' - i g out_0,
// g = E^-1 b, h = E^-T b (E^-1 precomputed on the host).
//
// One iteration of Algorithm 1:
//   2-D: k_fx_col (axis 0 with the block), k_fx_row (axis 1, update);
//   3-D: strided FFT along axis 1 of all planes (k_spass), k_fx_col (axis 0
//        with the block), inverse strided FFT along axis 1, k_fx_row (axis 2).
//   k_fx_row: the planes' lines of a grid row in one block: inverse FFT -> u,
//        Delta = B (u - x) (flux planes exchanged through LDS), x += alpha
//        Delta, ||Delta||^2 partial, next t = B x + y, forward FFT.
//   k_fx_col: column tiles of every plane: forward FFT along axis 0, the
//        per-mode block applied across the planes in LDS (each thread takes
//        whole modes), inverse FFT.
// The FP64 residual uses the same kernels: k_fx_row (RFWD) transforms x, the
// middle passes and k_fx_col apply L / N, k_fx_row (RINV) forms
// y - L x - (x - B x).
#pragma once
#include <type_traits>

#include "passes.hpp"

namespace usp {

struct FluxSym {
  double A[2];
  double E[9][2];        // D x D row-major
  double Einv[9][2];
  double q[3];           // q_k = s0 s_k / c
  double pscale[3];      // 2 pi / (n h) per axis
  int n[3];              // grid sides (n[2] = 1 in 2-D)
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

// Column kernel geometry for NP planes and W columns per block (the host
// launches W = 2, or 1 where the tiles exceed LDS); 4 elements per thread when NP W N/4
// threads fit a block, else 8; twiddles in LDS when they fit beside the tiles.
template <class C, int N, int NP, int W_> struct FxCol {
  static constexpr int W = W_;
  static constexpr int tile_bytes = NP * N * (W + 1) * (int)sizeof(C);
  static constexpr bool LINE = NP * W * (N / 4) <= 1024;
  static constexpr int E = LINE ? 4 : 8, T = N / E;
  using P = typename std::conditional<LINE, typename LinePlan<N>::P, typename FxColPlan<N>::P>::type;
  static constexpr int THREADS = NP * W * T;
  static constexpr bool VALID = tile_bytes <= 160 * 1024 && THREADS <= 1024 && W * (int)sizeof(C) <= 128 && W <= N;
  static constexpr bool TWL = tile_bytes + N * (int)sizeof(C) <= 160 * 1024;
};

// z <- M(p)^-1 z (INV) or (M(p) - I) z, times sc, for one mode's D + 1 plane
// values (FP64); b the real vector of the mode's scaled wavenumbers
template <int D, bool INV>
__device__ __forceinline__ void fx_apply_block(const FluxSym& fs, const double (&b)[D], double sc,
                                               double (&z)[D + 1][2]) {
  auto cm = [](double ar, double ai, double br, double bi, double& or_, double& oi) {
    or_ = ar * br - ai * bi;
    oi = ar * bi + ai * br;
  };
  double o[D + 1][2];
  if (!INV) {
    // row 0: (A - 1) z0 + i b^T z';  row k: i b_k z0 + ((E - I) z')_k
    double r0 = (fs.A[0] - 1.0) * z[0][0] - fs.A[1] * z[0][1];
    double i0 = (fs.A[0] - 1.0) * z[0][1] + fs.A[1] * z[0][0];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      r0 -= b[k] * z[1 + k][1];
      i0 += b[k] * z[1 + k][0];
    }
    o[0][0] = r0;
    o[0][1] = i0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double rr = -b[k] * z[0][1], ii = b[k] * z[0][0];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double er = fs.E[k * D + j][0] - (k == j ? 1.0 : 0.0), ei = fs.E[k * D + j][1];
        double pr, pi;
        cm(er, ei, z[1 + j][0], z[1 + j][1], pr, pi);
        rr += pr;
        ii += pi;
      }
      o[1 + k][0] = rr;
      o[1 + k][1] = ii;
    }
  } else {
    double g[D][2], h[D][2];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      g[k][0] = g[k][1] = h[k][0] = h[k][1] = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        g[k][0] += fs.Einv[k * D + j][0] * b[j];
        g[k][1] += fs.Einv[k * D + j][1] * b[j];
        h[k][0] += fs.Einv[j * D + k][0] * b[j];
        h[k][1] += fs.Einv[j * D + k][1] * b[j];
      }
    }
    double sr = fs.A[0], si = fs.A[1];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      sr += b[k] * g[k][0];
      si += b[k] * g[k][1];
    }
    // out_0 = (z0 - i h^T z') / s
    double nr = z[0][0], ni = z[0][1];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double pr, pi;
      cm(h[k][0], h[k][1], z[1 + k][0], z[1 + k][1], pr, pi);
      nr += pi;   // - i (pr + i pi) = pi - i pr
      ni -= pr;
    }
    const double dd = sr * sr + si * si;
    const double o0r = (nr * sr + ni * si) / dd, o0i = (ni * sr - nr * si) / dd;
    o[0][0] = o0r;
    o[0][1] = o0i;
    // out' = E^-1 z' - i g out_0
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double rr = 0.0, ii = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        double pr, pi;
        cm(fs.Einv[k * D + j][0], fs.Einv[k * D + j][1], z[1 + j][0], z[1 + j][1], pr, pi);
        rr += pr;
        ii += pi;
      }
      double gr, gi;
      cm(g[k][0], g[k][1], o0r, o0i, gr, gi);
      o[1 + k][0] = rr + gi;   // - i (gr + i gi) = gi - i gr
      o[1 + k][1] = ii - gr;
    }
  }
#pragma unroll
  for (int k = 0; k <= D; ++k) {
    z[k][0] = o[k][0] * sc;
    z[k][1] = o[k][1] * sc;
  }
}

// spectral-derivative wavenumber of frequency index k on an n-point axis (Nyquist zero)
__device__ __forceinline__ double fx_wavenumber(int k, int n, double scale) {
  if ((n % 2) == 0 && k == n / 2) return 0.0;
  return scale * (double)(k < (n + 1) / 2 ? k : k - n);
}

// Axis-0 pass over W columns of the D + 1 planes: forward FFT, the per-mode
// block ((L + I)^-1 if INV, else L) times 1/n_total, inverse FFT.  Plane k,
// position p, column col (an index over the other axes, the last one
// fastest) lives at data[k n + p ncols + col]; the grid has ncols / W blocks
// of FxCol::THREADS threads (FxCol::VALID).
template <class C, int N, int D, int W_, bool INV>
__global__ void __launch_bounds__((FxCol<C, N, D + 1, W_>::THREADS))
k_fx_col(C* __restrict__ data, const C* __restrict__ tw, FluxSym fs) {
  using G = FxCol<C, N, D + 1, W_>;
  constexpr int W = G::W, E = G::E, T = G::T, NP = D + 1;
  __shared__ C tiles[NP * N * (W + 1)];
  __shared__ C tws[G::TWL ? N : 1];
  const C* twp = tw;
  if (G::TWL) {
    load_twiddles<C, N>(tws, tw);
    twp = tws;
  }
  const int tid = threadIdx.x;
  const int k = tid / (W * T), g = tid % (W * T), c = g % W, tt = g / W;
  const long ncols = (long)fs.n[1] * fs.n[2], n = (long)N * ncols;
  // consecutive column tiles on one XCD (blocks are dealt to the 8 XCDs in
  // turn), so that the row segments they share meet in that XCD's L2
  const int nb = gridDim.x, bb = blockIdx.x;
  const long bcol = (nb % 8 == 0) ? (long)(bb % 8) * (nb / 8) + bb / 8 : bb;
  const long col = bcol * W + c;
  const long base = k * n + col;
  LdsCol<C, W> line{tiles + k * N * (W + 1) + c};
  C v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = data[base + (long)(tt + T * e) * ncols];
  FftRun<C, N, E, -1, 1, typename G::P>::run(v, tt, line, twp, BlockSync{});
  // every plane's spectrum into its tile; then the block's N W modes are
  // shared out over all threads, each mode's values updated in place
#pragma unroll
  for (int e = 0; e < E; ++e) line[tt + T * e] = v[e];
  __syncthreads();
  const double sc = 1.0 / ((double)n);
  for (int m = tid; m < N * W; m += G::THREADS) {
    const int p = m / W, cm = m % W;
    const long cc = bcol * W + cm;
    double bvec[D];
    if (D == 2) {
      bvec[0] = fs.q[0] * fx_wavenumber((int)cc, fs.n[1], fs.pscale[1]);
      bvec[D - 1] = fs.q[D - 1] * fx_wavenumber(p, N, fs.pscale[0]);
    } else {
      bvec[0] = fs.q[0] * fx_wavenumber((int)(cc % fs.n[2]), fs.n[2], fs.pscale[2]);
      bvec[1] = fs.q[1] * fx_wavenumber((int)(cc / fs.n[2]), fs.n[1], fs.pscale[1]);
      bvec[D - 1] = fs.q[D - 1] * fx_wavenumber(p, N, fs.pscale[0]);
    }
    C* q = tiles + p * (W + 1) + cm;
    double z[NP][2];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const C a = q[j * N * (W + 1)];
      z[j][0] = (double)a.x;
      z[j][1] = (double)a.y;
    }
    fx_apply_block<D, INV>(fs, bvec, sc, z);
#pragma unroll
    for (int j = 0; j < NP; ++j) q[j * N * (W + 1)] = mk<C>(z[j][0], z[j][1]);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = line[tt + T * e];
  __syncthreads();   // the inverse FFT's first stage rewrites the tile
  FftRun<C, N, E, +1, 1, typename G::P>::run(v, tt, line, twp, BlockSync{});
#pragma unroll
  for (int e = 0; e < E; ++e) data[base + (long)(tt + T * e) * ncols] = v[e];
}

// Pass along the contiguous axis over the D + 1 planes' lines of LPB grid
// rows (ceil(nrows / LPB) blocks of (D + 1) G threads; the plane index is
// threadIdx.x / G; row r starts at voxel r N).  Cc: compute and spectrum
// type; Cx: storage type of x, y, b_u, b2.
//   FX_FIRST  t = B x + y (x = 0 unless has_x), forward FFT -> spec
//   FX_FUSED  spec -> inverse FFT = u; Delta = B (u - x); x += alpha Delta;
//             ||Delta||^2 block partial -> row0; t = B x + y; forward FFT -> spec
//   FX_RFWD   spec = forward FFT of x; with dcor, x += dcor first (stored)
//   FX_RINV   spec (= L x) -> inverse FFT; r = y - L x - x + B x;
//             ||r||^2 -> row0, ||y||^2 -> row1 (block partials); with r32,
//             r rounded to complex64 is stored there
// Rows at or beyond nrows compute on zeros and store nothing, so every thread
// takes every barrier.
template <class Cc, class Cx, int N, int D, int MODE>
__global__ void __launch_bounds__((D + 1) * FxRow<N>::G)
k_fx_row(Cc* __restrict__ spec, Cx* __restrict__ x, const Cx* __restrict__ y, const Cx* __restrict__ bu,
         const Cx* __restrict__ b2, const Cc* __restrict__ tw, double alpha, long nrows, int has_x,
         double* __restrict__ row0, double* __restrict__ row1, const float2* __restrict__ dcor,
         float2* __restrict__ r32) {
  using Rr = typename real_of<Cc>::type;
  using FR = FxRow<N>;
  using P = typename FR::PL::P;
  constexpr int E = FR::E, T = FR::T, LPB = FR::LPB, G = FR::G, NP = D + 1;
  constexpr int PADN = LdsRow<Cc>::padded(N);
  __shared__ Cc rows[NP * LPB * PADN];
  __shared__ Cc tws[N];
  __shared__ double scratch[64];
  load_twiddles<Cc, N>(tws, tw);
  const int tid = threadIdx.x;
  const int k = tid / G, g = tid % G, li = g / T, tt = g % T;
  const long r = (long)blockIdx.x * LPB + li;
  const bool act = r < nrows;
  const long n = nrows * N;
  const long vbase = r * N;              // voxel index of the row start
  const long base = k * n + vbase;       // plane k
  LdsRow<Cc> row{rows + (k * LPB + li) * PADN};
  // the flux planes' values of this thread's voxels through LDS (plane 0
  // takes part in the barriers only); the rows are free on entry and exit.
  // The FFTs of a line held by one wave synchronise that wave only: the
  // block barriers of the exchange order every use of a row by other waves
  auto exch = [&](const Cc (&mine)[E], Cc (&fl)[D][E]) {
#pragma unroll
    for (int e = 0; e < E; ++e) row[tt + T * e] = mine[e];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < D; ++j) {
      LdsRow<Cc> pr{rows + ((1 + j) * LPB + li) * PADN};
#pragma unroll
      for (int e = 0; e < E; ++e) fl[j][e] = pr[tt + T * e];
    }
    __syncthreads();
  };
  // row k of B at this thread's voxels: b_u for plane 0, row k - 1 of b2 else
  Cc bk[D][E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const long v = vbase + tt + T * e;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      Cc val = mk<Cc>(0.0, 0.0);
      if (act && MODE != FX_RFWD) {
        if (k == 0) {
          if (j == 0) val = cvt<Cc>(bu[v]);
        } else {
          val = cvt<Cc>(b2[(long)D * D * v + (k - 1) * D + j]);
        }
      }
      bk[j][e] = val;
    }
  }
  // (B z)_k from this plane's own values and the flux planes' values
  auto bapply = [&](int e, Cc own, const Cc (&fl)[D][E]) {
    if (k == 0) return cmul(bk[0][e], own);
    Cc acc = mk<Cc>(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < D; ++j) acc = cadd(acc, cmul(bk[j][e], fl[j][e]));
    return acc;
  };
  auto ld = [&](const Cx* src, int e) { return act ? cvt<Cc>(src[base + tt + T * e]) : mk<Cc>(0.0, 0.0); };

  Cc a[E];
  if (MODE == FX_FIRST) {
    Cc xv[E], fl[D][E];
#pragma unroll
    for (int e = 0; e < E; ++e) xv[e] = has_x ? ld(x, e) : mk<Cc>(0.0, 0.0);
    exch(xv, fl);
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = cadd(bapply(e, xv[e], fl), ld(y, e));
    FftRun<Cc, N, E, -1, 1, P>::run(a, tt, row, tws, LineSync<T>{});
    if (act) {
#pragma unroll
      for (int e = 0; e < E; ++e) spec[base + tt + T * e] = a[e];
    }
  } else if (MODE == FX_RFWD) {
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = ld(x, e);
    if (dcor && act) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        a[e] = cadd(a[e], cvt<Cc>(dcor[base + tt + T * e]));
        x[base + tt + T * e] = cvt<Cx>(a[e]);
      }
    }
    FftRun<Cc, N, E, -1, 1, P>::run(a, tt, row, tws, LineSync<T>{});
    if (act) {
#pragma unroll
      for (int e = 0; e < E; ++e) spec[base + tt + T * e] = a[e];
    }
  } else if (MODE == FX_FUSED) {
    Cc xv[E], yv[E], z[E], fl[D][E];
    const Rr al = (Rr)alpha;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      a[e] = act ? spec[base + tt + T * e] : mk<Cc>(0.0, 0.0);
      xv[e] = ld(x, e);
      yv[e] = ld(y, e);
    }
    FftRun<Cc, N, E, +1, 1, P>::run(a, tt, row, tws, LineSync<T>{});
#pragma unroll
    for (int e = 0; e < E; ++e) z[e] = csub(a[e], xv[e]);
    exch(z, fl);
    Rr acc = Rr(0);   // in the precision of the iteration
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const Cc dl = bapply(e, z[e], fl);
      xv[e] = cadd(xv[e], cscale(dl, al));
      acc += cnorm2(dl);
    }
    if (act) {
#pragma unroll
      for (int e = 0; e < E; ++e) x[base + tt + T * e] = cvt<Cx>(xv[e]);
    }
    exch(xv, fl);
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = cadd(bapply(e, xv[e], fl), yv[e]);
    FftRun<Cc, N, E, -1, 1, P>::run(a, tt, row, tws, LineSync<T>{});
    if (act) {
#pragma unroll
      for (int e = 0; e < E; ++e) spec[base + tt + T * e] = a[e];
    }
    // complex64: FP32 partials at the start of the row
    block_partial(acc, reinterpret_cast<Rr*>(scratch), reinterpret_cast<Rr*>(row0));
  } else {  // FX_RINV
    Cc xv[E], fl[D][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      a[e] = act ? spec[base + tt + T * e] : mk<Cc>(0.0, 0.0);
      xv[e] = ld(x, e);
    }
    FftRun<Cc, N, E, +1, 1, P>::run(a, tt, row, tws, LineSync<T>{});
    exch(xv, fl);
    double rr = 0.0, yy = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const Cc yv = ld(y, e);
      const Cc res = cadd(csub(csub(yv, a[e]), xv[e]), bapply(e, xv[e], fl));
      if (r32 && act) r32[base + tt + T * e] = cvt<float2>(res);
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

// complex128 -> complex64 copy (grid-stride)
template <int U = 0>
__global__ void __launch_bounds__(256) k_fx_to32(const double2* __restrict__ in, float2* __restrict__ out, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

// block i adds row (first + i) % ring of `part` (ncols partials of type R
// each, pitch elements of R apart) in a fixed order, in the precision of the
// partials, into out[(out_first + i) % out_ring]
template <class R>
__global__ void __launch_bounds__(256) k_fx_sum(const R* __restrict__ part, long pitch, int ncols, int first,
                                                int ring, double* __restrict__ out, int out_first, int out_ring) {
  __shared__ R scratch[64];
  const R* row = part + (long)((first + (int)blockIdx.x) % ring) * pitch;
  R acc = R(0);
  for (int i = threadIdx.x; i < ncols; i += blockDim.x) acc += row[i];
  const R s = block_sum(acc, scratch);
  if (threadIdx.x == 0) out[(out_first + (int)blockIdx.x) % out_ring] = s;
}

}  // namespace usp
