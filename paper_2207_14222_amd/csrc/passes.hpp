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
  double* row;  // per-block partial sums of this launch (NULL: none); a launch
                // in complex64 writes them as floats at the start of the row
};

template <class C> constexpr int x_threads() { return sizeof(C) == 8 ? 256 : 128; }

// copy a length-N twiddle table into LDS (whole block participates)
template <class C, int N>
__device__ __forceinline__ void load_twiddles(C* tws, const C* __restrict__ tw) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) tws[i] = tw[i];
  __syncthreads();
}

// |p|^2 on the FFT grid from frequency indices: p_k = 2 pi (k or k - n)/(n h),
// passed as per-axis scale (2 pi/(n h))^2.
template <class R> __device__ __forceinline__ R fsq(int k, int n) {
  const int f = (k < (n + 1) / 2) ? k : k - n;
  return (R)(f * f);
}

// streaming (non-temporal) global access for fields read or written once per
// pass, so that they do not evict the temporary spectrum from the caches
template <class C> __device__ __forceinline__ C ld_stream(const C* p) {
  if constexpr (sizeof(C) == 8) {
    const double d = __builtin_nontemporal_load(reinterpret_cast<const double*>(p));
    C c;
    __builtin_memcpy(&c, &d, 8);
    return c;
  } else {
    typedef double d2v __attribute__((ext_vector_type(2)));
    const d2v d = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
    C c;
    __builtin_memcpy(&c, &d, 16);
    return c;
  }
}
template <class C> __device__ __forceinline__ void st_stream(C* p, C v) {
  if constexpr (sizeof(C) == 8) {
    double d;
    __builtin_memcpy(&d, &v, 8);
    __builtin_nontemporal_store(d, reinterpret_cast<double*>(p));
  } else {
    typedef double d2v __attribute__((ext_vector_type(2)));
    d2v d;
    __builtin_memcpy(&d, &v, 16);
    __builtin_nontemporal_store(d, reinterpret_cast<d2v*>(p));
  }
}
template <bool NT, class C> __device__ __forceinline__ C ld(const C* p) {
  if constexpr (NT) return ld_stream(p);
  else return *p;
}
template <bool NT, class C> __device__ __forceinline__ void st(C* p, C v) {
  if constexpr (NT) st_stream(p, v);
  else *p = v;
}

// Number of block barriers one FFT of plan P executes (two per LDS exchange);
// threads that sit out an FFT execute the same number so barriers match.
template <int N, class P> struct FftSyncs;
template <int N> struct FftSyncs<N, Plan<>> { static constexpr int value = 0; };
template <int N, int R0, int... Rest> struct FftSyncs<N, Plan<R0, Rest...>> {
  static constexpr int value = (sizeof...(Rest) > 0 ? 2 : 0) + FftSyncs<N, Plan<Rest...>>::value;
};
template <int N, class P> __device__ __forceinline__ void idle_fft_syncs() {
#pragma unroll
  for (int i = 0; i < FftSyncs<N, P>::value; ++i) __syncthreads();
}

// Contiguous-axis pass.  Cc: compute (and spectrum storage) type; Cx: storage
// type of x, y, B.  Body for LPB lines starting at line0 (TH = LPB*T
// threads take part; threads >= TH only join the block barriers (none when a
// line fits in one wave) and must form whole
// waves).  tws: twiddles in LDS; lds: LPB padded rows.  Returns the thread's
// partial sum of |Delta|^2 (X_FUSED, in the precision of Cc) or |r|^2 (X_RINV).
// FL (fused pass only): bit 0 = load x, B, y before the inverse FFT;
// bit 1 = stream x, B, y (non-temporal loads / store).
// TL (X_FIRST / X_FUSED): 0 = t row-major like x; TL > 0 = t in column tiles
// of width TL, element (line, pos) at ((pos / TL) nlines + line) TL + pos % TL,
// so that the strided pass reads each tile as one contiguous block.
template <class Cc, class Cx, int N, int MODE, int FL, int LPB, int TL = 0>
__device__ __forceinline__ typename real_of<Cc>::type xpass_body(Cc* __restrict__ t, Cx* __restrict__ x, const Cx* __restrict__ y,
                                             const Cx* __restrict__ B, const float2* __restrict__ d,
                                             float2* __restrict__ r32, const Cc* tws, Cc* lds, double alpha,
                                             long line0, long nlines, int has_x) {
  using Rr = typename real_of<Cc>::type;
  using PP = PassPlan<N>;
  constexpr int E = PP::E, T = N / E;
  constexpr int TH = LPB * T;
  constexpr int PADN = LdsRow<Cc>::padded(N);
  // lines of at most 64 threads never straddle a wave: their exchanges need
  // no block barrier, and waves of one block run their FFTs independently
  constexpr bool WL = line_in_wave<T>();
  using Sync = LineSync<T>;
  const int tid = threadIdx.x;
  if (tid >= TH) {
    if (WL) return Rr(0);
    if (MODE == X_FUSED) {
      idle_fft_syncs<N, typename PP::P>();
      idle_fft_syncs<N, typename PP::P>();
    } else {
      idle_fft_syncs<N, typename PP::P>();
    }
    return Rr(0);
  }
  const int tt = tid % T, li = tid / T;
  const long line = line0 + li;
  const bool active = line < nlines;
  const long base = line * N;
  LdsRow<Cc> row{lds + li * PADN};
  Cc v[E];
  Rr acc = Rr(0);
  auto tix = [&](int pos) -> long {
    return TL ? ((long)(pos / TL) * nlines + line) * TL + pos % TL : base + pos;
  };

  if (MODE == X_FIRST) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const long p = base + tt + T * e;
      Cc val = mk<Cc>(0.0, 0.0);
      if (active) {
        val = cvt<Cc>(y[p]);
        if (has_x == 1) val = cadd(val, cmul(cvt<Cc>(B[p]), cvt<Cc>(x[p])));
        if (has_x == 2) x[p] = cvt<Cx>(mk<Cc>(0.0, 0.0));  // start of an inner solve: x = 0
      }
      v[e] = val;
    }
    FftRun<Cc, N, E, -1, 1, typename PP::P>::run(v, tt, row, tws, Sync{});
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) t[tix(tt + T * e)] = v[e];
    }
    return Rr(0);
  }

  if (MODE == X_FUSED) {
    // PF: x, B, y are loaded before the inverse FFT so their latency overlaps
    // it (more registers live across the FFT); otherwise after it.
    constexpr bool PF = (FL & 1) != 0, NT = (FL & 2) != 0;
    Cc xx[E], bb[E], yy[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const long p = base + tt + T * e;
      v[e] = active ? t[tix(tt + T * e)] : mk<Cc>(0.0, 0.0);
      if (PF) {
        xx[e] = active ? cvt<Cc>(ld<NT>(x + p)) : mk<Cc>(0.0, 0.0);
        bb[e] = active ? cvt<Cc>(ld<NT>(B + p)) : mk<Cc>(0.0, 0.0);
        yy[e] = active ? cvt<Cc>(ld<NT>(y + p)) : mk<Cc>(0.0, 0.0);
      }
    }
    FftRun<Cc, N, E, +1, 1, typename PP::P>::run(v, tt, row, tws, Sync{});
    if (!PF) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const long p = base + tt + T * e;
        xx[e] = active ? cvt<Cc>(ld<NT>(x + p)) : mk<Cc>(0.0, 0.0);
        bb[e] = active ? cvt<Cc>(ld<NT>(B + p)) : mk<Cc>(0.0, 0.0);
        yy[e] = active ? cvt<Cc>(ld<NT>(y + p)) : mk<Cc>(0.0, 0.0);
      }
    }
    const Rr a = (Rr)alpha;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const Cc dl = cmul(bb[e], csub(v[e], xx[e]));     // Delta = B (u - x)
      const Cc xn = cadd(xx[e], cscale(dl, a));         // x + alpha Delta
      acc += cnorm2(dl);
      if (active) st<NT>(x + base + tt + T * e, cvt<Cx>(xn));
      v[e] = cadd(cmul(bb[e], xn), yy[e]);              // next t = B x + y
    }
    FftRun<Cc, N, E, -1, 1, typename PP::P>::run(v, tt, row, tws, Sync{});
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) t[tix(tt + T * e)] = v[e];
    }
    return acc;
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
    FftRun<Cc, N, E, -1, 1, typename PP::P>::run(v, tt, row, tws, Sync{});
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) t[base + tt + T * e] = v[e];
    }
    return Rr(0);
  }

  // X_RINV.  FL bit 0: x, B, y loaded before the inverse FFT (their latency
  // overlaps it); bit 1: non-temporal loads.
  {
    constexpr bool PF = (FL & 1) != 0, NT = (FL & 2) != 0;
    Cc xx[E], bb[E], yy[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const long p = base + tt + T * e;
      v[e] = active ? t[p] : mk<Cc>(0.0, 0.0);
      if (PF) {
        xx[e] = active ? cvt<Cc>(ld<NT>(x + p)) : mk<Cc>(0.0, 0.0);
        bb[e] = active ? cvt<Cc>(ld<NT>(B + p)) : mk<Cc>(0.0, 0.0);
        yy[e] = active ? cvt<Cc>(ld<NT>(y + p)) : mk<Cc>(0.0, 0.0);
      }
    }
    FftRun<Cc, N, E, +1, 1, typename PP::P>::run(v, tt, row, tws, Sync{});
    if (!PF) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const long p = base + tt + T * e;
        xx[e] = active ? cvt<Cc>(ld<NT>(x + p)) : mk<Cc>(0.0, 0.0);
        bb[e] = active ? cvt<Cc>(ld<NT>(B + p)) : mk<Cc>(0.0, 0.0);
        yy[e] = active ? cvt<Cc>(ld<NT>(y + p)) : mk<Cc>(0.0, 0.0);
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      // r = y - L x - (1 - B) x, rounded in a fixed sequence (explicit fused
      // multiply-adds) so that every load plan gives the same bits
      Cc r;
      r.x = fma(bb[e].x, xx[e].x, fma(-bb[e].y, xx[e].y, (yy[e].x - v[e].x) - xx[e].x));
      r.y = fma(bb[e].x, xx[e].y, fma(bb[e].y, xx[e].x, (yy[e].y - v[e].y) - xx[e].y));
      acc += cnorm2(r);
      if (active && r32) r32[base + tt + T * e] = cvt<float2>(r);
    }
  }
  return acc;
}

template <class Cc, class Cx, int N, int MODE, int FL = 0>
__global__ void __launch_bounds__(x_threads<Cc>())
k_xpass(Cc* __restrict__ t, Cx* __restrict__ x, const Cx* __restrict__ y, const Cx* __restrict__ B,
        const float2* __restrict__ d, float2* __restrict__ r32, const Cc* __restrict__ tw, double alpha,
        int nlines, int has_x, RedArgs red) {
  constexpr int T = N / PassPlan<N>::E;
  constexpr int LPB = (x_threads<Cc>() / T) > 0 ? (x_threads<Cc>() / T) : 1;
  __shared__ Cc lds[LPB * LdsRow<Cc>::padded(N)];
  using Rr = typename real_of<Cc>::type;
  __shared__ Cc tws[N];
  __shared__ Rr scratch[64];
  load_twiddles<Cc, N>(tws, tw);
  const Rr acc = xpass_body<Cc, Cx, N, MODE, FL, LPB>(t, x, y, B, d, r32, tws, lds, alpha,
                                                     (long)blockIdx.x * LPB, nlines, has_x);
  if (MODE == X_FUSED || MODE == X_RINV) block_partial(acc, scratch, reinterpret_cast<Rr*>(red.row));
}

// Strided-axis pass over a tile of W adjacent columns.  Element (pos, col, b)
// lives at b*N*S + pos*S + col.  blockIdx.x: column tile, blockIdx.y: batch.
struct SymArgs {
  double sa, sm, sx;          // (2 pi/(n h))^2 of the transformed axis, n1 (0 in 2-D), n2
  int n1, log2_n2;            // n1 = 1 in 2-D
  double c0r, c0i, c2r, c2i;  // multiplier base: c0 + c2 |p|^2
  double scale;               // 1/Ntotal
};

// a column-tile width W is usable for length N if the tile and the twiddles fit
// in LDS and the block has at most 1024 threads
template <class C> constexpr bool s_width_ok(int N, int W, int E) {
  return (N * (W + 1) + N) * (int)sizeof(C) <= 160 * 1024 && W * (N / E) <= 1024;
}

// Body of the strided pass for columns col0 .. col0 + W - 1 of batch b.
// Threads >= W*T only join the barriers (whole waves, or no barriers at all
// for single-stage plans).  If tw_g is non-NULL the twiddles are copied into
// tws after the column loads are issued.  TILED: data in column tiles of
// width W (the TL layout of xpass_body with N lines, b = 0): the tile is the
// contiguous block of N W values at col0 N, and S is ignored.
template <class C, int N, int W, int MODE, bool TILED = false>
__device__ __forceinline__ void spass_body(C* __restrict__ data, const C* __restrict__ tw_g, C* tws, C* lds, long S,
                                           const SymArgs& sym, long col0, long b) {
  using Rr = typename real_of<C>::type;
  using PP = PassPlan<N>;
  constexpr int E = PP::E, T = N / E;
  const int tid = threadIdx.x;
  if (tid >= W * T) {
    if (tw_g) load_twiddles<C, N>(tws, tw_g);
    idle_fft_syncs<N, typename PP::P>();
    if (MODE == S_SYM || MODE == S_SYMA) idle_fft_syncs<N, typename PP::P>();
    return;
  }
  const int c = tid % W, tt = tid / W;
  const long col = col0 + c;
  if (TILED) S = W;
  const long base = TILED ? col0 * N + c : b * N * S + col;
  // the padded column's split of positions holds for this plan only
  static_assert(!TILED || std::is_same<typename PP::P, Plan<16, 16, 4>>::value, "tiled column plan");
  using Line = typename std::conditional<TILED, LdsColP<C, W>, LdsCol<C, W>>::type;
  Line line{lds + c};
  C v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = data[base + (long)(tt + T * e) * S];
  if (tw_g) load_twiddles<C, N>(tws, tw_g);

  if (MODE == S_INV) {
    FftRun<C, N, E, +1, 1, typename PP::P>::run(v, tt, line, tws, BlockSync{});
  } else {
    FftRun<C, N, E, -1, 1, typename PP::P>::run(v, tt, line, tws, BlockSync{});
  }
  if (MODE == S_SYM || MODE == S_SYMA) {
    const int n2 = 1 << sym.log2_n2;
    const int cl = (int)col;
    const Rr qc = (Rr)sym.sm * fsq<Rr>(cl >> sym.log2_n2, sym.n1) + (Rr)sym.sx * fsq<Rr>(cl & (n2 - 1), n2);
    const Rr sa = (Rr)sym.sa;
    // the 1/Ntotal of the inverse transform is a power of two, so it is folded
    // exactly into the coefficients: scale / m = 1 / (m / scale), m scale
    const double k = MODE == S_SYM ? 1.0 / sym.scale : sym.scale;
    const Rr c0r = (Rr)(sym.c0r * k), c0i = (Rr)(sym.c0i * k), c2r = (Rr)(sym.c2r * k), c2i = (Rr)(sym.c2i * k);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const Rr p2 = sa * fsq<Rr>(tt + T * e, N) + qc;
      C m;
      m.x = c0r + c2r * p2;
      m.y = c0i + c2i * p2;
      if (MODE == S_SYM) m = crecip(m);
      v[e] = cmul(v[e], m);
    }
    FftRun<C, N, E, +1, 1, typename PP::P>::run(v, tt, line, tws, BlockSync{});
  }
#pragma unroll
  for (int e = 0; e < E; ++e) data[base + (long)(tt + T * e) * S] = v[e];
}

template <class C, int N, int W, int MODE>
__global__ void __launch_bounds__(W * (N / PassPlan<N>::E))
k_spass(C* __restrict__ data, const C* __restrict__ tw, long S, SymArgs sym) {
  __shared__ C lds[N * (W + 1)];
  __shared__ C tws[N];
  spass_body<C, N, W, MODE>(data, tw, tws, lds, S, sym, (long)blockIdx.x * W, (long)blockIdx.y);
}

}  // namespace usp
