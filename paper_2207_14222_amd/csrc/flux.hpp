// Kernels of steady diffusion in flux form with a tensor coefficient
// (Sec. 3.2, Eq. diffusion-equation-matrix-form) on a 2-D periodic grid.
// The unknown x = [u; Jx; Jy] is stored component-major, [3][n0][n1] (n1
// contiguous, the x axis).  Per voxel B = I - V is block diagonal: b_u and the
// 2 x 2 block [[b_xx, b_xy], [b_yx, b_yy]] acting on (Jx, Jy).  L's symbol is a
// 3 x 3 block per Fourier mode,
//     L(p) = S [[mubar, i p1, i p0], [i p1, Di_xx, Di_xy], [i p0, Di_yx, Di_yy]] S / c,
// (p the spectral-derivative wavenumbers, Nyquist mode zero; S = diag(s)).
// One iteration of Algorithm 1: k_fx_update (Delta = B (u - x), update, and
// the next t = B x + y), k_xfft along n1 for the 3 n0 component lines, the
// strided FFT along n0 (k_spass, batch of 3 planes), k_fx_sym (per-mode
// (L + I)^-1 with the 1/N of the inverse transform), the inverse strided
// FFT and the inverse k_xfft.
#pragma once
#include "passes.hpp"

namespace usp {

struct FluxSym {
  double s[3];          // equilibration
  double c;             // overall scale
  double mubar[2];
  double dibar[4][2];   // Di_xx, Di_xy, Di_yx, Di_yy
  double pscale0, pscale1;  // 2 pi / (n h) per axis
  int n0, n1;
};

// pure FFT along the contiguous axis of `nlines` lines of length N, in place
template <class C, int N, int DIR>
__global__ void __launch_bounds__(x_threads<C>())
k_xfft(C* __restrict__ data, const C* __restrict__ tw, int nlines) {
  using PP = PassPlan<N>;
  constexpr int E = PP::E, T = N / E;
  constexpr int LPB = (x_threads<C>() / T) > 0 ? (x_threads<C>() / T) : 1;
  constexpr int TH = LPB * T;
  __shared__ C lds[LPB * LdsRow<C>::padded(N)];
  __shared__ C tws[N];
  load_twiddles<C, N>(tws, tw);
  const int tid = threadIdx.x;
  if (tid >= TH) {
    idle_fft_syncs<N, typename PP::P>();
    return;
  }
  const int tt = tid % T, li = tid / T;
  const long line = (long)blockIdx.x * LPB + li;
  const bool active = line < nlines;
  const long base = line * N;
  LdsRow<C> row{lds + li * LdsRow<C>::padded(N)};
  C a[E];
#pragma unroll
  for (int e = 0; e < E; ++e) a[e] = active ? data[base + tt + T * e] : mk<C>(0.0, 0.0);
  FftRun<C, N, E, DIR, 1, typename PP::P>::run(a, tt, row, tws, BlockSync{});
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) data[base + tt + T * e] = a[e];
  }
}

// B applied to one voxel's (u, Jx, Jy)
template <class C>
__device__ __forceinline__ void fx_bapply(const C* __restrict__ bu, const C* __restrict__ b2, long v, long n,
                                          const C (&z)[3], C (&o)[3]) {
  o[0] = cmul(bu[v], z[0]);
  o[1] = cadd(cmul(b2[4 * v + 0], z[1]), cmul(b2[4 * v + 1], z[2]));
  o[2] = cadd(cmul(b2[4 * v + 2], z[1]), cmul(b2[4 * v + 3], z[2]));
}

// t = B x + y (has_x) or t = y
template <class C>
__global__ void __launch_bounds__(256) k_fx_first(const C* __restrict__ x, const C* __restrict__ y,
                                                  const C* __restrict__ bu, const C* __restrict__ b2,
                                                  C* __restrict__ t, long n, int has_x) {
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < n; v += (long)gridDim.x * blockDim.x) {
    C z[3], o[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) z[k] = has_x ? x[k * n + v] : mk<C>(0.0, 0.0);
    fx_bapply(bu, b2, v, n, z, o);
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k * n + v] = cadd(o[k], y[k * n + v]);
  }
}

// Delta = B (u - x) with u in t; x += alpha Delta; ||Delta||^2 partials; t = B x + y
template <class C>
__global__ void __launch_bounds__(256) k_fx_update(C* __restrict__ t, C* __restrict__ x, const C* __restrict__ y,
                                                   const C* __restrict__ bu, const C* __restrict__ b2, double alpha,
                                                   long n, double* __restrict__ row) {
  using Rr = typename real_of<C>::type;
  __shared__ double scratch[64];
  const Rr a = (Rr)alpha;
  double acc = 0.0;
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < n; v += (long)gridDim.x * blockDim.x) {
    C z[3], dl[3], xn[3], o[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) z[k] = csub(t[k * n + v], x[k * n + v]);
    fx_bapply(bu, b2, v, n, z, dl);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      xn[k] = cadd(x[k * n + v], cscale(dl[k], a));
      x[k * n + v] = xn[k];
      acc += cabs2(dl[k]);
    }
    fx_bapply(bu, b2, v, n, xn, o);
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k * n + v] = cadd(o[k], y[k * n + v]);
  }
  block_partial(acc, scratch, row);
}

// 3 x 3 complex inverse by the adjugate (in double)
__device__ __forceinline__ void zinv3(const double (&m)[3][3][2], double (&r)[3][3][2]) {
  auto mul = [](const double* a, const double* b, double* o) {
    o[0] = a[0] * b[0] - a[1] * b[1];
    o[1] = a[0] * b[1] + a[1] * b[0];
  };
  double cof[3][3][2];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      double p[2], q[2];
      mul(m[i1][j1], m[i2][j2], p);
      mul(m[i1][j2], m[i2][j1], q);
      cof[i][j][0] = p[0] - q[0];
      cof[i][j][1] = p[1] - q[1];
    }
  double det[2] = {0.0, 0.0};
  for (int j = 0; j < 3; ++j) {
    double p[2];
    mul(m[0][j], cof[0][j], p);
    det[0] += p[0];
    det[1] += p[1];
  }
  const double dd = det[0] * det[0] + det[1] * det[1];
  const double id[2] = {det[0] / dd, -det[1] / dd};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) mul(cof[j][i], id, r[i][j]);  // adjugate = cofactor transpose
}

// Per Fourier mode (k0, k1): t <- M(p) t / (n0 n1), M = (L + I)^-1 (inverse) or L
template <class C>
__global__ void __launch_bounds__(256) k_fx_sym(C* __restrict__ t, FluxSym fs, int inverse) {
  using Rr = typename real_of<C>::type;
  const long n = (long)fs.n0 * fs.n1;
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < n; v += (long)gridDim.x * blockDim.x) {
    const int k0 = (int)(v / fs.n1), k1 = (int)(v % fs.n1);
    const int f0 = k0 < (fs.n0 + 1) / 2 ? k0 : k0 - fs.n0, f1 = k1 < (fs.n1 + 1) / 2 ? k1 : k1 - fs.n1;
    const double p0 = (fs.n0 % 2 == 0 && k0 == fs.n0 / 2) ? 0.0 : fs.pscale0 * f0;
    const double p1 = (fs.n1 % 2 == 0 && k1 == fs.n1 / 2) ? 0.0 : fs.pscale1 * f1;
    double m[3][3][2];
    const double* s = fs.s;
    const double ic = 1.0 / fs.c;
    m[0][0][0] = s[0] * s[0] * fs.mubar[0] * ic;
    m[0][0][1] = s[0] * s[0] * fs.mubar[1] * ic;
    m[0][1][0] = 0.0; m[0][1][1] = s[0] * s[1] * p1 * ic;
    m[1][0][0] = 0.0; m[1][0][1] = s[0] * s[1] * p1 * ic;
    m[0][2][0] = 0.0; m[0][2][1] = s[0] * s[2] * p0 * ic;
    m[2][0][0] = 0.0; m[2][0][1] = s[0] * s[2] * p0 * ic;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        m[1 + a][1 + b][0] = s[1 + a] * s[1 + b] * fs.dibar[2 * a + b][0] * ic;
        m[1 + a][1 + b][1] = s[1 + a] * s[1 + b] * fs.dibar[2 * a + b][1] * ic;
      }
    double r[3][3][2];
    if (inverse) {
      for (int i = 0; i < 3; ++i) m[i][i][0] += 1.0;
      zinv3(m, r);
    } else {
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          r[i][j][0] = m[i][j][0];
          r[i][j][1] = m[i][j][1];
        }
    }
    const double sc = 1.0 / (double)n;
    C in[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) in[k] = t[k * n + v];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double o0 = 0.0, o1 = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        o0 += r[i][j][0] * (double)in[j].x - r[i][j][1] * (double)in[j].y;
        o1 += r[i][j][0] * (double)in[j].y + r[i][j][1] * (double)in[j].x;
      }
      t[i * n + v] = mk<C>((Rr)(o0 * sc), (Rr)(o1 * sc));
    }
  }
}

// FP64 residual: S holds L x (after the inverse transforms); r = y - L x - (x - B x);
// partials of ||r||^2 (row0) and ||y||^2 (row1)
template <class C>
__global__ void __launch_bounds__(256) k_fx_res(const double2* __restrict__ Sx, const C* __restrict__ x,
                                                const C* __restrict__ y, const C* __restrict__ bu,
                                                const C* __restrict__ b2, long n, double* __restrict__ row0,
                                                double* __restrict__ row1) {
  __shared__ double scratch[64];
  double rr = 0.0, yy = 0.0;
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < n; v += (long)gridDim.x * blockDim.x) {
    double2 z[3], bz[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) z[k] = cvt<double2>(x[k * n + v]);
    const double2 b0 = cvt<double2>(bu[v]);
    bz[0] = cmul(b0, z[0]);
    bz[1] = cadd(cmul(cvt<double2>(b2[4 * v + 0]), z[1]), cmul(cvt<double2>(b2[4 * v + 1]), z[2]));
    bz[2] = cadd(cmul(cvt<double2>(b2[4 * v + 2]), z[1]), cmul(cvt<double2>(b2[4 * v + 3]), z[2]));
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double2 yv = cvt<double2>(y[k * n + v]);
      const double2 r = cadd(csub(csub(yv, Sx[k * n + v]), z[k]), bz[k]);
      rr += cabs2(r);
      yy += cabs2(yv);
    }
  }
  const double a = block_sum(rr, scratch);
  const double b = block_sum(yy, scratch);
  if (threadIdx.x == 0) {
    row0[blockIdx.x] = a;
    row1[blockIdx.x] = b;
  }
}

// x (storage C) -> double2 copy into the residual spectrum buffer
template <class C>
__global__ void __launch_bounds__(256) k_fx_widen(const C* __restrict__ x, double2* __restrict__ S, long n3) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n3; i += (long)gridDim.x * blockDim.x)
    S[i] = cvt<double2>(x[i]);
}

// block r adds row r of `part` (ncols partials, pitch) in a fixed order into out[r]
template <int U = 0>
__global__ void __launch_bounds__(256) k_fx_sum(const double* __restrict__ part, long pitch, int ncols,
                                                double* __restrict__ out) {
  __shared__ double scratch[64];
  const double* row = part + (long)blockIdx.x * pitch;
  double acc = 0.0;
  for (int i = threadIdx.x; i < ncols; i += blockDim.x) acc += row[i];
  const double s = block_sum(acc, scratch);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

}  // namespace usp
