// Kernels of the Krylov drivers (BiCGSTAB, restarted GMRES(m), CG for
// Hermitian positive definite systems) on the preconditioned system with the
// forward problem eliminated (Sec. 2.1):
//     P v = B [v - (L + I)^-1 (B v)],      b = B (L + I)^-1 y,
// so one step of Algorithm 1 is x <- x + alpha (b - P x).
//
// P v runs as the iteration's pass structure: k_kfirst (t = FFT along n2 of
// B v, or of y for b), the strided passes with 1/(N (l(p) + 1)) (shared with
// the iteration), and k_klast (inverse FFT along n2, w = B (v - u) or B u,
// with the dot products a method needs fused in as per-block partial rows).
// Vector updates take their scalars from device memory (written by k_kscal),
// so an iteration queues without host round trips.  Complex dot products are
// <a, b> = sum conj(a) b, accumulated in double.
#pragma once
#include "passes.hpp"

namespace usp {

// slots of the device scalar array (doubles, complex values as re, im)
enum KSlot {
  KS_RHO = 0, KS_RHON = 2, KS_ALPHA = 4, KS_OMEGA = 6, KS_BETA = 8, KS_RV = 10, KS_TS = 12, KS_TT = 14,
  KS_RR = 15, KS_FLAG = 16, KS_NRM = 17,
  KS_CRR = 18,   // CG: |r|^2 at a check
  KS_CGG = 20,   // CG: gamma_i = |r_i|^2 in slot 20 + (i & 1)
  KS_CGA = 22,   // CG: alpha_i (complex) in slots 22 + 2 (i & 1), + 1
  KS_H = 32, KS_COEF = 512
};
enum KScalMode { KSM_INIT = 0, KSM_BETA = 1, KSM_ALPHA = 2, KSM_OMEGA = 3 };

__device__ __forceinline__ void zdiv(double ar, double ai, double br, double bi, double& cr, double& ci) {
  const double d = br * br + bi * bi;
  cr = (ar * br + ai * bi) / d;
  ci = (ai * br - ar * bi) / d;
}

// the BiCGSTAB scalar recurrences, one thread
__global__ void k_kscal(double* ks, int mode) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (mode == KSM_INIT) {
    ks[KS_RHO] = 1.0; ks[KS_RHO + 1] = 0.0;
    ks[KS_ALPHA] = 1.0; ks[KS_ALPHA + 1] = 0.0;
    ks[KS_OMEGA] = 1.0; ks[KS_OMEGA + 1] = 0.0;
    ks[KS_BETA] = 0.0; ks[KS_BETA + 1] = 0.0;
    ks[KS_FLAG] = 0.0;
  } else if (mode == KSM_BETA) {  // beta = (rho_new / rho)(alpha / omega); rho = rho_new
    double ar, ai, br, bi;
    zdiv(ks[KS_RHON], ks[KS_RHON + 1], ks[KS_RHO], ks[KS_RHO + 1], ar, ai);
    zdiv(ks[KS_ALPHA], ks[KS_ALPHA + 1], ks[KS_OMEGA], ks[KS_OMEGA + 1], br, bi);
    const double pr = ar * br - ai * bi, pi = ar * bi + ai * br;
    const bool ok = pr == pr && pi == pi;
    ks[KS_BETA] = ok ? pr : 0.0;
    ks[KS_BETA + 1] = ok ? pi : 0.0;
    if (!ok) ks[KS_FLAG] += 1.0;
    ks[KS_RHO] = ks[KS_RHON];
    ks[KS_RHO + 1] = ks[KS_RHON + 1];
  } else if (mode == KSM_ALPHA) {  // alpha = rho / <r^, v>
    const double dr = ks[KS_RV], di = ks[KS_RV + 1];
    if (dr == 0.0 && di == 0.0) {
      ks[KS_ALPHA] = ks[KS_ALPHA + 1] = 0.0;
      ks[KS_FLAG] += 1.0;
    } else {
      zdiv(ks[KS_RHO], ks[KS_RHO + 1], dr, di, ks[KS_ALPHA], ks[KS_ALPHA + 1]);
    }
  } else {  // omega = <t, s> / <t, t>
    const double tt = ks[KS_TT];
    if (tt == 0.0) {
      ks[KS_OMEGA] = ks[KS_OMEGA + 1] = 0.0;
      ks[KS_FLAG] += 1.0;
    } else {
      ks[KS_OMEGA] = ks[KS_TS] / tt;
      ks[KS_OMEGA + 1] = ks[KS_TS + 1] / tt;
    }
  }
}

template <class C> __device__ __forceinline__ C kz(const double* s) {
  return mk<C>(s[0], s[1]);
}
// conj(a) * b accumulated in double
template <class C> __device__ __forceinline__ void cdot_acc(const C& a, const C& b, double& re, double& im) {
  re += (double)a.x * b.x + (double)a.y * b.y;
  im += (double)a.x * b.y - (double)a.y * b.x;
}

// two per-block partials at once (deterministic, as block_partial)
__device__ __forceinline__ void block_partial2(double a, double b, double* scratch, double* row_a, double* row_b) {
  const double sa = block_sum(a, scratch);
  const double sb = block_sum(b, scratch);
  if (threadIdx.x == 0) {
    row_a[blockIdx.x] = sa;
    row_b[blockIdx.x] = sb;
  }
}

// First pass of P v (or of b): t = FFT along n2 of (B ? B v : v).
template <class C, int N>
__global__ void __launch_bounds__(x_threads<C>())
k_kfirst(C* __restrict__ t, const C* __restrict__ v, const C* __restrict__ B, const C* __restrict__ tw, int nlines) {
  using PP = PassPlan<N>;
  constexpr int E = PP::E, T = N / E;
  constexpr int LPB = (x_threads<C>() / T) > 0 ? (x_threads<C>() / T) : 1;
  constexpr int TH = LPB * T;
  __shared__ C lds[LPB * LdsRow<C>::padded(N)];
  __shared__ C tws[N];
  load_twiddles<C, N>(tws, tw);
  const int tid = threadIdx.x;
  if (tid >= TH) {
    if (!line_in_wave<T>()) idle_fft_syncs<N, typename PP::P>();
    return;
  }
  const int tt = tid % T, li = tid / T;
  const long line = (long)blockIdx.x * LPB + li;
  const bool active = line < nlines;
  const long base = line * N;
  LdsRow<C> row{lds + li * LdsRow<C>::padded(N)};
  C a[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const long p = base + tt + T * e;
    C val = mk<C>(0.0, 0.0);
    if (active) {
      val = v[p];
      if (B) val = cmul(B[p], val);
    }
    a[e] = val;
  }
  FftRun<C, N, E, -1, 1, typename PP::P>::run(a, tt, row, tws, LineSync<T>{});
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) t[base + tt + T * e] = a[e];
  }
}

// Last pass: u = inverse FFT along n2 of t (already scaled by 1/(N (l + 1))),
// w = B (v - u) (RHS = false) or w = B u (RHS = true; v unused).  Dot partials,
// one row each (row pitch `pitch`): bit 0 <q, w> (rows 0, 1), bit 1 <w, v>
// (rows 2, 3), bit 2 |w|^2 (row 4), bit 3 |v|^2 (row 5; RHS = false).
template <class C, int N, bool RHS>
__global__ void __launch_bounds__(x_threads<C>())
k_klast(const C* __restrict__ t, const C* __restrict__ v, const C* __restrict__ B, C* __restrict__ w,
        const C* __restrict__ q, const C* __restrict__ tw, int nlines, double* __restrict__ rows, long pitch,
        int dots) {
  using PP = PassPlan<N>;
  constexpr int E = PP::E, T = N / E;
  constexpr int LPB = (x_threads<C>() / T) > 0 ? (x_threads<C>() / T) : 1;
  constexpr int TH = LPB * T;
  __shared__ C lds[LPB * LdsRow<C>::padded(N)];
  __shared__ C tws[N];
  __shared__ double scratch[64];
  load_twiddles<C, N>(tws, tw);
  const int tid = threadIdx.x;
  double qr = 0.0, qi = 0.0, wr = 0.0, wi = 0.0, ww = 0.0, vv2 = 0.0;
  if (tid < TH) {
    const int tt = tid % T, li = tid / T;
    const long line = (long)blockIdx.x * LPB + li;
    const bool active = line < nlines;
    const long base = line * N;
    LdsRow<C> row{lds + li * LdsRow<C>::padded(N)};
    C a[E];
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = active ? t[base + tt + T * e] : mk<C>(0.0, 0.0);
    FftRun<C, N, E, +1, 1, typename PP::P>::run(a, tt, row, tws, LineSync<T>{});
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const long p = base + tt + T * e;
        const C bb = B[p];
        C out;
        C vv = mk<C>(0.0, 0.0);
        if (RHS) {
          out = cmul(bb, a[e]);
        } else {
          vv = v[p];
          out = cmul(bb, csub(vv, a[e]));
        }
        w[p] = out;
        if (dots & 1) cdot_acc(q[p], out, qr, qi);
        if (dots & 2) cdot_acc(out, vv, wr, wi);
        if (dots & 4) ww += (double)out.x * out.x + (double)out.y * out.y;
        if (dots & 8) vv2 += (double)vv.x * vv.x + (double)vv.y * vv.y;
      }
    }
  } else if (!line_in_wave<T>()) {
    idle_fft_syncs<N, typename PP::P>();
  }
  if (dots & 1) block_partial2(qr, qi, scratch, rows, rows + pitch);
  if (dots & 2) block_partial2(wr, wi, scratch, rows + 2 * pitch, rows + 3 * pitch);
  if (dots & 4) block_partial(ww, scratch, rows + 4 * pitch);
  if (dots & 8) block_partial(vv2, scratch, rows + 5 * pitch);
}

// ---- vector kernels (grid-stride; per-block partial rows of width gridDim.x) ----

// r = b - w, with |r|^2 partials in row 0
template <class C>
__global__ void __launch_bounds__(256) k_ksub(C* __restrict__ r, const C* b, const C* __restrict__ w, long n,
                                              double* __restrict__ rows) {
  __shared__ double scratch[64];
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const C z = csub(b[i], w[i]);
    r[i] = z;
    acc += (double)z.x * z.x + (double)z.y * z.y;
  }
  block_partial(acc, scratch, rows);
}

// BiCGSTAB: p = r + beta (p - omega v)
template <class C>
__global__ void __launch_bounds__(256) k_bicg_p(C* __restrict__ p, const C* __restrict__ r, const C* __restrict__ v,
                                                const double* __restrict__ ks, long n) {
  const C beta = kz<C>(ks + KS_BETA), omega = kz<C>(ks + KS_OMEGA);
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = cadd(r[i], cmul(beta, csub(p[i], cmul(omega, v[i]))));
}

// BiCGSTAB: s = r - alpha v;  x = x + alpha p
template <class C>
__global__ void __launch_bounds__(256) k_bicg_s(C* __restrict__ s, const C* __restrict__ r, const C* __restrict__ v,
                                                C* __restrict__ x, const C* __restrict__ p,
                                                const double* __restrict__ ks, long n) {
  const C alpha = kz<C>(ks + KS_ALPHA);
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    s[i] = csub(r[i], cmul(alpha, v[i]));
    x[i] = cadd(x[i], cmul(alpha, p[i]));
  }
}

// BiCGSTAB: x = x + omega s;  r = s - omega t;  partials <r^, r> (rows 0, 1) and |r|^2 (row 2)
template <class C>
__global__ void __launch_bounds__(256) k_bicg_r(C* __restrict__ x, const C* __restrict__ s, const C* __restrict__ t,
                                                C* __restrict__ r, const C* __restrict__ rhat,
                                                const double* __restrict__ ks, long n, double* __restrict__ rows,
                                                long pitch) {
  __shared__ double scratch[64];
  const C omega = kz<C>(ks + KS_OMEGA);
  double dr = 0.0, di = 0.0, rr = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const C si = s[i];
    x[i] = cadd(x[i], cmul(omega, si));
    const C ri = csub(si, cmul(omega, t[i]));
    r[i] = ri;
    cdot_acc(rhat[i], ri, dr, di);
    rr += (double)ri.x * ri.x + (double)ri.y * ri.y;
  }
  block_partial2(dr, di, scratch, rows, rows + pitch);
  block_partial(rr, scratch, rows + 2 * pitch);
}

// ordered sum of n partials, the same value in every thread of every block
// that calls it on the same row (fixed strides, fixed reduction tree)
__device__ __forceinline__ double row_total(const double* __restrict__ row, int n, double* scratch) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += row[i];
  return block_sum(acc, scratch);
}

// CG step in the Chronopoulos-Gear arrangement (one reduction point per
// iteration; s = P p is carried by a recurrence instead of recomputed):
//   gamma_i = |r_i|^2 (row 5) and delta_i = r_i^H w_i (rows 2, 3 hold
//   <w, r> = conj(delta)) with w_i = P r_i, both summed from the last pass's
//   partials; beta_i = gamma_i / gamma_{i-1}, alpha_i = gamma_i / (delta_i -
//   beta_i gamma_i / alpha_{i-1}) (beta_0 = 0, alpha_0 = gamma_0 / delta_0);
//   p = r + beta p, s = w + beta s, x += alpha p, r -= alpha s,
// then t = FFT along n2 of B r for the next P r.  Every block derives the same
// scalars; block 0 keeps gamma_i and alpha_i in the ks slots of parity i for
// step i + 1.  A zero denominator gives alpha = 0 and raises ks[KS_FLAG].
template <class C, int N>
__global__ void __launch_bounds__(x_threads<C>())
k_cgcg_first(C* __restrict__ t, C* __restrict__ x, C* __restrict__ r, C* __restrict__ p, C* __restrict__ s,
             const C* __restrict__ w, const C* __restrict__ B, const C* __restrict__ tw, int nlines,
             const double* __restrict__ rows, long pitch, int nrow, double* __restrict__ ks, int it) {
  using PP = PassPlan<N>;
  using Rr = typename real_of<C>::type;
  constexpr int E = PP::E, T = N / E;
  constexpr int LPB = (x_threads<C>() / T) > 0 ? (x_threads<C>() / T) : 1;
  constexpr int TH = LPB * T;
  __shared__ C lds[LPB * LdsRow<C>::padded(N)];
  __shared__ C tws[N];
  __shared__ double scratch[64];
  const double g = row_total(rows + 5 * pitch, nrow, scratch);
  const double dr = row_total(rows + 2 * pitch, nrow, scratch), di = -row_total(rows + 3 * pitch, nrow, scratch);
  double beta = 0.0, ar = 0.0, ai = 0.0;
  bool bad = false;
  if (it == 0) {
    if (dr == 0.0 && di == 0.0) bad = true;
    else zdiv(g, 0.0, dr, di, ar, ai);
  } else {
    const int q = (it - 1) & 1;
    const double gp = ks[KS_CGG + q], apr = ks[KS_CGA + 2 * q], api = ks[KS_CGA + 2 * q + 1];
    beta = gp > 0.0 ? g / gp : 0.0;
    double cr = 0.0, ci = 0.0;
    if (apr == 0.0 && api == 0.0) bad = true;
    else zdiv(beta * g, 0.0, apr, api, cr, ci);
    const double er = dr - cr, ei = di - ci;
    if (bad || (er == 0.0 && ei == 0.0)) bad = true;
    else zdiv(g, 0.0, er, ei, ar, ai);
  }
  if (bad || !(ar == ar && ai == ai)) ar = ai = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ks[KS_CGG + (it & 1)] = g;
    ks[KS_CGA + 2 * (it & 1)] = ar;
    ks[KS_CGA + 2 * (it & 1) + 1] = ai;
    if (bad) ks[KS_FLAG] += 1.0;
  }
  load_twiddles<C, N>(tws, tw);
  const int tid = threadIdx.x;
  if (tid >= TH) {
    if (!line_in_wave<T>()) idle_fft_syncs<N, typename PP::P>();
    return;
  }
  const C alpha = mk<C>(ar, ai);
  const int tt = tid % T, li = tid / T;
  const long line = (long)blockIdx.x * LPB + li;
  const bool active = line < nlines;
  const long base = line * N;
  LdsRow<C> row{lds + li * LdsRow<C>::padded(N)};
  C a[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const long q = base + tt + T * e;
    C val = mk<C>(0.0, 0.0);
    if (active) {
      const C pn = cadd(r[q], cscale(p[q], (Rr)beta));
      const C sn = cadd(w[q], cscale(s[q], (Rr)beta));
      p[q] = pn;
      s[q] = sn;
      x[q] = cadd(x[q], cmul(alpha, pn));
      const C rn = csub(r[q], cmul(alpha, sn));
      r[q] = rn;
      val = cmul(B[q], rn);
    }
    a[e] = val;
  }
  FftRun<C, N, E, -1, 1, typename PP::P>::run(a, tt, row, tws, LineSync<T>{});
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) t[base + tt + T * e] = a[e];
  }
}


// |z|^2 partials in row 0 (grid-stride)
template <class C>
__global__ void __launch_bounds__(256) k_knorm2(const C* __restrict__ z, long n, double* __restrict__ rows) {
  __shared__ double scratch[64];
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc += (double)z[i].x * z[i].x + (double)z[i].y * z[i].y;
  block_partial(acc, scratch, rows);
}

// sum of (Im z)^2 partials in row 0 (a test that B is real)
template <class C>
__global__ void __launch_bounds__(256) k_imag2(const C* __restrict__ z, long n, double* __restrict__ rows) {
  __shared__ double scratch[64];
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc += (double)z[i].y * z[i].y;
  block_partial(acc, scratch, rows);
}

// GMRES: partials of <V_i, w> for i < k (rows 2i, 2i + 1; basis vector i at
// V + i * stride, n elements each); each block owns a
// contiguous chunk of KE * 256 elements, held in registers while the basis streams.
template <class C, int KE>
__global__ void __launch_bounds__(256) k_mdot(const C* __restrict__ V, long stride, long n, int k,
                                              const C* __restrict__ w, double* __restrict__ rows, long pitch) {
  __shared__ double scratch[64];
  const long c0 = (long)blockIdx.x * KE * 256;
  C wl[KE];
#pragma unroll
  for (int e = 0; e < KE; ++e) {
    const long j = c0 + e * 256 + threadIdx.x;
    wl[e] = j < n ? w[j] : mk<C>(0.0, 0.0);
  }
  for (int i = 0; i < k; ++i) {
    const C* vi = V + (long)i * stride;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int e = 0; e < KE; ++e) {
      const long j = c0 + e * 256 + threadIdx.x;
      if (j < n) cdot_acc(vi[j], wl[e], re, im);
    }
    block_partial2(re, im, scratch, rows + 2 * i * pitch, rows + (2 * i + 1) * pitch);
  }
}

// y = y + sign * sum_{i<k} c_i V_i (V_i at V + i * stride; c: k complex doubles on the device);
// optional |y|^2 partials in row 0.
template <class C>
__global__ void __launch_bounds__(256) k_maxpy(C* __restrict__ y, const C* __restrict__ V, long stride, long n, int k,
                                               const double* __restrict__ c, double sign, double* __restrict__ rows) {
  __shared__ double scratch[64];
  double acc = 0.0;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    C s = mk<C>(0.0, 0.0);
    for (int i = 0; i < k; ++i) s = cadd(s, cmul(mk<C>(sign * c[2 * i], sign * c[2 * i + 1]), V[(long)i * stride + j]));
    const C z = cadd(y[j], s);
    y[j] = z;
    acc += (double)z.x * z.x + (double)z.y * z.y;
  }
  if (rows) block_partial(acc, scratch, rows);
}

// out = in / sqrt(nrm2[0])
template <class C>
__global__ void __launch_bounds__(256) k_kscale(C* __restrict__ out, const C* __restrict__ in, long n,
                                                const double* __restrict__ nrm2) {
  const double s = 1.0 / sqrt(nrm2[0]);
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x)
    out[j] = cscale(in[j], (typename real_of<C>::type)s);
}

}  // namespace usp
