// Small element-wise and reduction kernels used around the solver: canonical
// fields (B = 1 - v, y), norms, the ||V|| < 1 check, precision casts, and the
// FP64 true residual of 1-D problems.
#pragma once
#include "fft.hpp"
#include "solve1d.hpp"

namespace usp {

// B = 1 - (q - bias)/c,  y = src_scale * S / c   (canonical form, Sec. 2.2)
template <class Co>
__global__ void k_canonical_fields(const double2* __restrict__ q, const double2* __restrict__ S, long n,
                                   double br, double bi, double cr, double ci, double src_scale,
                                   Co* __restrict__ B, Co* __restrict__ y) {
  const double2 ic = crecip(mk<double2>(cr, ci));
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    if (B) {
      const double2 v = cmul(csub(q[i], mk<double2>(br, bi)), ic);
      B[i] = cvt<Co>(mk<double2>(1.0 - v.x, -v.y));
    }
    if (y) y[i] = cvt<Co>(cscale(cmul(S[i], ic), src_scale));
  }
}

// per-block partial sums of |z|^2 into row[block]
template <class C>
__global__ void __launch_bounds__(256) k_norm2(const C* __restrict__ z, long n, double* row) {
  __shared__ double scratch[64];
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc += cabs2(z[i]);
  block_partial(acc, scratch, row);
}

// Block r adds row r of `part` (ncols partials of type R, row pitch `pitch`
// elements of R) in a fixed order, in the precision of the partials, and
// writes out[(first + r) % nmod].
template <class R>
__global__ void __launch_bounds__(256) k_sum_rows(const R* __restrict__ part, long pitch, int ncols,
                                                  double* __restrict__ out, int first, int nmod) {
  __shared__ R scratch[64];
  const R* row = part + (long)blockIdx.x * pitch;
  R acc = R(0);
  for (int i = threadIdx.x; i < ncols; i += blockDim.x) acc += row[i];
  const R s = block_sum(acc, scratch);
  if (threadIdx.x == 0) out[(first + (int)blockIdx.x) % nmod] = s;
}

// per-block max |1 - B|  ->  partials[block]
template <class C>
__global__ void __launch_bounds__(256) k_max_v(const C* __restrict__ B, long n, double* partials) {
  __shared__ double s[256];
  double m = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double vr = 1.0 - (double)B[i].x, vi = -(double)B[i].y;
    m = fmax(m, vr * vr + vi * vi);
  }
  s[threadIdx.x] = m;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(256) k_max_final(const double* __restrict__ partials, int n, double* out) {
  __shared__ double s[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, partials[i]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(s[0]);
}

// dst = src in 16-byte units, non-temporal: each block copies one contiguous
// chunk of 4 x 256 units (four loads in flight per thread, then four stores);
// measured the fastest of the grid-stride and chunked forms tried (1 GiB:
// 6.2 TB/s of read + write against 5.2 TB/s for a grid-stride loop)
constexpr int kCopyUnroll = 4;
__global__ void __launch_bounds__(256) k_stream_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                                     long n) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  const d2v* s = reinterpret_cast<const d2v*>(src);
  d2v* d = reinterpret_cast<d2v*>(dst);
  const long base = (long)blockIdx.x * blockDim.x * kCopyUnroll + threadIdx.x;
  d2v v[kCopyUnroll];
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const long j = base + (long)u * blockDim.x;
    if (j < n) v[u] = __builtin_nontemporal_load(s + j);
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const long j = base + (long)u * blockDim.x;
    if (j < n) __builtin_nontemporal_store(v[u], d + j);
  }
}

// complex128 -> complex64
__global__ void k_to_c64(const double2* __restrict__ a, float2* __restrict__ b, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = cvt<float2>(a[i]);
}

// FP64 true residual of a 1-D problem (single workgroup):
// r = y - L x - (1 - B) x - G x,  out[0] = ||r||^2, out[1] = ||y||^2.
template <class Cx, int N>
__global__ void __launch_bounds__(N / LinePlan<N>::E)
k_residual1d(const Cx* __restrict__ x, const Cx* __restrict__ y, const Cx* __restrict__ B,
             const int* __restrict__ gi, const Cx* __restrict__ g0, const Cx* __restrict__ g1,
             const double2* __restrict__ tw, Sym1D sym, double* __restrict__ out) {
  using LP = LinePlan<N>;
  constexpr int E = LP::E, T = N / E;
  __shared__ double2 lds[LdsRow<double2>::padded(N)];
  __shared__ double2 xs[N];
  __shared__ double scratch[64];
  const int t = threadIdx.x;
  LdsRow<double2> row{lds};
  double2 v[E], xv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    xv[e] = cvt<double2>(x[t + T * e]);
    v[e] = xv[e];
    xs[t + T * e] = xv[e];
  }
  FftRun<double2, N, E, -1, 1, typename LP::P>::run(v, t, row, tw, BlockSync{});
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = cmul(v[e], sym1d_mult<double2, N>(sym, t + T * e, false));
  FftRun<double2, N, E, +1, 1, typename LP::P>::run(v, t, row, tw, BlockSync{});
  __syncthreads();
  double rr = 0.0, yy = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int p = t + T * e;
    const double2 yv = cvt<double2>(y[p]), bv = cvt<double2>(B[p]);
    double2 r = cadd(csub(csub(yv, v[e]), xv[e]), cmul(bv, xv[e]));
    if (gi) {
      const int i0 = min(max(gi[p], 0), N - 1);
      const int i1 = (i0 + 1 < N) ? i0 + 1 : N - 1;
      r = csub(r, cadd(cmul(cvt<double2>(g0[p]), xs[i0]), cmul(cvt<double2>(g1[p]), xs[i1])));
    }
    rr += cabs2(r);
    yy += cabs2(yv);
  }
  rr = block_sum(rr, scratch);
  yy = block_sum(yy, scratch);
  if (t == 0) {
    out[0] = rr;
    out[1] = yy;
  }
}

}  // namespace usp
