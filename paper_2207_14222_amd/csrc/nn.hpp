// Kernels of the learned initial guess: a small 3-D convolutional network on
// channels-last bf16 activations with fp32 accumulation on the matrix cores.
//
// Tensors: activations [V][C] bf16 (stored as raw 16-bit words), V = D*H*W
// voxels with x fastest, C a multiple of 16; conv weights [COUT][TAPS][CIN]
// bf16 (fp32 master copy in the same layout); biases fp32 [COUT].  A 3x3x3
// convolution with zero padding is an implicit GEMM
//     out[v][co] = sum_{tap, ci} in[v + off(tap)][ci] * w[co][tap][ci]
// computed with v_mfma_f32_16x16x16 bf16 tiles: one wave owns 16 voxels and
// all output channels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace usp {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
// round to nearest even
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ v4s ld4(const uint16_t* p) {
  const uint2 q = *reinterpret_cast<const uint2*>(p);
  v4s r;
  r[0] = (short)(q.x & 0xffff);
  r[1] = (short)(q.x >> 16);
  r[2] = (short)(q.y & 0xffff);
  r[3] = (short)(q.y >> 16);
  return r;
}

// Implicit-GEMM convolution.  TAPS = 27 (3x3x3, padding 1) or 1 (1x1x1).
// SIGN = +1: forward (neighbour v + off); SIGN = -1 with the weight layout
// [CIN_fwd][TAPS][COUT_fwd] gives the gradient with respect to the input.
// The first `cstore` output channels are written with row pitch `cstore`
// (bf16, or fp32 when out_f32), after bias and optional ReLU.
template <int CIN, int COUT, int TAPS, int SIGN, bool RELU>
__global__ void __launch_bounds__(256)
k_conv(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w, const float* __restrict__ bias,
       uint16_t* __restrict__ out_bf, float* __restrict__ out_f32, int cstore, int D, int H, int W) {
  constexpr int NT = COUT / 16, KC = CIN / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long V = (long)D * H * W;
  const long v0 = ((long)blockIdx.x * 4 + wave) * 16;
  if (v0 >= V) return;  // whole wave; the kernel has no block barrier
  const int i = lane & 15, kq = lane >> 4;
  const long v = v0 + i;
  const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)(v / ((long)W * H));
  v4f acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int tap = 0; tap < TAPS; ++tap) {
    int dz = 0, dy = 0, dx = 0;
    if (TAPS == 27) {
      dz = tap / 9 - 1;
      dy = (tap / 3) % 3 - 1;
      dx = tap % 3 - 1;
    }
    const int zz = z + SIGN * dz, yy = y + SIGN * dy, xx = x + SIGN * dx;
    const bool ok = zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W;
    const long nb = ((long)zz * H + yy) * W + xx;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const v4s a = ok ? ld4(in + nb * CIN + kc * 16 + 4 * kq) : v4s{0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const v4s b = ld4(w + ((long)(t * 16 + i) * TAPS + tap) * CIN + kc * 16 + 4 * kq);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int co = t * 16 + i;
    if (co >= cstore) continue;
    const float bb = bias ? bias[co] : 0.f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float val = acc[t][e] + bb;
      if (RELU) val = fmaxf(val, 0.f);
      const long o = (v0 + 4 * kq + e) * cstore + co;
      if (out_f32) out_f32[o] = val;
      else out_bf[o] = f2bf(val);
    }
  }
}

// Weight gradient partials.  Work item = (voxel chunk c, tap, (co-tile,
// ci-tile) pair), one per wave:
//   part[c][tap][co][ci] = sum_{v in chunk c} in[v + off(tap)][ci] * g[v][co]
// (a GEMM over voxels: A = g^T (co x v), B = shifted input (v x ci)).
template <int CIN, int COUT, int TAPS>
__global__ void __launch_bounds__(256)
k_wgrad(const uint16_t* __restrict__ in, const uint16_t* __restrict__ g, float* __restrict__ part, int chunk,
        int nchunks, int D, int H, int W) {
  constexpr int MT = COUT / 16, NTl = CIN / 16, PAIRS = MT * NTl;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const long V = (long)D * H * W;
  const long item = (long)blockIdx.x * 4 + wave;
  if (item >= (long)nchunks * TAPS * PAIRS) return;  // whole wave; no block barrier in this kernel
  const int pair = (int)(item % PAIRS);
  const int tap = (int)((item / PAIRS) % TAPS);
  const long c = item / ((long)PAIRS * TAPS);
  const int mt = pair / NTl, nt = pair % NTl;
  int dz = 0, dy = 0, dx = 0;
  if (TAPS == 27) {
    dz = tap / 9 - 1;
    dy = (tap / 3) % 3 - 1;
    dx = tap % 3 - 1;
  }
  const long c0 = c * chunk;
  const long c1 = (c0 + chunk < V) ? c0 + chunk : V;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (long vs = c0; vs < c1; vs += 16) {
    v4s a, b;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const long v = vs + 4 * kq + e;
      short av = 0, bv = 0;
      if (v < c1) {
        av = (short)g[v * COUT + mt * 16 + i];
        const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)(v / ((long)W * H));
        const int zz = z + dz, yy = y + dy, xx = x + dx;
        if (zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W)
          bv = (short)in[(((long)zz * H + yy) * W + xx) * CIN + nt * 16 + i];
      }
      a[e] = av;
      b[e] = bv;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  // lane holds C[co = mt*16 + 4 kq + e][ci = nt*16 + i]
  float* dst = part + (c * TAPS + tap) * (long)COUT * CIN;
#pragma unroll
  for (int e = 0; e < 4; ++e) dst[(mt * 16 + 4 * kq + e) * CIN + nt * 16 + i] = acc[e];
}

// out[j] = sum_c part[c][j] over nchunks (fixed order), written to the
// [COUT][TAPS][CIN] gradient layout from the [chunk][TAPS][COUT][CIN] partials.
__global__ void k_wgrad_reduce(const float* __restrict__ part, float* __restrict__ dw, int nchunks, int taps, int cout,
                               int cin) {
  const long n = (long)taps * cout * cin;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += part[(long)c * n + j];
    const int tap = (int)(j / ((long)cout * cin)), co = (int)((j / cin) % cout), ci = (int)(j % cin);
    dw[((long)co * taps + tap) * cin + ci] = s;
  }
}

// bias gradient partials: part[block][co] = sum over the block's voxels of g[v][co]
__global__ void k_bgrad(const uint16_t* __restrict__ g, float* __restrict__ part, long V, int C, int chunk) {
  const long v0 = (long)blockIdx.x * chunk;
  for (int co = threadIdx.x; co < C; co += blockDim.x) {
    float s = 0.f;
    for (long v = v0; v < v0 + chunk && v < V; ++v) s += bf2f(g[v * C + co]);
    part[(long)blockIdx.x * C + co] = s;
  }
}
__global__ void k_bgrad_reduce(const float* __restrict__ part, float* __restrict__ db, int nchunks, int C) {
  for (int co = threadIdx.x; co < C; co += blockDim.x) {
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += part[(long)c * C + co];
    db[co] = s;
  }
}

// 2x2x2 average pooling and its gradient; nearest upsampling and its gradient
// (channels-last bf16, the coarse grid has D/2 x H/2 x W/2 voxels)
__global__ void k_pool2(const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int D, int H, int W, int C) {
  const int Do = D / 2, Ho = H / 2, Wo = W / 2;
  const long n = (long)Do * Ho * Wo * C;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    const int c = (int)(j % C);
    const long vo = j / C;
    const int xo = (int)(vo % Wo), yo = (int)((vo / Wo) % Ho), zo = (int)(vo / ((long)Wo * Ho));
    float s = 0.f;
    for (int d = 0; d < 8; ++d) {
      const long vi = ((long)(2 * zo + (d >> 2)) * H + (2 * yo + ((d >> 1) & 1))) * W + (2 * xo + (d & 1));
      s += bf2f(in[vi * C + c]);
    }
    out[j] = f2bf(0.125f * s);
  }
}
__global__ void k_pool2_back(const uint16_t* __restrict__ gout, uint16_t* __restrict__ gin, int D, int H, int W,
                             int C) {
  const long n = (long)D * H * W * C;
  const int Ho = H / 2, Wo = W / 2;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    const int c = (int)(j % C);
    const long v = j / C;
    const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)(v / ((long)W * H));
    const long vo = ((long)(z / 2) * Ho + y / 2) * Wo + x / 2;
    gin[j] = f2bf(0.125f * bf2f(gout[vo * C + c]));
  }
}
// out (fine grid D x H x W) = in (coarse) at (z/2, y/2, x/2), written into
// channels [c0, c0 + C) of an output with Ctot channels
__global__ void k_up2(const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int D, int H, int W, int C,
                      int Ctot, int c0) {
  const long n = (long)D * H * W * C;
  const int Ho = H / 2, Wo = W / 2;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    const int c = (int)(j % C);
    const long v = j / C;
    const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)(v / ((long)W * H));
    const long vo = ((long)(z / 2) * Ho + y / 2) * Wo + x / 2;
    out[v * Ctot + c0 + c] = in[vo * C + c];
  }
}
// gradient of k_up2: coarse[vo][c] = sum of the 8 fine children's gradients
__global__ void k_up2_back(const uint16_t* __restrict__ gfine, uint16_t* __restrict__ gcoarse, int D, int H, int W,
                           int C, int Ctot, int c0) {
  const int Do = D / 2, Ho = H / 2, Wo = W / 2;
  const long n = (long)Do * Ho * Wo * C;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    const int c = (int)(j % C);
    const long vo = j / C;
    const int xo = (int)(vo % Wo), yo = (int)((vo / Wo) % Ho), zo = (int)(vo / ((long)Wo * Ho));
    float s = 0.f;
    for (int d = 0; d < 8; ++d) {
      const long vi = ((long)(2 * zo + (d >> 2)) * H + (2 * yo + ((d >> 1) & 1))) * W + (2 * xo + (d & 1));
      s += bf2f(gfine[vi * Ctot + c0 + c]);
    }
    gcoarse[j] = f2bf(s);
  }
}
// copy channels: dst[v][d0 + c] = src[v][s0 + c], c < C
__global__ void k_chcopy(const uint16_t* __restrict__ src, int Cs, int s0, uint16_t* __restrict__ dst, int Cd, int d0,
                         int C, long V) {
  const long n = V * C;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    const long v = j / C;
    const int c = (int)(j % C);
    dst[v * Cd + d0 + c] = src[v * Cs + s0 + c];
  }
}
// g_pre = g_post * (y > 0), optionally accumulating into an existing gradient
__global__ void k_relu_back(const uint16_t* __restrict__ y, const uint16_t* __restrict__ g, uint16_t* __restrict__ out,
                            long n, int accumulate) {
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    float gv = bf2f(y[j]) > 0.f ? bf2f(g[j]) : 0.f;
    if (accumulate) gv += bf2f(out[j]);
    out[j] = f2bf(gv);
  }
}
// dst += src (bf16)
__global__ void k_add_bf(uint16_t* __restrict__ dst, const uint16_t* __restrict__ src, long n) {
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x)
    dst[j] = f2bf(bf2f(dst[j]) + bf2f(src[j]));
}

// Network input from the complex refractive index n + i kappa: channel 0
// (Re n - n_bg)/n_span, channel 1 kappa/kappa_max, channel 2 the source plane
// indicator (z == plane), channels 3..15 zero.
__global__ void k_features(const float2* __restrict__ nidx, uint16_t* __restrict__ out, int D, int H, int W,
                           double n_bg, double n_span, double kappa_max, int plane) {
  const long V = (long)D * H * W;
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < V; v += (long)gridDim.x * blockDim.x) {
    const int z = (int)(v / ((long)W * H));
    const float2 q = nidx[v];
    uint16_t* o = out + v * 16;
    o[0] = f2bf((float)((q.x - n_bg) / n_span));
    o[1] = f2bf((float)(q.y / kappa_max));
    o[2] = f2bf(z == plane ? 1.f : 0.f);
    for (int c = 3; c < 16; ++c) o[c] = 0;
  }
}

// Relative L2 loss between the prediction p[v][0..1] (fp32, Re/Im scaled by
// 1/s) and the target field x[v] (complex64): per-block partials of
// |s p - x|^2 and |x|^2; the gradient g[v][c] (bf16, 16 channels, zero beyond 2)
// = 2 s (s p - x) / ||x||^2 is written by k_loss_grad once ||x||^2 is known.
__global__ void k_loss_parts(const float* __restrict__ p, const float2* __restrict__ x, float s, long V,
                             double* __restrict__ part) {
  __shared__ double sh[2][256];
  double a = 0.0, b = 0.0;
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < V; v += (long)gridDim.x * blockDim.x) {
    const double er = (double)s * p[2 * v] - x[v].x, ei = (double)s * p[2 * v + 1] - x[v].y;
    a += er * er + ei * ei;
    b += (double)x[v].x * x[v].x + (double)x[v].y * x[v].y;
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0][0];
    part[2 * blockIdx.x + 1] = sh[1][0];
  }
}
__global__ void k_loss_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nb; ++i) {
      a += part[2 * i];
      b += part[2 * i + 1];
    }
    out[0] = a / b;  // relative squared error
    out[1] = b;
  }
}
__global__ void k_loss_grad(const float* __restrict__ p, const float2* __restrict__ x, float s, long V,
                            const double* __restrict__ lossv, uint16_t* __restrict__ g) {
  const float scale = (float)(2.0 * s / lossv[1]);
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < V; v += (long)gridDim.x * blockDim.x) {
    uint16_t* o = g + v * 16;
    o[0] = f2bf(scale * (s * p[2 * v] - x[v].x));
    o[1] = f2bf(scale * (s * p[2 * v + 1] - x[v].y));
    for (int c = 2; c < 16; ++c) o[c] = 0;
  }
}

// Adam step on fp32 master parameters; writes the bf16 copy used by the kernels.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       uint16_t* __restrict__ wb, long n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.f - b1) * gj;
    const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    const float wj = w[j] - lr * (mj / c1) / (sqrtf(vj / c2) + eps);
    w[j] = wj;
    if (wb) wb[j] = f2bf(wj);
  }
}

// [COUT][TAPS][CIN] -> [CIN][TAPS][COUT] (weights for the input gradient)
__global__ void k_wtrans(const uint16_t* __restrict__ w, uint16_t* __restrict__ wt, int cout, int taps, int cin) {
  const long n = (long)cout * taps * cin;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    const int ci = (int)(j % cin), tap = (int)((j / cin) % taps), co = (int)(j / ((long)cin * taps));
    wt[((long)ci * taps + tap) * cout + co] = w[j];
  }
}

// fp32 -> bf16 and bf16 -> fp32 conversions
__global__ void k_f2bf(const float* __restrict__ a, uint16_t* __restrict__ b, long n) {
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) b[j] = f2bf(a[j]);
}

// prediction (fp32 [V][2], scaled by 1/s) -> complex128 field s p
__global__ void k_pred_field(const float* __restrict__ p, float s, double2* __restrict__ x, long V) {
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < V; v += (long)gridDim.x * blockDim.x) {
    double2 z;
    z.x = (double)s * p[2 * v];
    z.y = (double)s * p[2 * v + 1];
    x[v] = z;
  }
}

}  // namespace usp
