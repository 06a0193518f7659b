// Kernels of the learned initial guess: a small 3-D convolutional network on
// bf16 activations with fp32 accumulation on the matrix cores.
//
// Activation layout: 16-channel planes.  A tensor with C channels (C a
// multiple of 16) over V = D*H*W voxels (x fastest) is C/16 planes of
// [V][16] bf16 (raw 16-bit words):
//     element (v, c) at  ((c / 16) * V + v) * 16 + c % 16
// so the 16 x 16 (voxel x channel) operand of one v_mfma_f32_16x16x16 bf16
// is 512 contiguous bytes for 16 consecutive voxels, and concatenating
// tensors along channels is placing their planes one after the other.
// Conv weights [COUT][TAPS][CIN] bf16 (fp32 master copy in the same layout)
// are repacked into fragment order for the kernels (k_wpack); biases fp32.
//
// A 3x3x3 convolution with zero padding is an implicit GEMM
//     out[v][co] = sum_{tap, ci} in[v + off(tap)][ci] * w[co][tap][ci].
// Operand lane layout of v_mfma_f32_16x16x16 bf16 (A 16x16, B 16x16, D = A B):
// lane l holds A[l % 16][4 (l / 16) + e] and B[4 (l / 16) + e][l % 16] for
// e = 0..3, and D[4 (l / 16) + e][l % 16] in element e of its accumulator.
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

__device__ __forceinline__ v4s as_v4s(uint2 q) {
  v4s r;
  r[0] = (short)(q.x & 0xffff);
  r[1] = (short)(q.x >> 16);
  r[2] = (short)(q.y & 0xffff);
  r[3] = (short)(q.y >> 16);
  return r;
}
__device__ __forceinline__ v4s ld4(const uint16_t* p) { return as_v4s(*reinterpret_cast<const uint2*>(p)); }

__device__ __forceinline__ void tap_offsets(int tap, int taps, int& dz, int& dy, int& dx) {
  dz = dy = dx = 0;
  if (taps == 27) {
    dz = tap / 9 - 1;
    dy = (tap / 3) % 3 - 1;
    dx = tap % 3 - 1;
  }
}

// Weights in fragment order.  For a convolution with CIN input and COUT
// output channels (KC = CIN/16 input planes, NT = COUT/16 output tiles):
// * 1 tap: the B operand of v_mfma_f32_16x16x16 bf16 for (kc, t) is 64 lanes x 4 bf16,
//     pk[(kc * NT + t) * 64 + l][e] = Wc[t*16 + l%16][0][kc*16 + 4 (l/16) + e];
// * 27 taps: the B operand of v_mfma_f32_16x16x32 bf16 for (tap pair tp, kc, t) is
//   64 lanes x 8 bf16; lanes of group g = l/16 hold tap 2 tp + g/2 (zero weights
//   for the 28th tap) and input channels kc*16 + 8 (g%2) + e:
//     pk[((tp * KC + kc) * NT + t) * 64 + l][e] = Wc[t*16 + l%16][2 tp + g/2][kc*16 + 8 (g%2) + e].
// The activation operand is laid out the same way (same tap and channel per
// lane group and element), so the product sums over (tap, channel) whatever the
// instruction's internal order of the K slots.  Wc = w (forward, w is
// [COUT][TAPS][CIN]) or, for the input gradient, Wc[a][tap][b] = w[b][tap][a]
// (cin/cout are the forward layer's).  Packed sizes: cin*cout (1 tap),
// 28*cin*cout (27 taps).
__global__ void k_wpack(const uint16_t* __restrict__ w, uint16_t* __restrict__ pk, int cout, int taps, int cin,
                        int transposed) {
  const int ci_c = transposed ? cout : cin;   // input channels of the packed convolution
  const int co_c = transposed ? cin : cout;   // its output channels
  const int KC = ci_c / 16, NT = co_c / 16;
  auto wc = [&](int a, int tap, int b) -> uint16_t {
    return transposed ? w[((long)b * taps + tap) * cin + a] : w[((long)a * taps + tap) * cin + b];
  };
  if (taps == 1) {
    const long n = (long)ci_c * co_c;
    for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
      const int e = (int)(j & 3), l = (int)((j >> 2) & 63);
      const long rest = j >> 8;
      const int t = (int)(rest % NT), kc = (int)(rest / NT);
      pk[j] = wc(t * 16 + (l & 15), 0, kc * 16 + 4 * (l >> 4) + e);
    }
    return;
  }
  const long n = 28L * ci_c * co_c;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    const int e = (int)(j & 7), l = (int)((j >> 3) & 63);
    const long rest = j >> 9;
    const int t = (int)(rest % NT), kc = (int)((rest / NT) % KC), tp = (int)(rest / ((long)NT * KC));
    const int g = l >> 4, tap = 2 * tp + (g >> 1);
    pk[j] = tap < taps ? wc(t * 16 + (l & 15), tap, kc * 16 + 8 * (g & 1) + e) : (uint16_t)0;
  }
}

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
__device__ __forceinline__ v8bf as_v8bf(uint4 q) { return __builtin_bit_cast(v8bf, q); }

// 1x1x1 convolution (the head) with v_mfma_f32_16x16x16 bf16 and the 1-tap
// packing.  SIGN = -1 with transposed packing gives the gradient with respect
// to the input.  One wave computes MV tiles of 16 consecutive voxels x all
// COUT channels.  Output: bf16 planes (all COUT channels), or fp32 rows
// [V][cstore] of the first cstore channels when out_f32; bias and ReLU first.
template <int CIN, int COUT, int TAPS, int SIGN, bool RELU, int MV>
__global__ void __launch_bounds__(256)
k_conv(const uint16_t* __restrict__ in, const uint2* __restrict__ wpk, const float* __restrict__ bias,
       uint16_t* __restrict__ out_bf, float* __restrict__ out_f32, int cstore, int D, int H, int W) {
  constexpr int NT = COUT / 16, KC = CIN / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int V = D * H * W;
  const int vw = (blockIdx.x * 4 + wave) * (16 * MV);
  if (vw >= V) return;  // whole wave; the kernel has no block barrier
  const int i = lane & 15, kq = lane >> 4;
  int xm[MV], ym[MV], zm[MV];
  bool live[MV];
#pragma unroll
  for (int m = 0; m < MV; ++m) {
    const int v = vw + 16 * m + i;
    live[m] = vw + 16 * m < V;  // V is a multiple of 16: tiles are whole
    xm[m] = v % W;
    ym[m] = (v / W) % H;
    zm[m] = v / (W * H);
  }
  v4f acc[MV][NT];
#pragma unroll
  for (int m = 0; m < MV; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int tap = 0; tap < TAPS; ++tap) {
    int dz, dy, dx;
    tap_offsets(tap, TAPS, dz, dy, dx);
    int nb[MV];
    bool ok[MV];
#pragma unroll
    for (int m = 0; m < MV; ++m) {
      const int zz = zm[m] + SIGN * dz, yy = ym[m] + SIGN * dy, xx = xm[m] + SIGN * dx;
      ok[m] = live[m] && zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W;
      nb[m] = (zz * H + yy) * W + xx;
    }
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      v4s b[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) b[t] = as_v4s(wpk[((tap * KC + kc) * NT + t) * 64 + lane]);
#pragma unroll
      for (int m = 0; m < MV; ++m) {
        const v4s a = ok[m] ? ld4(in + ((long)kc * V + nb[m]) * 16 + 4 * kq) : v4s{0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[t], acc[m][t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int co = t * 16 + i;
    const float bb = bias ? bias[co] : 0.f;
#pragma unroll
    for (int m = 0; m < MV; ++m) {
      if (!live[m]) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float val = acc[m][t][e] + bb;
        if (RELU) val = fmaxf(val, 0.f);
        const long v = vw + 16 * m + 4 * kq + e;
        if (out_f32) {
          if (co < cstore) out_f32[v * cstore + co] = val;
        } else {
          out_bf[((long)t * V + v) * 16 + i] = f2bf(val);
        }
      }
    }
  }
}

// Store of one 16-voxel x 16-channel accumulator tile: lane (j, g) holds
// channel t*16 + j of voxels v0 + 4 g + e.
template <bool RELU>
__device__ __forceinline__ void conv_store(const v4f& acc, int t, long v0, int lane, float bb, long V,
                                           uint16_t* __restrict__ out_bf, float* __restrict__ out_f32, int cstore) {
  const int j = lane & 15, g = lane >> 4;
  const int co = t * 16 + j;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float val = acc[e] + bb;
    if (RELU) val = fmaxf(val, 0.f);
    const long v = v0 + 4 * g + e;
    if (out_f32) {
      if (co < cstore) out_f32[v * cstore + co] = val;
    } else {
      out_bf[((long)t * V + v) * 16 + j] = f2bf(val);
    }
  }
}

// 3x3x3 convolution with v_mfma_f32_16x16x32 bf16, two taps per product
// (27-tap packing), operands loaded from global memory.  One wave computes MV
// tiles of 16 consecutive voxels x all COUT channels.  For grids too small or
// too irregular for the LDS-staged kernel.
// TS > 1 (small grids): the output tiles are split over TS blocks
// (blockIdx.y takes tiles [y NT/TS, (y + 1) NT/TS)), for TS times the waves.
template <int CIN, int COUT, int SIGN, bool RELU, int MV, int TS = 1>
__global__ void __launch_bounds__(256)
k_conv27(const uint16_t* __restrict__ in, const uint4* __restrict__ wpk, const float* __restrict__ bias,
         uint16_t* __restrict__ out_bf, float* __restrict__ out_f32, int cstore, int D, int H, int W) {
  constexpr int NTA = COUT / 16, NT = NTA / TS, KC = CIN / 16;
  static_assert(NTA % TS == 0, "tile split");
  const int t0 = blockIdx.y * NT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int V = D * H * W;
  const int vw = (blockIdx.x * 4 + wave) * (16 * MV);
  if (vw >= V) return;  // whole wave; the kernel has no block barrier
  const int i = lane & 15, g = lane >> 4;
  int xm[MV], ym[MV], zm[MV];
  bool live[MV];
#pragma unroll
  for (int m = 0; m < MV; ++m) {
    const int v = vw + 16 * m + i;
    live[m] = vw + 16 * m < V;
    xm[m] = v % W;
    ym[m] = (v / W) % H;
    zm[m] = v / (W * H);
  }
  v4f acc[MV][NT];
#pragma unroll
  for (int m = 0; m < MV; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int tp = 0; tp < 14; ++tp) {
    int tap = 2 * tp + (g >> 1);
    if (tap > 26) tap = 26;  // its weights are zero
    int dz, dy, dx;
    tap_offsets(tap, 27, dz, dy, dx);
    int nb[MV];
    bool ok[MV];
#pragma unroll
    for (int m = 0; m < MV; ++m) {
      const int zz = zm[m] + SIGN * dz, yy = ym[m] + SIGN * dy, xx = xm[m] + SIGN * dx;
      ok[m] = live[m] && zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W;
      nb[m] = (zz * H + yy) * W + xx;
    }
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      v8bf b[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) b[t] = as_v8bf(wpk[((tp * KC + kc) * NTA + t0 + t) * 64 + lane]);
#pragma unroll
      for (int m = 0; m < MV; ++m) {
        const uint4 q = ok[m] ? *reinterpret_cast<const uint4*>(in + ((long)kc * V + nb[m]) * 16 + 8 * (g & 1))
                              : uint4{0u, 0u, 0u, 0u};
        const v8bf a = as_v8bf(q);
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[t], acc[m][t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const float bb = bias ? bias[(t0 + t) * 16 + (lane & 15)] : 0.f;
#pragma unroll
    for (int m = 0; m < MV; ++m)
      if (live[m]) conv_store<RELU>(acc[m][t], t0 + t, vw + 16 * m, lane, bb, V, out_bf, out_f32, cstore);
  }
}

// 3x3x3 convolution, LDS-staged: a block computes a brick of ZB x BY x BX
// output voxels (BX = 16 BXT, BY = 16 / BXT: 16 tiles of 16 voxels per
// z-plane, 4 per wave, four waves per z-plane) and, for each 16-channel input
// plane in turn, stages the (ZB+2) x (BY+2) x (BX+2) input voxels it touches
// (halo zero-filled at the grid faces) in LDS, from where all 27 taps read
// their operands (16 bytes per lane, two taps per v_mfma_f32_16x16x32 bf16).
// Two z-planes per block stage 4 planes for 2 outputs instead of 3 for 1.
// Needs W % BX == 0, H % BY == 0 and D % ZB == 0.
template <int BXT, int ZB = 1> struct ConvTile {
  static constexpr int BX = 16 * BXT, BY = 16 / BXT, SX = BX + 2, SY = BY + 2;
  static constexpr int PLANE_U4 = (ZB + 2) * SY * SX * 2;   // two 16-byte halves per staged voxel
  static constexpr int THREADS = 256 * ZB;
};

template <int CIN, int COUT, int SIGN, bool RELU, int BXT, int ZB = 1>
__global__ void __launch_bounds__(256 * ZB)
k_conv_lds(const uint16_t* __restrict__ in, const uint4* __restrict__ wpk, const float* __restrict__ bias,
           uint16_t* __restrict__ out_bf, float* __restrict__ out_f32, int cstore, int D, int H, int W) {
  using TL = ConvTile<BXT, ZB>;
  constexpr int NT = COUT / 16, KC = CIN / 16, NTH = TL::THREADS;
  constexpr int BX = TL::BX, BY = TL::BY, SX = TL::SX, SY = TL::SY;
  __shared__ uint4 stg[TL::PLANE_U4];
  const int tid = threadIdx.x, lane = tid & 63, wave = (tid >> 6) & 3, zq = tid >> 8;
  const int i = lane & 15, g = lane >> 4;
  const long V = (long)D * H * W;
  const int nxb = W / BX, nyb = H / BY;
  const int xb = blockIdx.x % nxb, yb = (blockIdx.x / nxb) % nyb, z0 = (blockIdx.x / (nxb * nyb)) * ZB;
  const int x0 = xb * BX, y0 = yb * BY;
  // the wave's 4 tiles in output plane z0 + zq: tile q = 4 wave + m at row
  // q / BXT, x offset 16 (q % BXT)
  int lbase[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int q = 4 * wave + m, r = q / BXT, xt = q % BXT;
    lbase[m] = ((zq + 1) * SY + r + 1) * SX + 16 * xt + i + 1;
  }
  v4f acc[4][NT];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = v4f{0.f, 0.f, 0.f, 0.f};
  const uint4* in4 = reinterpret_cast<const uint4*>(in);
  for (int kc = 0; kc < KC; ++kc) {
    __syncthreads();  // the previous plane's reads are done
    auto stage = [&](int u) -> uint4 {
      const int half = u & 1, vox = u >> 1;
      const int sx = vox % SX, sy = (vox / SX) % SY, sz = vox / (SX * SY);
      const int zz = z0 - 1 + sz, yy = y0 - 1 + sy, xx = x0 - 1 + sx;
      if (zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W)
        return in4[((long)kc * V + ((long)zz * H + yy) * W + xx) * 2 + half];
      return uint4{0u, 0u, 0u, 0u};
    };
    if constexpr (KC <= 3) {
      // every load of the plane is issued before the LDS stores: a load
      // followed at once by its store would wait out each load's latency
      // (batches of 5 measured 2% slower; with more input planes the held
      // loads cost occupancy and the plain loop below was faster)
      constexpr int NU = (TL::PLANE_U4 + NTH - 1) / NTH;
      uint4 q[NU];
#pragma unroll
      for (int k = 0; k < NU; ++k) {
        const int u = tid + NTH * k;
        q[k] = u < TL::PLANE_U4 ? stage(u) : uint4{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int k = 0; k < NU; ++k) {
        const int u = tid + NTH * k;
        if (u < TL::PLANE_U4) stg[u] = q[k];
      }
    } else {
      for (int u = tid; u < TL::PLANE_U4; u += NTH) stg[u] = stage(u);
    }
    __syncthreads();
    for (int tp = 0; tp < 14; ++tp) {
      int tap = 2 * tp + (g >> 1);
      if (tap > 26) tap = 26;  // its weights are zero
      int dz, dy, dx;
      tap_offsets(tap, 27, dz, dy, dx);
      const int off = SIGN * ((dz * SY + dy) * SX + dx);
      v8bf b[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) b[t] = as_v8bf(wpk[((tp * KC + kc) * NT + t) * 64 + lane]);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const v8bf a = as_v8bf(stg[(lbase[m] + off) * 2 + (g & 1)]);
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[t], acc[m][t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const float bb = bias ? bias[t * 16 + (lane & 15)] : 0.f;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int q = 4 * wave + m, r = q / BXT, xt = q % BXT;
      const long v0 = ((long)(z0 + zq) * H + y0 + r) * W + x0 + 16 * xt;
      conv_store<RELU>(acc[m][t], t, v0, lane, bb, V, out_bf, out_f32, cstore);
    }
  }
}

// Taps per wave in the weight gradient: the gradient operand (unshifted) is
// loaded once and used for TG taps; TG * (COUT/16) * (CIN/16) accumulator
// tiles stay within 36.
__host__ __device__ constexpr int wgrad_tg(int cin, int cout, int taps) {
  return taps == 1 ? 1
                   : ((cin / 16) * (cout / 16) * 27 <= 36 ? 27
                                                          : ((cin / 16) * (cout / 16) * 9 <= 36
                                                                 ? 9
                                                                 : ((cin / 16) * (cout / 16) * 3 <= 36 ? 3 : 1)));
}

// Weight gradient partials.  Wave work item = (row chunk c, tap group): the
// wave sums over the rows (z, y) of its chunk and every x,
//   part[c][tap][co][ci] = sum g[z,y,x][co] * in[z+dz, y+dy, x+dx][ci]
// for the TG taps of its group and every (co, ci) tile: a GEMM over voxels
// with A = g^T (co x voxel) and B = the shifted input (voxel x ci).  Rows whose
// shifted row lies outside the grid contribute nothing and are skipped.
template <int CIN, int COUT, int TAPS, int TG>
__global__ void __launch_bounds__(256)
k_wgrad(const uint16_t* __restrict__ in, const uint16_t* __restrict__ g, float* __restrict__ part, int rows_per_chunk,
        int nchunks, int D, int H, int W) {
  constexpr int MT = COUT / 16, NTl = CIN / 16, NG = TAPS / TG;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const long V = (long)D * H * W;
  const int item = blockIdx.x * 4 + wave;
  if (item >= nchunks * NG) return;  // whole wave; no block barrier in this kernel
  const int grp = item % NG, c = item / NG;
  const int r0 = c * rows_per_chunk;
  const int r1 = min(r0 + rows_per_chunk, D * H);
  v4f acc[TG][MT][NTl];
#pragma unroll
  for (int t = 0; t < TG; ++t)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTl; ++nt) acc[t][mt][nt] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int r = r0; r < r1; ++r) {
    const int z = r / H, y = r - (r / H) * H;
    for (int xs = 0; xs < W; xs += 16) {
      const int xl = xs + 4 * kq;  // this lane's voxels are x = xl .. xl + 3 of row r
      v4s a[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          a[mt][e] = (xl + e < W) ? (short)g[((long)mt * V + (long)r * W + xl + e) * 16 + i] : (short)0;
#pragma unroll
      for (int t = 0; t < TG; ++t) {
        int dz, dy, dx;
        tap_offsets(grp * TG + t, TAPS, dz, dy, dx);
        const int zz = z + dz, yy = y + dy;
        if (zz < 0 || zz >= D || yy < 0 || yy >= H) continue;  // uniform across the wave
        const long sb = ((long)zz * H + yy) * W;
#pragma unroll
        for (int nt = 0; nt < NTl; ++nt) {
          v4s b;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int x = xl + e + dx;
            b[e] = (xl + e < W && x >= 0 && x < W) ? (short)in[((long)nt * V + sb + x) * 16 + i] : (short)0;
          }
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            acc[t][mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mt], b, acc[t][mt][nt], 0, 0, 0);
        }
      }
    }
  }
  // lane holds D[co = mt*16 + 4 kq + e][ci = nt*16 + i]
#pragma unroll
  for (int t = 0; t < TG; ++t) {
    float* dst = part + ((long)c * TAPS + grp * TG + t) * (long)COUT * CIN;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTl; ++nt)
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[(mt * 16 + 4 * kq + e) * CIN + nt * 16 + i] = acc[t][mt][nt][e];
  }
}

// Weight gradient of a 3x3x3 convolution as a sweep along y (grids with
// W % 32 == 0).  The activation and the output gradient are first copied from
// the 16-channel planes to voxel-blocked rows: element (c, v) at
// (block(v) C + c) 8 + v % 8, so the 8 consecutive voxels of one channel that a
// lane contributes to a 32-deep product are 16 contiguous bytes and the 16
// channels of an operand 256 contiguous bytes.  The activation copy carries a
// zero plane before and after the grid in z and a zero row before and after
// every plane in y ([(D + 2)][(H + 2)][W / 8][C][8]), so every load of it is in
// bounds and needs no mask; the gradient copy is unpadded ([V / 8][C][8]).
//
// A wave owns one chunk (plane z, 32 voxels of x, a run of rows y) and one
// 16 x 16 tile (gradient channels co, activation channels ci) and accumulates
// all 27 taps,
//   part[chunk][tap][co][ci] = sum_v g[co][v] in[ci][v + off(tap)],
// on v_mfma_f32_16x16x32 bf16 with K = 32 voxels (lane group j of the wave
// takes voxels x0 + 8 j .. + 7; A and B take the same voxel for the same K
// slot, so the sum is right whatever the order of the slots).  The x offset of
// a tap is moved onto the gradient: sum_v g[v] in[v + dx] = sum_u g[u - dx]
// in[u] with g = 0 outside the grid row, so B is always an aligned 16-byte load
// of activation row (z + dz, y + dy) and only the three A operands g[u + 1],
// g[u], g[u - 1] are assembled per step, from one aligned load and the two
// neighbouring dwords, with byte-align operations.  The nine activation rows
// of a step are held in registers as a window over (dz, dy); each step loads
// the three rows y + 2 of planes z - 1, z, z + 1 and the gradient row y + 1 for
// the next step, and four register slots rotate through the unrolled loop.
// With bias the waves of the first activation tile also sum the gradient (one
// more product against a B of ones) into the bias columns of the chunk's
// partial row: part[chunk][27 COUT CIN + co] = sum_v g[co][v].
// Consecutive chunks run along z and the logical blocks are dealt to XCDs in
// contiguous ranges, so the three planes a row is read for share an L2.
__global__ void __launch_bounds__(256) k_to_blocks(const uint16_t* __restrict__ in, uint16_t* __restrict__ out,
                                                   long V, int C) {
  // block: plane p, 128 voxels (16 blocks of 8); LDS rows of 20 u16 per voxel
  __shared__ __align__(16) uint16_t sh[128 * 20];
  const long nb = V / 8;
  const long tiles = (nb + 15) / 16;
  const int np = C / 16;
  for (long t = blockIdx.x; t < tiles * np; t += gridDim.x) {
    const int p = (int)(t % np);
    const long b0 = (t / np) * 16;
    const int tv = threadIdx.x >> 1, half = threadIdx.x & 1;
    const long v = b0 * 8 + tv;
    if (v < V) {
      const uint4 q = *reinterpret_cast<const uint4*>(in + ((long)p * V + v) * 16 + 8 * half);
      uint2* d = reinterpret_cast<uint2*>(sh + tv * 20 + 8 * half);
      d[0] = make_uint2(q.x, q.y);
      d[1] = make_uint2(q.z, q.w);
    }
    __syncthreads();
    const int bl = threadIdx.x >> 4, c = threadIdx.x & 15;
    if (b0 + bl < nb) {
      uint32_t w[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        w[k] = (uint32_t)sh[(8 * bl + 2 * k) * 20 + c] | ((uint32_t)sh[(8 * bl + 2 * k + 1) * 20 + c] << 16);
      *reinterpret_cast<uint4*>(out + (((b0 + bl) * C) + 16 * p + c) * 8) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    __syncthreads();
  }
}

// planes -> zero-padded voxel-blocked rows [(D + 2)][(H + 2)][W / 8][C][8]: the
// interior from the planes, then the zero rows (rows 0 and H + 1 of the D + 2
// planes, rows 1 .. H of planes 0 and D + 1)
__global__ void __launch_bounds__(256) k_to_blocks_padded(const uint16_t* __restrict__ in,
                                                          uint16_t* __restrict__ out, int D, int H, int W, int C) {
  __shared__ __align__(16) uint16_t sh[128 * 20];
  const long V = (long)D * H * W, nb = V / 8;
  const long tiles = (nb + 15) / 16;
  const int np = C / 16, wb = W / 8;
  for (long t = blockIdx.x; t < tiles * np; t += gridDim.x) {
    const int p = (int)(t % np);
    const long b0 = (t / np) * 16;
    const int tv = threadIdx.x >> 1, half = threadIdx.x & 1;
    const long v = b0 * 8 + tv;
    if (v < V) {
      const uint4 q = *reinterpret_cast<const uint4*>(in + ((long)p * V + v) * 16 + 8 * half);
      uint2* d = reinterpret_cast<uint2*>(sh + tv * 20 + 8 * half);
      d[0] = make_uint2(q.x, q.y);
      d[1] = make_uint2(q.z, q.w);
    }
    __syncthreads();
    const int bl = threadIdx.x >> 4, c = threadIdx.x & 15;
    const long b = b0 + bl;
    if (b < nb) {
      uint32_t w[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        w[k] = (uint32_t)sh[(8 * bl + 2 * k) * 20 + c] | ((uint32_t)sh[(8 * bl + 2 * k + 1) * 20 + c] << 16);
      const long zy = b / wb, xb = b - zy * wb;
      const long z = zy / H, y = zy - z * H;
      const long pb = ((z + 1) * (H + 2) + (y + 1)) * wb + xb;
      *reinterpret_cast<uint4*>(out + ((pb * C) + 16 * p + c) * 8) = make_uint4(w[0], w[1], w[2], w[3]);
    }
    __syncthreads();
  }
  const long row = (long)W * C / 8;  // 16-byte units per padded row
  const long nz = (2L * (D + 2) + 2L * H) * row;
  for (long k = blockIdx.x * 256L + threadIdx.x; k < nz; k += (long)gridDim.x * 256) {
    const long r = k / row, e = k - r * row;
    long z, y;
    if (r < 2L * (D + 2)) {
      z = r >> 1;
      y = (r & 1) ? H + 1 : 0;
    } else {
      const long q = r - 2L * (D + 2);
      y = (q >> 1) + 1;
      z = (q & 1) ? D + 1 : 0;
    }
    reinterpret_cast<uint4*>(out + (z * (H + 2) + y) * (long)W * C)[e] = make_uint4(0u, 0u, 0u, 0u);
  }
}

// one step of the y sweep: products of gradient row y with activation rows
// y - 1, y, y + 1 (sm, s0, sp; three planes each) for the 27 taps, and the
// loads of the next step (sn: row y + 2 through xnext, the padded row y + 3
// clamped to the last padded row; gn/pn/nn: gradient row y + 1 through gnext)
template <bool BIAS>
__device__ __forceinline__ void wgrad_roll_step(v4f (&acc)[27], v4f& accb, const uint4 (&sm)[3], const uint4 (&s0)[3],
                                                const uint4 (&sp)[3], uint4 (&sn)[3], const uint4& gc, uint32_t gpv,
                                                uint32_t gnx, uint4& gn, uint32_t& pn, uint32_t& nn,
                                                const uint16_t* __restrict__ xnext, long PZ,
                                                const uint16_t* __restrict__ gnext, int dprev, int dnext,
                                                uint32_t mprev, uint32_t mnext) {
#pragma unroll
  for (int dz = 0; dz < 3; ++dz) sn[dz] = *reinterpret_cast<const uint4*>(xnext + dz * PZ);
  gn = *reinterpret_cast<const uint4*>(gnext);
  pn = *reinterpret_cast<const uint32_t*>(gnext + dprev) & mprev;
  nn = *reinterpret_cast<const uint32_t*>(gnext + dnext) & mnext;
  // gm = g[u + 1] (tap dx = -1), gc = g[u] (dx = 0), gp = g[u - 1] (dx = +1)
  uint4 gm, gp;
  gm.x = __builtin_amdgcn_alignbit(gc.y, gc.x, 16);
  gm.y = __builtin_amdgcn_alignbit(gc.z, gc.y, 16);
  gm.z = __builtin_amdgcn_alignbit(gc.w, gc.z, 16);
  gm.w = __builtin_amdgcn_alignbit(gnx, gc.w, 16);
  gp.x = __builtin_amdgcn_alignbit(gc.x, gpv, 16);
  gp.y = __builtin_amdgcn_alignbit(gc.y, gc.x, 16);
  gp.z = __builtin_amdgcn_alignbit(gc.z, gc.y, 16);
  gp.w = __builtin_amdgcn_alignbit(gc.w, gc.z, 16);
  const v8bf a0 = as_v8bf(gm), a1 = as_v8bf(gc), a2 = as_v8bf(gp);
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const v8bf b = as_v8bf(dy == 0 ? sm[dz] : (dy == 1 ? s0[dz] : sp[dz]));
      const int t = dz * 9 + dy * 3;
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b, acc[t], 0, 0, 0);
      acc[t + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b, acc[t + 1], 0, 0, 0);
      acc[t + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b, acc[t + 2], 0, 0, 0);
    }
  if (BIAS) {
    const uint4 ones = make_uint4(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u);  // bf16 1.0 x 8
    accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, as_v8bf(ones), accb, 0, 0, 0);
  }
}

// partial rows of the weight gradient's sweep: 27 COUT CIN weights, then COUT bias sums
template <int CIN, int COUT> constexpr long wgrad_row_pitch() { return 27L * COUT * CIN + COUT; }

template <int CIN, int COUT, bool BIAS>
__device__ __forceinline__ void wgrad_roll_body(const uint16_t* __restrict__ xp, const uint16_t* __restrict__ gb,
                                                float* __restrict__ part, int chunk, int nt, int mt, int ny, int D,
                                                int H, int W) {
  const int lane = threadIdx.x & 63, i = lane & 15, j = lane >> 4;
  const int nxs = W / 32;
  const int z = chunk % D, xs = (chunk / D) % nxs, yp = chunk / (D * nxs);
  const int y0 = yp * ny, y1 = min(y0 + ny, H);
  const int x0 = xs * 32 + 8 * j;
  const int xoff = x0 * CIN + (nt * 16 + i) * 8;   // lane's element offset within an activation row
  const int goff = x0 * COUT + (mt * 16 + i) * 8;  // and within a gradient row
  const int dprev = x0 == 0 ? 0 : -COUT * 8 + 6, dnext = x0 + 8 == W ? 0 : COUT * 8;
  const uint32_t mprev = x0 == 0 ? 0u : ~0u, mnext = x0 + 8 == W ? 0u : ~0u;
  const long PY = (long)W * CIN, PZ = (long)(H + 2) * PY, GY = (long)W * COUT;
  v4f acc[27], accb = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  // padded plane z is grid plane z - 1; padded row y is grid row y - 1
  const uint16_t* xz = xp + (long)z * PZ + xoff;
  uint4 S0[3], S1[3], S2[3], S3[3];
  {
    const long r0 = (long)min(y0, H + 1) * PY, r1 = (long)min(y0 + 1, H + 1) * PY, r2 = (long)min(y0 + 2, H + 1) * PY;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz) {
      S0[dz] = *reinterpret_cast<const uint4*>(xz + dz * PZ + r0);
      S1[dz] = *reinterpret_cast<const uint4*>(xz + dz * PZ + r1);
      S2[dz] = *reinterpret_cast<const uint4*>(xz + dz * PZ + r2);
    }
  }
  const uint16_t* gz = gb + (long)z * H * GY + goff;
  const uint16_t* g0 = gz + (long)min(y0, H - 1) * GY;
  uint4 G0 = *reinterpret_cast<const uint4*>(g0), G1;
  uint32_t P0 = *reinterpret_cast<const uint32_t*>(g0 + dprev) & mprev, P1;
  uint32_t N0 = *reinterpret_cast<const uint32_t*>(g0 + dnext) & mnext, N1;
#define USP_WG_STEP(SM, S0_, SP, SN, GC, PC, NC, GN, PN, NN, YY)                                                   \
  wgrad_roll_step<BIAS>(acc, accb, SM, S0_, SP, SN, GC, PC, NC, GN, PN, NN, xz + (long)min((YY) + 3, H + 1) * PY, PZ, \
                        gz + (long)min((YY) + 1, H - 1) * GY, dprev, dnext, mprev, mnext)
  for (int y = y0; y < y1; y += 4) {
    USP_WG_STEP(S0, S1, S2, S3, G0, P0, N0, G1, P1, N1, y);
    if (y + 1 < y1) USP_WG_STEP(S1, S2, S3, S0, G1, P1, N1, G0, P0, N0, y + 1);
    if (y + 2 < y1) USP_WG_STEP(S2, S3, S0, S1, G0, P0, N0, G1, P1, N1, y + 2);
    if (y + 3 < y1) USP_WG_STEP(S3, S0, S1, S2, G1, P1, N1, G0, P0, N0, y + 3);
  }
#undef USP_WG_STEP
  // lane holds D[co = mt*16 + 4 j + e][ci = nt*16 + i]
  float* row = part + (long)chunk * wgrad_row_pitch<CIN, COUT>();
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    float* dst = row + t * COUT * CIN;
#pragma unroll
    for (int e = 0; e < 4; ++e) dst[(mt * 16 + 4 * j + e) * CIN + nt * 16 + i] = acc[t][e];
  }
  if (BIAS && i == 0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) row[27 * COUT * CIN + mt * 16 + 4 * j + e] = accb[e];
  }
}

// work item = (chunk, co tile mt, ci tile nt), nt fastest; chunk = (y part, x segment, z), z fastest.
// Logical block L = 4 items; the launch has a multiple of 8 blocks and block b runs logical block
// (b % 8) (grid / 8) + b / 8, so each XCD takes a contiguous range of chunks.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256)
k_wgrad_roll(const uint16_t* __restrict__ xp, const uint16_t* __restrict__ gb, float* __restrict__ part, int bias,
             int ny, int nchunks, int D, int H, int W, int nlog) {
  constexpr int NT = CIN / 16, MT = COUT / 16, NS = NT * MT;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int per = gridDim.x / 8;
  const int L = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (L >= nlog) return;
  const int item = L * 4 + wave;
  if (item >= nchunks * NS) return;  // whole wave; no block barrier in this kernel
  const int chunk = item / NS, sub = item % NS, nt = sub % NT, mt = sub / NT;
  if (bias && nt == 0)
    wgrad_roll_body<CIN, COUT, true>(xp, gb, part, chunk, nt, mt, ny, D, H, W);
  else
    wgrad_roll_body<CIN, COUT, false>(xp, gb, part, chunk, nt, mt, ny, D, H, W);
}

// dw[co][tap][ci] = sum over chunks c of part[c][tap][co][ci] (and, for
// columns past the weights, db[co] = sum over c of part[c][n + co]), in two
// passes with a fixed order: pass 1 sums the chunks of segment s (seg
// consecutive chunks, in increasing order) into seg_sum[s][j]; pass 2 adds the
// segments in increasing order.  Partial rows are `pitch` floats apart, the
// first ncols of each are reduced; j = (tap cout + co) cin + ci for j < n.
__global__ void __launch_bounds__(256)
k_wgrad_reduce_seg(const float* __restrict__ part, long pitch, float* __restrict__ seg_sum, int nchunks, int seg,
                   long ncols) {
  const long j = (long)blockIdx.x * 256 + threadIdx.x;
  if (j >= ncols) return;
  const int c0 = blockIdx.y * seg, c1 = min(c0 + seg, nchunks);
  // loads issued eight at a time, added in chunk order
  float s = 0.f;
  int c = c0;
  for (; c + 8 <= c1; c += 8) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = part[(long)(c + k) * pitch + j];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
  }
  for (; c < c1; ++c) s += part[(long)c * pitch + j];
  seg_sum[(long)blockIdx.y * ncols + j] = s;
}
__global__ void __launch_bounds__(256)
k_wgrad_reduce_fin(const float* __restrict__ seg_sum, long ncols, float* __restrict__ dw, float* __restrict__ db,
                   int nseg, int taps, int cout, int cin) {
  const long n = (long)taps * cout * cin;
  const long j = (long)blockIdx.x * 256 + threadIdx.x;
  if (j >= ncols) return;
  float t = 0.f;
  int q = 0;
  for (; q + 8 <= nseg; q += 8) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = seg_sum[(long)(q + k) * ncols + j];
#pragma unroll
    for (int k = 0; k < 8; ++k) t += v[k];
  }
  for (; q < nseg; ++q) t += seg_sum[(long)q * ncols + j];
  if (j >= n) {
    db[j - n] = t;
    return;
  }
  const int tap = (int)(j / ((long)cout * cin)), co = (int)((j / cin) % cout), ci = (int)(j % cin);
  dw[((long)co * taps + tap) * cin + ci] = t;
}

__device__ __forceinline__ void unpack8(uint4 q, float* f) {
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    f[2 * k] = __uint_as_float(w[k] << 16);
    f[2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
  }
}
__device__ __forceinline__ uint4 pack8(const float* f) {
  uint32_t w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = (uint32_t)f2bf(f[2 * k]) | ((uint32_t)f2bf(f[2 * k + 1]) << 16);
  return uint4{w[0], w[1], w[2], w[3]};
}

// Bias gradient partials: part[b][p*16 + c] = sum over the chunk's voxels of
// g(v, p*16 + c); grid (chunks, planes), 256 threads = 128 voxel lanes x 2
// halves of 8 channels (16-byte loads); lane sums combined in order.
__global__ void __launch_bounds__(256)
k_bgrad(const uint16_t* __restrict__ g, float* __restrict__ part, long V, int C, int chunk) {
  __shared__ float sh[128][17];
  const int half = threadIdx.x & 1, vl = threadIdx.x >> 1, p = blockIdx.y;
  const long v0 = (long)blockIdx.x * chunk;
  const long v1 = v0 + chunk < V ? v0 + chunk : V;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (long v = v0 + vl; v < v1; v += 128) {
    float f[8];
    unpack8(*reinterpret_cast<const uint4*>(g + ((long)p * V + v) * 16 + 8 * half), f);
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] += f[k];
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) sh[vl][8 * half + k] = s[k];
  __syncthreads();
  if (threadIdx.x < 16) {
    float t = 0.f;
    for (int q = 0; q < 128; ++q) t += sh[q][threadIdx.x];
    part[(long)blockIdx.x * C + p * 16 + threadIdx.x] = t;
  }
}
// db[co] = sum over chunks (one block per channel, lanes strided over chunks, then in order)
__global__ void __launch_bounds__(256)
k_bgrad_reduce(const float* __restrict__ part, float* __restrict__ db, int nchunks, int C) {
  __shared__ float sh[256];
  const int co = blockIdx.x;
  float s = 0.f;
  for (int c = threadIdx.x; c < nchunks; c += 256) s += part[(long)c * C + co];
  sh[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int q = 0; q < 256; ++q) t += sh[q];
    db[co] = t;
  }
}

// ---- pooling, upsampling, copies: 8 channels (16 bytes) per thread ----------
// 2x2x2 average pooling (fine D x H x W -> coarse), per plane.
__global__ void k_pool2(const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int D, int H, int W, int C) {
  const int Do = D / 2, Ho = H / 2, Wo = W / 2;
  const long V = (long)D * H * W, Vo = (long)Do * Ho * Wo;
  const long n = (C / 16) * Vo * 2;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    const int half = (int)(j & 1);
    const long r = j >> 1;
    const long vo = r % Vo;
    const int p = (int)(r / Vo);
    const int xo = (int)(vo % Wo), yo = (int)((vo / Wo) % Ho), zo = (int)(vo / ((long)Wo * Ho));
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int d = 0; d < 8; ++d) {
      const long vi = ((long)(2 * zo + (d >> 2)) * H + (2 * yo + ((d >> 1) & 1))) * W + (2 * xo + (d & 1));
      float f[8];
      unpack8(*reinterpret_cast<const uint4*>(in + ((long)p * V + vi) * 16 + 8 * half), f);
#pragma unroll
      for (int k = 0; k < 8; ++k) s[k] += f[k];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] *= 0.125f;
    *reinterpret_cast<uint4*>(out + ((long)p * Vo + vo) * 16 + 8 * half) = pack8(s);
  }
}
// gradient of k_pool2: fine = coarse parent / 8
__global__ void k_pool2_back(const uint16_t* __restrict__ gout, uint16_t* __restrict__ gin, int D, int H, int W,
                             int C) {
  const int Ho = H / 2, Wo = W / 2;
  const long V = (long)D * H * W, Vo = (long)(D / 2) * Ho * Wo;
  const long n = (C / 16) * V * 2;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    const int half = (int)(j & 1);
    const long r = j >> 1;
    const long v = r % V;
    const int p = (int)(r / V);
    const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)(v / ((long)W * H));
    const long vo = ((long)(z / 2) * Ho + y / 2) * Wo + x / 2;
    float f[8];
    unpack8(*reinterpret_cast<const uint4*>(gout + ((long)p * Vo + vo) * 16 + 8 * half), f);
#pragma unroll
    for (int k = 0; k < 8; ++k) f[k] *= 0.125f;
    *reinterpret_cast<uint4*>(gin + ((long)p * V + v) * 16 + 8 * half) = pack8(f);
  }
}
// Nearest upsampling: out (fine grid D x H x W, planes c0/16 ..) = in (coarse,
// C channels) at (z/2, y/2, x/2).
__global__ void k_up2(const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int D, int H, int W, int C, int c0) {
  const int Ho = H / 2, Wo = W / 2;
  const long V = (long)D * H * W, Vo = (long)(D / 2) * Ho * Wo;
  const long n = (C / 16) * V * 2;
  const int p0 = c0 / 16;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    const int half = (int)(j & 1);
    const long r = j >> 1;
    const long v = r % V;
    const int p = (int)(r / V);
    const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)(v / ((long)W * H));
    const long vo = ((long)(z / 2) * Ho + y / 2) * Wo + x / 2;
    *reinterpret_cast<uint4*>(out + ((long)(p0 + p) * V + v) * 16 + 8 * half) =
        *reinterpret_cast<const uint4*>(in + ((long)p * Vo + vo) * 16 + 8 * half);
  }
}
// gradient of k_up2: coarse = sum of the 8 fine children (planes c0/16 .. of gfine)
__global__ void k_up2_back(const uint16_t* __restrict__ gfine, uint16_t* __restrict__ gcoarse, int D, int H, int W,
                           int C, int c0) {
  const int Do = D / 2, Ho = H / 2, Wo = W / 2;
  const long V = (long)D * H * W, Vo = (long)Do * Ho * Wo;
  const long n = (C / 16) * Vo * 2;
  const int p0 = c0 / 16;
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
    const int half = (int)(j & 1);
    const long r = j >> 1;
    const long vo = r % Vo;
    const int p = (int)(r / Vo);
    const int xo = (int)(vo % Wo), yo = (int)((vo / Wo) % Ho), zo = (int)(vo / ((long)Wo * Ho));
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int d = 0; d < 8; ++d) {
      const long vi = ((long)(2 * zo + (d >> 2)) * H + (2 * yo + ((d >> 1) & 1))) * W + (2 * xo + (d & 1));
      float f[8];
      unpack8(*reinterpret_cast<const uint4*>(gfine + ((long)(p0 + p) * V + vi) * 16 + 8 * half), f);
#pragma unroll
      for (int k = 0; k < 8; ++k) s[k] += f[k];
    }
    *reinterpret_cast<uint4*>(gcoarse + ((long)p * Vo + vo) * 16 + 8 * half) = pack8(s);
  }
}
// contiguous copy of n8 * 8 bf16 (whole planes)
__global__ void k_copy8(const uint4* __restrict__ src, uint4* __restrict__ dst, long n8) {
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n8; j += (long)gridDim.x * blockDim.x) dst[j] = src[j];
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

// The same two element-wise operations on 8 bf16 values (16 bytes) per thread
// and access, for 16-byte aligned operands and n % 8 == 0 (n8 = n / 8).
__global__ void k_relu_back8(const uint4* __restrict__ y, const uint4* __restrict__ g, uint4* __restrict__ out,
                             long n8, int accumulate) {
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n8; j += (long)gridDim.x * blockDim.x) {
    float fy[8], fg[8], fo[8];
    unpack8(y[j], fy);
    unpack8(g[j], fg);
    if (accumulate) unpack8(out[j], fo);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float v = fy[k] > 0.f ? fg[k] : 0.f;
      fo[k] = accumulate ? fo[k] + v : v;
    }
    out[j] = pack8(fo);
  }
}
__global__ void k_add_bf8(uint4* __restrict__ dst, const uint4* __restrict__ src, long n8) {
  for (long j = blockIdx.x * (long)blockDim.x + threadIdx.x; j < n8; j += (long)gridDim.x * blockDim.x) {
    float a[8], b[8];
    unpack8(dst[j], a);
    unpack8(src[j], b);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] += b[k];
    dst[j] = pack8(a);
  }
}

// Network input from the complex refractive index n + i kappa (one plane of
// 16 channels): channel 0 (Re n - n_bg)/n_span, channel 1 kappa/kappa_max,
// channel 2 the source plane indicator (z == plane), channels 3, 4 the real
// and imaginary parts of the source's Gaussian beam amp(x, y) =
// exp(-((x - W/2)^2 + (y - H/2)^2)/w0^2) carried along z with the phase and
// attenuation of the medium, exp(i k0h sum (n + i kappa)) (trapezoid between
// neighbouring planes, from the source plane up and down), channels 5..15
// zero.  The path sums are in double, the phase is reduced to [-pi, pi] in
// double before the float sine/cosine.
__device__ __forceinline__ void feature_row(uint16_t* o, float2 q, bool on_plane, float amp, double pr, double pi,
                                            double k0h, double n_bg, double n_span, double kappa_max) {
  const float a = amp * expf((float)(-k0h * pi));
  const double t = k0h * pr;
  const float ph = (float)(t - 6.283185307179586 * rint(t * 0.15915494309189535));
  float sn, cs;
  sincosf(ph, &sn, &cs);
  float f[8] = {(float)((q.x - n_bg) / n_span), (float)(q.y / kappa_max), on_plane ? 1.f : 0.f, a * cs, a * sn,
                0.f, 0.f, 0.f};
  uint4* w = reinterpret_cast<uint4*>(o);
  w[0] = pack8(f);
  w[1] = uint4{0u, 0u, 0u, 0u};
}
// One block: kFeatCols (x, y) columns x kFeatSeg segments of z.  The path sums
// are P(z) - P(plane) with P(z) the running trapezoid sum from z = 0: each
// thread sums its segment, the segment sums are scanned through LDS (and P at
// the source plane taken from its segment), then each thread walks its
// segment again writing the features.
constexpr int kFeatCols = 32, kFeatSeg = 8;
__global__ void __launch_bounds__(kFeatCols * kFeatSeg)
k_features(const float2* __restrict__ nidx, uint16_t* __restrict__ out, int D, int H, int W, double n_bg,
           double n_span, double kappa_max, int plane, double k0h, double w0) {
  __shared__ double segsum[kFeatSeg][kFeatCols][2];
  __shared__ double pplane[kFeatCols][2];
  const long cols = (long)H * W;
  const int c = threadIdx.x % kFeatCols, sg = threadIdx.x / kFeatCols;
  const long col = (long)blockIdx.x * kFeatCols + c;
  const bool act = col < cols;
  const int L = (D + kFeatSeg - 1) / kFeatSeg;
  const int z0 = sg * L, z1 = min(D, z0 + L);
  // trapezoid term of plane w >= 1: (n[w - 1] + n[w]) / 2
  auto term = [&](int w, double& tr, double& ti) {
    const float2 a = nidx[(long)(w - 1) * cols + col], b = nidx[(long)w * cols + col];
    tr = 0.5 * ((double)a.x + b.x);
    ti = 0.5 * ((double)a.y + b.y);
  };
  double sr = 0.0, si = 0.0;
  if (act) {
    for (int w = max(z0, 1); w < z1; ++w) {
      double tr, ti;
      term(w, tr, ti);
      sr += tr;
      si += ti;
      if (w == plane) {   // P(plane) - P(z0 - 1 .. ) of this segment
        pplane[c][0] = sr;
        pplane[c][1] = si;
      }
    }
  }
  if (plane == 0 && sg == 0) {
    pplane[c][0] = 0.0;
    pplane[c][1] = 0.0;
  }
  segsum[sg][c][0] = sr;
  segsum[sg][c][1] = si;
  __syncthreads();
  double p0r = 0.0, p0i = 0.0;   // P before this segment
  for (int k = 0; k < sg; ++k) {
    p0r += segsum[k][c][0];
    p0i += segsum[k][c][1];
  }
  const int spl = plane / L;     // segment holding the source plane
  double ppr = 0.0, ppi = 0.0;
  for (int k = 0; k < spl; ++k) {
    ppr += segsum[k][c][0];
    ppi += segsum[k][c][1];
  }
  if (plane > 0 && max(spl * L, 1) <= plane) {
    ppr += pplane[c][0];
    ppi += pplane[c][1];
  }
  if (!act) return;
  const double dx = (double)(col % W) - 0.5 * W, dy = (double)(col / W) - 0.5 * H;
  const float amp = (float)exp(-(dx * dx + dy * dy) / (w0 * w0));
  double Pr = p0r, Pi = p0i;
  for (int z = z0; z < z1; ++z) {
    if (z >= 1) {
      double tr, ti;
      term(z, tr, ti);
      Pr += tr;
      Pi += ti;
    }
    const double sgn = z >= plane ? 1.0 : -1.0;
    feature_row(out + ((long)z * cols + col) * 16, nidx[(long)z * cols + col], z == plane, amp, sgn * (Pr - ppr),
                sgn * (Pi - ppi), k0h, n_bg, n_span, kappa_max);
  }
}

// Relative L2 loss between the prediction p[v][0..1] (fp32, Re/Im scaled by
// 1/s) and the target field x[v] (complex64): per-block partials of
// |s p - x|^2 and |x|^2; the gradient g (one plane of 16 channels, zero beyond
// 2) = 2 s (s p - x) / ||x||^2 is written by k_loss_grad once ||x||^2 is known.
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
// one block of 256: lane sums over blocks q = lane, lane + 256, ..., then in order
__global__ void k_loss_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double sh[2][256];
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nb; q += blockDim.x) {
    a += part[2 * q];
    b += part[2 * q + 1];
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int q = 0; q < (int)blockDim.x; ++q) {
      sa += sh[0][q];
      sb += sh[1][q];
    }
    out[0] = sa / sb;  // relative squared error
    out[1] = sb;
  }
}
__global__ void k_loss_grad(const float* __restrict__ p, const float2* __restrict__ x, float s, long V,
                            const double* __restrict__ lossv, uint16_t* __restrict__ g) {
  const float scale = (float)(2.0 * s / lossv[1]);
  for (long v = blockIdx.x * (long)blockDim.x + threadIdx.x; v < V; v += (long)gridDim.x * blockDim.x) {
    float f[8] = {scale * (s * p[2 * v] - x[v].x), scale * (s * p[2 * v + 1] - x[v].y), 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    uint4* o = reinterpret_cast<uint4*>(g + v * 16);
    o[0] = pack8(f);
    o[1] = uint4{0u, 0u, 0u, 0u};
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

// fp32 -> bf16
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
