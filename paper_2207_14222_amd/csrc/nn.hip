// C ABI of the learned-initial-guess network kernels (nn.hpp): convolution
// forward / input gradient / weight gradient on the matrix cores, pooling,
// upsampling, channel copies, ReLU gradient, loss, Adam and conversions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/usp.h"
#include "nn.hpp"
#include "op.hpp"

using namespace usp;

namespace {

inline int grid_for(long n, int bs = 256) { return (int)std::min<long>((n + bs - 1) / bs, 65536); }

// shapes used by the network (cin, cout) for 3x3x3 and the 1x1x1 head
template <class F>
bool with_conv_shape(int cin, int cout, int taps, F&& f) {
#define USP_CASE(CI, CO, TP)                                                                  \
  if (cin == CI && cout == CO && taps == TP) {                                               \
    f(std::integral_constant<int, CI>{}, std::integral_constant<int, CO>{}, std::integral_constant<int, TP>{}); \
    return true;                                                                              \
  }
  USP_CASE(16, 16, 27)
  USP_CASE(16, 32, 27)
  USP_CASE(32, 16, 27)
  USP_CASE(32, 32, 27)
  USP_CASE(32, 64, 27)
  USP_CASE(64, 32, 27)
  USP_CASE(64, 64, 27)
  USP_CASE(64, 128, 27)
  USP_CASE(128, 64, 27)
  USP_CASE(192, 64, 27)
  USP_CASE(64, 192, 27)
  USP_CASE(96, 32, 27)
  USP_CASE(32, 96, 27)
  USP_CASE(48, 16, 27)
  USP_CASE(16, 48, 27)
  USP_CASE(16, 16, 1)
#undef USP_CASE
  return false;
}

// Row chunking of the weight gradient: about 4096 waves, partials within 128 MiB.
struct WgradSplit {
  int rows_per_chunk, nchunks, tg;
};
WgradSplit wgrad_split(int D, int H, int cin, int cout, int taps) {
  const int tg = wgrad_tg(cin, cout, taps);
  const int ng = taps / tg;
  const long R = (long)D * H;
  long nch = std::min<long>(R, std::max<long>(1, (4096 + ng - 1) / ng));
  long rpc = (R + nch - 1) / nch;
  nch = (R + rpc - 1) / rpc;
  while (nch > 1 && nch * taps * (long)cout * cin * 4 > (128l << 20)) {
    rpc *= 2;
    nch = (R + rpc - 1) / rpc;
  }
  return {(int)rpc, (int)nch, tg};
}

// The y-sweep weight gradient (k_wgrad_roll) serves 3x3x3 convolutions on
// grids with W % 32 == 0: chunks = (plane, 32 voxels of x, a run of ny rows),
// one wave per chunk and 16 x 16 channel tile.  The rows are split into the
// fewest runs that give at least 1536 waves (six per CU; the kernel holds two
// per SIMD), with partials within 128 MiB.
struct RollSplit {
  bool use;
  int ny, nchunks;
};
RollSplit roll_split(int D, int H, int W, int cin, int cout, int taps) {
  if (taps != 27 || W % 32) return {false, 0, 0};
  const long tiles = (long)(cin / 16) * (cout / 16);
  const long base = (long)D * (W / 32);
  auto part_bytes = [&](long nyp) { return nyp * base * 27L * cout * cin * 4; };
  long nyp = 1;
  while (nyp * base * tiles < 1536 && nyp * 2 <= H && part_bytes(nyp * 2) <= (128l << 20)) nyp *= 2;
  const long ny = (H + nyp - 1) / nyp;
  nyp = (H + ny - 1) / ny;
  if (nyp * base * tiles >= (1l << 31)) return {false, 0, 0};
  return {true, (int)ny, (int)(nyp * base)};
}
// bytes of the zero-padded activation copy and of the gradient copy
long xpad_bytes(int D, int H, int W, int cin) { return (long)align_up(2L * (D + 2) * (H + 2) * W * cin); }
long gblk_bytes(long V, int cout) { return (long)align_up(2 * V * (long)cout); }

// Segments of the two-pass partial reduction: about 2048 blocks of 256 outputs
// in pass 1, at most kMaxSeg segments.
constexpr int kMaxSeg = 64;
struct SegPlan {
  int seg, nseg;
};
SegPlan seg_plan(int nchunks, long n) {
  const long cols = (n + 255) / 256;
  long nseg = std::min<long>(std::min<long>(kMaxSeg, nchunks), std::max<long>(1, (2048 + cols - 1) / cols));
  const long seg = (nchunks + nseg - 1) / nseg;
  nseg = (nchunks + seg - 1) / seg;
  return {(int)seg, (int)nseg};
}

constexpr long kBiasChunk = 4096;

bool planes_ok(int c) { return c > 0 && c % 16 == 0; }
bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

extern "C" {

int usp_nn_pack_weights(const void* w, void* packed, int cout, int taps, int cin, int transposed, void* stream) {
  if (!w || !packed || !planes_ok(cin) || !planes_ok(cout) || (taps != 1 && taps != 27))
    return fail(USP_ERR_INVALID, "invalid argument");
  const long n = (taps == 27 ? 28L : 1L) * cin * cout;
  hipLaunchKernelGGL(k_wpack, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, (const uint16_t*)w,
                     (uint16_t*)packed, cout, taps, cin, transposed ? 1 : 0);
  LAUNCHCHK("k_wpack");
  return 0;
}

int usp_nn_conv3d(const void* in, const void* wpk, const float* bias, void* out, int out_f32, int cstore, int D, int H,
                  int W, int cin, int cout, int taps, int sign, int relu, void* stream) {
  if (!in || !wpk || !out || D < 1 || H < 1 || W < 1 || cstore < 1 || cstore > cout || (sign != 1 && sign != -1))
    return fail(USP_ERR_INVALID, "invalid argument");
  if (!out_f32 && cstore != cout) return fail(USP_ERR_INVALID, "bf16 output keeps every output channel");
  const long V = (long)D * H * W;
  if (V % 16 || V > (1l << 30)) return fail(USP_ERR_UNSUPPORTED_SHAPE, "the voxel count must be a multiple of 16");
  if (sign < 0 && relu) return fail(USP_ERR_INVALID, "the input-gradient convolution takes no ReLU");
  hipStream_t st = (hipStream_t)stream;
  uint16_t* ob = out_f32 ? nullptr : (uint16_t*)out;
  float* of = out_f32 ? (float*)out : nullptr;
  const uint16_t* ip = (const uint16_t*)in;
  const bool big = V >= (1l << 18);
  // schedule: LDS-staged bricks on large grids whose sides fit the brick, else operands from global memory
  const int bxt = !big ? 0 : (W % 64 == 0 && H % 4 == 0) ? 4 : (W % 16 == 0 && H % 16 == 0) ? 1 : 0;
  // two output z-planes per brick for 16 input channels where the grid keeps
  // about 4096 bricks or more (measured at 128^3: 16 -> 16 60 -> 51 us, its
  // input gradient 62 -> 55 us, 16 -> 48 input gradient 131 -> 122 us; with
  // 48 input channels 147 -> 197 us, so those keep one plane)
  const bool zb2 = bxt == 4 && cin == 16 && D % 2 == 0 && V >= (1l << 21);
  bool ok = with_conv_shape(cin, cout, taps, [&](auto CI, auto CO, auto TP) {
    constexpr int ci = decltype(CI)::value, co = decltype(CO)::value, tp = decltype(TP)::value;
    auto launch = [&](auto SG, auto RL) {
      constexpr int sg = decltype(SG)::value;
      constexpr bool rl = decltype(RL)::value;
      if constexpr (tp == 1) {
        const uint2* wp = (const uint2*)wpk;
        if (big)
          hipLaunchKernelGGL((k_conv<ci, co, 1, sg, rl, 4>), dim3((unsigned)((V + 255) / 256)), dim3(256), 0, st, ip,
                             wp, bias, ob, of, cstore, D, H, W);
        else
          hipLaunchKernelGGL((k_conv<ci, co, 1, sg, rl, 1>), dim3((unsigned)((V + 63) / 64)), dim3(256), 0, st, ip,
                             wp, bias, ob, of, cstore, D, H, W);
      } else {
        const uint4* wp = (const uint4*)wpk;
        if constexpr (ci == 16) {
          if (zb2) {
            hipLaunchKernelGGL((k_conv_lds<ci, co, sg, rl, 4, 2>), dim3((unsigned)(V / 512)), dim3(512), 0, st, ip,
                               wp, bias, ob, of, cstore, D, H, W);
            return;
          }
        }
        if (bxt == 4)
          hipLaunchKernelGGL((k_conv_lds<ci, co, sg, rl, 4>), dim3((unsigned)(V / 256)), dim3(256), 0, st, ip, wp, bias,
                             ob, of, cstore, D, H, W);
        else if (bxt == 1)
          hipLaunchKernelGGL((k_conv_lds<ci, co, sg, rl, 1>), dim3((unsigned)(V / 256)), dim3(256), 0, st, ip, wp, bias,
                             ob, of, cstore, D, H, W);
        else if (big)
          hipLaunchKernelGGL((k_conv27<ci, co, sg, rl, 4>), dim3((unsigned)((V + 255) / 256)), dim3(256), 0, st, ip,
                             wp, bias, ob, of, cstore, D, H, W);
        else {
          // small grids: split the output tiles over up to 8 blocks until
          // there are about 2048 blocks (measured on the 32^3 and 16^3
          // levels: 4 / 1024 gave 0.673 -> 0.645 ms per forward, 8 / 2048 0.637)
          const long nb = (V + 63) / 64;
          int ts = 1;
          while (ts < 8 && nb * ts < 2048 && (co / 16) % (2 * ts) == 0) ts *= 2;
          auto go = [&](auto TSC) {
            constexpr int tsv = decltype(TSC)::value;
            if constexpr ((co / 16) % tsv == 0)
              hipLaunchKernelGGL((k_conv27<ci, co, sg, rl, 1, tsv>), dim3((unsigned)nb, tsv), dim3(256), 0, st, ip,
                                 wp, bias, ob, of, cstore, D, H, W);
          };
          if (ts == 8) go(std::integral_constant<int, 8>{});
          else if (ts == 4) go(std::integral_constant<int, 4>{});
          else if (ts == 2) go(std::integral_constant<int, 2>{});
          else go(std::integral_constant<int, 1>{});
        }
      }
    };
    using P1 = std::integral_constant<int, 1>;
    using M1 = std::integral_constant<int, -1>;
    using T = std::true_type;
    using F = std::false_type;
    if (sign > 0) {
      if (relu) launch(P1{}, T{});
      else launch(P1{}, F{});
    } else {
      launch(M1{}, F{});
    }
  });
  if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "convolution shape not instantiated");
  LAUNCHCHK("k_conv");
  return 0;
}

int usp_nn_wgrad_workspace(int D, int H, int W, int cin, int cout, int taps, size_t* bytes) {
  if (!bytes || D < 1 || H < 1 || W < 1 || !planes_ok(cin) || !planes_ok(cout) || (taps != 1 && taps != 27))
    return fail(USP_ERR_INVALID, "invalid argument");
  const long V = (long)D * H * W;
  const RollSplit rs = roll_split(D, H, W, cin, cout, taps);
  if (rs.use) {
    // partial rows of 27 cout cin weights + cout bias sums, and the segment sums of the reduction
    const long pitch = 27L * cout * cin + cout;
    *bytes = xpad_bytes(D, H, W, cin) + gblk_bytes(V, cout) + sizeof(float) * ((long)rs.nchunks + kMaxSeg) * pitch +
             256;
    return 0;
  }
  const WgradSplit sp = wgrad_split(D, H, cin, cout, taps);
  const long bch = (V + kBiasChunk - 1) / kBiasChunk;
  *bytes = sizeof(float) * ((long)sp.nchunks * taps * cout * cin + bch * (long)cout + (long)kMaxSeg * taps * cout * cin) +
           256;
  return 0;
}

int usp_nn_conv3d_wgrad(const void* in, const void* g, float* dw, float* db, void* ws, size_t ws_bytes, int D, int H,
                        int W, int cin, int cout, int taps, void* stream) {
  if (!in || !g || !dw || !ws) return fail(USP_ERR_INVALID, "invalid argument");
  size_t need = 0;
  if (usp_nn_wgrad_workspace(D, H, W, cin, cout, taps, &need)) return USP_ERR_INVALID;
  if (ws_bytes < need) return fail(USP_ERR_WORKSPACE, "wgrad workspace too small");
  const long V = (long)D * H * W;
  const RollSplit rs = roll_split(D, H, W, cin, cout, taps);
  const WgradSplit sp = wgrad_split(D, H, cin, cout, taps);
  const int nch = rs.use ? rs.nchunks : sp.nchunks;
  hipStream_t st = (hipStream_t)stream;
  // workspace: y sweep: padded activation copy, gradient copy, partial rows (weights and bias sums),
  // segment sums; row chunks: weight partials, bias partials, segment sums
  const long n = (long)taps * cout * cin;
  const long pitch = rs.use ? n + cout : n;             // floats between partial rows
  const long ncols = rs.use && db ? n + cout : n;       // columns the reduction adds up
  uint16_t* xp = (uint16_t*)ws;
  uint16_t* gb = (uint16_t*)((char*)ws + (rs.use ? xpad_bytes(D, H, W, cin) : 0));
  float* part = (float*)((char*)ws + (rs.use ? xpad_bytes(D, H, W, cin) + gblk_bytes(V, cout) : 0));
  const long bch = (V + kBiasChunk - 1) / kBiasChunk;   // bias chunks of the row-chunk path
  float* bpart = part + (long)nch * pitch;               // row-chunk path only
  float* seg_sum = rs.use ? bpart : bpart + bch * cout;
  bool ok = with_conv_shape(cin, cout, taps, [&](auto CI, auto CO, auto TP) {
    constexpr int ci = decltype(CI)::value, co = decltype(CO)::value, tp = decltype(TP)::value;
    if constexpr (tp == 27) {
      if (rs.use) {
        const long tiles = (V / 8 + 15) / 16;
        hipLaunchKernelGGL(k_to_blocks_padded, dim3((unsigned)std::min<long>(tiles * (ci / 16), 1l << 20)), dim3(256),
                           0, st, (const uint16_t*)in, xp, D, H, W, ci);
        hipLaunchKernelGGL(k_to_blocks, dim3((unsigned)std::min<long>(tiles * (co / 16), 1l << 20)), dim3(256), 0,
                           st, (const uint16_t*)g, gb, V, co);
        const long items = (long)rs.nchunks * (ci / 16) * (co / 16);
        const int nlog = (int)((items + 3) / 4);
        hipLaunchKernelGGL((k_wgrad_roll<ci, co>), dim3((unsigned)((nlog + 7) / 8 * 8)), dim3(256), 0, st, xp, gb,
                           part, db ? 1 : 0, rs.ny, rs.nchunks, D, H, W, nlog);
        return;
      }
    }
    constexpr int tg = wgrad_tg(ci, co, tp);
    const long items = (long)sp.nchunks * (tp / tg);
    hipLaunchKernelGGL((k_wgrad<ci, co, tp, tg>), dim3((unsigned)((items + 3) / 4)), dim3(256), 0, st,
                       (const uint16_t*)in, (const uint16_t*)g, part, sp.rows_per_chunk, sp.nchunks, D, H, W);
  });
  if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "convolution shape not instantiated");
  const SegPlan sg = seg_plan(nch, ncols);
  hipLaunchKernelGGL(k_wgrad_reduce_seg, dim3((unsigned)((ncols + 255) / 256), sg.nseg), dim3(256), 0, st, part,
                     pitch, seg_sum, nch, sg.seg, ncols);
  hipLaunchKernelGGL(k_wgrad_reduce_fin, dim3((unsigned)((ncols + 255) / 256)), dim3(256), 0, st, seg_sum, ncols, dw,
                     db, sg.nseg, taps, cout, cin);
  if (db && !rs.use) {
    hipLaunchKernelGGL(k_bgrad, dim3((unsigned)bch, cout / 16), dim3(256), 0, st, (const uint16_t*)g, bpart, V, cout,
                       (int)kBiasChunk);
    hipLaunchKernelGGL(k_bgrad_reduce, dim3(cout), dim3(256), 0, st, bpart, db, (int)bch, cout);
  }
  LAUNCHCHK("k_wgrad");
  return 0;
}

int usp_nn_pool2(const void* in, void* out, int D, int H, int W, int C, int backward, void* stream) {
  if (!in || !out || (D | H | W) & 1 || !planes_ok(C)) return fail(USP_ERR_INVALID, "invalid argument");
  hipStream_t st = (hipStream_t)stream;
  const long V = (long)D * H * W;
  if (!backward)
    hipLaunchKernelGGL(k_pool2, dim3(grid_for(V / 8 * (C / 16) * 2)), dim3(256), 0, st, (const uint16_t*)in,
                       (uint16_t*)out, D, H, W, C);
  else  // in = gradient on the coarse grid, out = gradient on the fine grid
    hipLaunchKernelGGL(k_pool2_back, dim3(grid_for(V * (C / 16) * 2)), dim3(256), 0, st, (const uint16_t*)in,
                       (uint16_t*)out, D, H, W, C);
  LAUNCHCHK("k_pool2");
  return 0;
}

int usp_nn_upsample2(const void* in, void* out, int D, int H, int W, int C, int Ctot, int c0, int backward,
                     void* stream) {
  if (!in || !out || (D | H | W) & 1 || c0 < 0 || c0 + C > Ctot || !planes_ok(C) || c0 % 16)
    return fail(USP_ERR_INVALID, "invalid argument");
  hipStream_t st = (hipStream_t)stream;
  const long V = (long)D * H * W;
  if (!backward)
    hipLaunchKernelGGL(k_up2, dim3(grid_for(V * (C / 16) * 2)), dim3(256), 0, st, (const uint16_t*)in, (uint16_t*)out,
                       D, H, W, C, c0);
  else  // in = gradient of the fine concatenated tensor, out = coarse gradient
    hipLaunchKernelGGL(k_up2_back, dim3(grid_for(V / 8 * (C / 16) * 2)), dim3(256), 0, st, (const uint16_t*)in,
                       (uint16_t*)out, D, H, W, C, c0);
  LAUNCHCHK("k_up2");
  return 0;
}

int usp_nn_channel_copy(const void* src, int Cs, int s0, void* dst, int Cd, int d0, int C, long V, void* stream) {
  if (!src || !dst || s0 < 0 || d0 < 0 || s0 + C > Cs || d0 + C > Cd || !planes_ok(C) || s0 % 16 || d0 % 16)
    return fail(USP_ERR_INVALID, "invalid argument");
  const long n8 = V * C / 8;
  hipLaunchKernelGGL(k_copy8, dim3(grid_for(n8)), dim3(256), 0, (hipStream_t)stream,
                     (const uint4*)((const uint16_t*)src + (long)s0 * V), (uint4*)((uint16_t*)dst + (long)d0 * V), n8);
  LAUNCHCHK("k_copy8");
  return 0;
}

int usp_nn_relu_backward(const void* y, const void* g, void* out, long n, int accumulate, void* stream) {
  if (!y || !g || !out) return fail(USP_ERR_INVALID, "invalid argument");
  if (aligned16(y) && aligned16(g) && aligned16(out) && n % 8 == 0)
    hipLaunchKernelGGL(k_relu_back8, dim3(grid_for(n / 8)), dim3(256), 0, (hipStream_t)stream, (const uint4*)y,
                       (const uint4*)g, (uint4*)out, n / 8, accumulate);
  else
    hipLaunchKernelGGL(k_relu_back, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, (const uint16_t*)y,
                       (const uint16_t*)g, (uint16_t*)out, n, accumulate);
  LAUNCHCHK("k_relu_back");
  return 0;
}

int usp_nn_add(void* dst, const void* src, long n, void* stream) {
  if (!dst || !src) return fail(USP_ERR_INVALID, "invalid argument");
  if (aligned16(dst) && aligned16(src) && n % 8 == 0)
    hipLaunchKernelGGL(k_add_bf8, dim3(grid_for(n / 8)), dim3(256), 0, (hipStream_t)stream, (uint4*)dst,
                       (const uint4*)src, n / 8);
  else
    hipLaunchKernelGGL(k_add_bf, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, (uint16_t*)dst,
                       (const uint16_t*)src, n);
  LAUNCHCHK("k_add_bf");
  return 0;
}

int usp_nn_features(const void* nidx, void* out, int D, int H, int W, double n_bg, double n_span, double kappa_max,
                    int plane, double k0h, double w0, void* stream) {
  if (!nidx || !out || D < 1 || H < 1 || W < 1 || plane < 0 || plane >= D || !(n_span > 0.0) || !(kappa_max > 0.0) ||
      !(w0 > 0.0))
    return fail(USP_ERR_INVALID, "invalid argument");
  const long cols = (long)H * W;
  hipLaunchKernelGGL(k_features, dim3((unsigned)((cols + kFeatCols - 1) / kFeatCols)), dim3(kFeatCols * kFeatSeg), 0,
                     (hipStream_t)stream, (const float2*)nidx, (uint16_t*)out, D, H, W, n_bg, n_span, kappa_max, plane,
                     k0h, w0);
  LAUNCHCHK("k_features");
  return 0;
}

int usp_nn_loss(const float* pred, const void* target, float scale, long V, void* grad, void* ws, double* loss_out,
                void* stream) {
  if (!pred || !target || !ws) return fail(USP_ERR_INVALID, "invalid argument");
  hipStream_t st = (hipStream_t)stream;
  const int nb = 1024;
  double* part = (double*)ws;
  double* res = part + 2 * nb;
  hipLaunchKernelGGL(k_loss_parts, dim3(nb), dim3(256), 0, st, pred, (const float2*)target, scale, V, part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, part, nb, res);
  if (grad)
    hipLaunchKernelGGL(k_loss_grad, dim3(grid_for(V)), dim3(256), 0, st, pred, (const float2*)target, scale, V, res,
                       (uint16_t*)grad);
  LAUNCHCHK("k_loss");
  if (loss_out) {
    HIPCHK(hipMemcpyAsync(loss_out, res, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return 0;
}

int usp_nn_adam(float* w, const float* g, float* m, float* v, void* wb, long n, float lr, float b1, float b2, float eps,
                int step, void* stream) {
  if (!w || !g || !m || !v || step < 1) return fail(USP_ERR_INVALID, "invalid argument");
  const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, w, g, m, v, (uint16_t*)wb, n, lr,
                     b1, b2, eps, c1, c2);
  LAUNCHCHK("k_adam");
  return 0;
}

int usp_nn_to_bf16(const float* a, void* b, long n, void* stream) {
  if (!a || !b) return fail(USP_ERR_INVALID, "invalid argument");
  hipLaunchKernelGGL(k_f2bf, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, a, (uint16_t*)b, n);
  LAUNCHCHK("k_f2bf");
  return 0;
}

int usp_nn_pred_to_field(const float* pred, float scale, void* x, long V, void* stream) {
  if (!pred || !x) return fail(USP_ERR_INVALID, "invalid argument");
  hipLaunchKernelGGL(k_pred_field, dim3(grid_for(V)), dim3(256), 0, (hipStream_t)stream, pred, scale, (double2*)x, V);
  LAUNCHCHK("k_pred_field");
  return 0;
}

}  // extern "C"
