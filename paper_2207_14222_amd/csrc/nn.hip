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

long wgrad_chunk(long V) {
  long c = std::max<long>(256, V * 27 / 2048);
  return (c + 15) / 16 * 16;
}

}  // namespace

extern "C" {

int usp_nn_conv3d(const void* in, const void* w, const float* bias, void* out, int out_f32, int cstore, int D, int H,
                  int W, int cin, int cout, int taps, int sign, int relu, void* stream) {
  if (!in || !w || !out || D < 1 || H < 1 || W < 1 || cstore < 1 || cstore > cout || (sign != 1 && sign != -1))
    return fail(USP_ERR_INVALID, "invalid argument");
  const long V = (long)D * H * W;
  if (V % 16) return fail(USP_ERR_UNSUPPORTED_SHAPE, "the voxel count must be a multiple of 16");
  if (sign < 0 && relu) return fail(USP_ERR_INVALID, "the input-gradient convolution takes no ReLU");
  const int blocks = (int)((V / 16 + 3) / 4);
  hipStream_t st = (hipStream_t)stream;
  uint16_t* ob = out_f32 ? nullptr : (uint16_t*)out;
  float* of = out_f32 ? (float*)out : nullptr;
  const uint16_t *ip = (const uint16_t*)in, *wp = (const uint16_t*)w;
  bool ok = with_conv_shape(cin, cout, taps, [&](auto CI, auto CO, auto TP) {
    constexpr int ci = decltype(CI)::value, co = decltype(CO)::value, tp = decltype(TP)::value;
    if (sign > 0) {
      if (relu)
        hipLaunchKernelGGL((k_conv<ci, co, tp, 1, true>), dim3(blocks), dim3(256), 0, st, ip, wp, bias, ob, of, cstore,
                           D, H, W);
      else
        hipLaunchKernelGGL((k_conv<ci, co, tp, 1, false>), dim3(blocks), dim3(256), 0, st, ip, wp, bias, ob, of,
                           cstore, D, H, W);
    } else {
      hipLaunchKernelGGL((k_conv<ci, co, tp, -1, false>), dim3(blocks), dim3(256), 0, st, ip, wp, bias, ob, of, cstore,
                         D, H, W);
    }
  });
  if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "convolution shape not instantiated");
  LAUNCHCHK("k_conv");
  return 0;
}

int usp_nn_wgrad_workspace(int D, int H, int W, int cin, int cout, int taps, size_t* bytes) {
  if (!bytes) return fail(USP_ERR_INVALID, "bytes is NULL");
  const long V = (long)D * H * W;
  const long chunk = wgrad_chunk(V);
  const long nch = (V + chunk - 1) / chunk;
  const long bch = (V + 4095) / 4096;
  *bytes = sizeof(float) * (nch * taps * (long)cout * cin + bch * (long)cout) + 256;
  return 0;
}

int usp_nn_conv3d_wgrad(const void* in, const void* g, float* dw, float* db, void* ws, size_t ws_bytes, int D, int H,
                        int W, int cin, int cout, int taps, void* stream) {
  if (!in || !g || !dw || !ws) return fail(USP_ERR_INVALID, "invalid argument");
  size_t need = 0;
  usp_nn_wgrad_workspace(D, H, W, cin, cout, taps, &need);
  if (ws_bytes < need) return fail(USP_ERR_WORKSPACE, "wgrad workspace too small");
  const long V = (long)D * H * W;
  const long chunk = wgrad_chunk(V);
  const int nch = (int)((V + chunk - 1) / chunk);
  hipStream_t st = (hipStream_t)stream;
  float* part = (float*)ws;
  bool ok = with_conv_shape(cin, cout, taps, [&](auto CI, auto CO, auto TP) {
    constexpr int ci = decltype(CI)::value, co = decltype(CO)::value, tp = decltype(TP)::value;
    const long items = (long)nch * tp * (co / 16) * (ci / 16);
    hipLaunchKernelGGL((k_wgrad<ci, co, tp>), dim3((unsigned)((items + 3) / 4)), dim3(256), 0, st,
                       (const uint16_t*)in, (const uint16_t*)g, part, (int)chunk, nch, D, H, W);
  });
  if (!ok) return fail(USP_ERR_UNSUPPORTED_SHAPE, "convolution shape not instantiated");
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(grid_for((long)taps * cout * cin)), dim3(256), 0, st, part, dw, nch, taps,
                     cout, cin);
  if (db) {
    float* bpart = part + (long)nch * taps * cout * cin;
    const int bch = (int)((V + 4095) / 4096);
    hipLaunchKernelGGL(k_bgrad, dim3(bch), dim3(256), 0, st, (const uint16_t*)g, bpart, V, cout, 4096);
    hipLaunchKernelGGL(k_bgrad_reduce, dim3(1), dim3(256), 0, st, bpart, db, bch, cout);
  }
  LAUNCHCHK("k_wgrad");
  return 0;
}

int usp_nn_pool2(const void* in, void* out, int D, int H, int W, int C, int backward, void* stream) {
  if (!in || !out || (D | H | W) & 1) return fail(USP_ERR_INVALID, "even grid sizes required");
  hipStream_t st = (hipStream_t)stream;
  if (!backward)
    hipLaunchKernelGGL(k_pool2, dim3(grid_for((long)D * H * W * C / 8)), dim3(256), 0, st, (const uint16_t*)in,
                       (uint16_t*)out, D, H, W, C);
  else  // in = gradient on the coarse grid, out = gradient on the fine grid
    hipLaunchKernelGGL(k_pool2_back, dim3(grid_for((long)D * H * W * C)), dim3(256), 0, st, (const uint16_t*)in,
                       (uint16_t*)out, D, H, W, C);
  LAUNCHCHK("k_pool2");
  return 0;
}

int usp_nn_upsample2(const void* in, void* out, int D, int H, int W, int C, int Ctot, int c0, int backward,
                     void* stream) {
  if (!in || !out || (D | H | W) & 1 || c0 < 0 || c0 + C > Ctot) return fail(USP_ERR_INVALID, "invalid argument");
  hipStream_t st = (hipStream_t)stream;
  if (!backward)
    hipLaunchKernelGGL(k_up2, dim3(grid_for((long)D * H * W * C)), dim3(256), 0, st, (const uint16_t*)in,
                       (uint16_t*)out, D, H, W, C, Ctot, c0);
  else  // in = gradient of the fine concatenated tensor, out = coarse gradient
    hipLaunchKernelGGL(k_up2_back, dim3(grid_for((long)D * H * W * C / 8)), dim3(256), 0, st, (const uint16_t*)in,
                       (uint16_t*)out, D, H, W, C, Ctot, c0);
  LAUNCHCHK("k_up2");
  return 0;
}

int usp_nn_channel_copy(const void* src, int Cs, int s0, void* dst, int Cd, int d0, int C, long V, void* stream) {
  if (!src || !dst || s0 + C > Cs || d0 + C > Cd) return fail(USP_ERR_INVALID, "invalid argument");
  hipLaunchKernelGGL(k_chcopy, dim3(grid_for(V * C)), dim3(256), 0, (hipStream_t)stream, (const uint16_t*)src, Cs, s0,
                     (uint16_t*)dst, Cd, d0, C, V);
  LAUNCHCHK("k_chcopy");
  return 0;
}

int usp_nn_relu_backward(const void* y, const void* g, void* out, long n, int accumulate, void* stream) {
  if (!y || !g || !out) return fail(USP_ERR_INVALID, "invalid argument");
  hipLaunchKernelGGL(k_relu_back, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, (const uint16_t*)y,
                     (const uint16_t*)g, (uint16_t*)out, n, accumulate);
  LAUNCHCHK("k_relu_back");
  return 0;
}

int usp_nn_add(void* dst, const void* src, long n, void* stream) {
  if (!dst || !src) return fail(USP_ERR_INVALID, "invalid argument");
  hipLaunchKernelGGL(k_add_bf, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, (uint16_t*)dst,
                     (const uint16_t*)src, n);
  LAUNCHCHK("k_add_bf");
  return 0;
}

int usp_nn_features(const void* nidx, void* out, int D, int H, int W, double n_bg, double n_span, double kappa_max,
                    int plane, void* stream) {
  if (!nidx || !out || !(n_span > 0.0) || !(kappa_max > 0.0)) return fail(USP_ERR_INVALID, "invalid argument");
  hipLaunchKernelGGL(k_features, dim3(grid_for((long)D * H * W)), dim3(256), 0, (hipStream_t)stream,
                     (const float2*)nidx, (uint16_t*)out, D, H, W, n_bg, n_span, kappa_max, plane);
  LAUNCHCHK("k_features");
  return 0;
}

int usp_nn_loss(const float* pred, const void* target, float scale, long V, void* grad, void* ws, double* loss_out,
                void* stream) {
  if (!pred || !target || !ws || !loss_out) return fail(USP_ERR_INVALID, "invalid argument");
  hipStream_t st = (hipStream_t)stream;
  const int nb = 1024;
  double* part = (double*)ws;
  double* res = part + 2 * nb;
  hipLaunchKernelGGL(k_loss_parts, dim3(nb), dim3(256), 0, st, pred, (const float2*)target, scale, V, part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, st, part, nb, res);
  if (grad)
    hipLaunchKernelGGL(k_loss_grad, dim3(grid_for(V)), dim3(256), 0, st, pred, (const float2*)target, scale, V, res,
                       (uint16_t*)grad);
  LAUNCHCHK("k_loss");
  HIPCHK(hipMemcpyAsync(loss_out, res, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
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

int usp_nn_transpose_weights(const void* w, void* wt, int cout, int taps, int cin, void* stream) {
  if (!w || !wt) return fail(USP_ERR_INVALID, "invalid argument");
  hipLaunchKernelGGL(k_wtrans, dim3(grid_for((long)cout * taps * cin)), dim3(256), 0, (hipStream_t)stream,
                     (const uint16_t*)w, (uint16_t*)wt, cout, taps, cin);
  LAUNCHCHK("k_wtrans");
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
