// Internal header shared by the library's translation units: operator handle
// layout, workspace layout and helpers.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/usp.h"
#include "antisym.hpp"

namespace usp_detail {

// records the message of the last error on this thread and returns `code`
int fail(int code, const std::string& msg);


#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(USP_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCHK(what)                                                                \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess) return fail(USP_ERR_HIP, std::string(what ": ") + hipGetErrorString(e_)); \
  } while (0)

constexpr int kHist = 1 << 16;   // device ring of ||Delta||^2 values
constexpr int kRows = 32;        // pending per-iteration partial-sum rows between finalisations
constexpr int kMinN = 8, kMaxN = 1024;

inline bool pow2_in_range(int n) { return n >= kMinN && n <= kMaxN && (n & (n - 1)) == 0; }
inline int ilog2(long n) {
  int l = 0;
  while ((1L << l) < n) ++l;
  return l;
}

template <class F>
bool with_n(int n, F&& f) {
  switch (n) {
    case 8: f(std::integral_constant<int, 8>{}); return true;
    case 16: f(std::integral_constant<int, 16>{}); return true;
    case 32: f(std::integral_constant<int, 32>{}); return true;
    case 64: f(std::integral_constant<int, 64>{}); return true;
    case 128: f(std::integral_constant<int, 128>{}); return true;
    case 256: f(std::integral_constant<int, 256>{}); return true;
    case 512: f(std::integral_constant<int, 512>{}); return true;
    case 1024: f(std::integral_constant<int, 1024>{}); return true;
    default: return false;
  }
}

inline size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
  size_t t = 0, S = 0, B32 = 0, r32 = 0, d32 = 0, adj_j = 0, adj_w = 0;
  size_t partials = 0, hist = 0, scal = 0, hist_true = 0, info = 0;
  size_t twf[11] = {0}, twd[11] = {0};
  size_t total = 0;
  long nblk = 0;
};

struct Dims {
  int ndim, n0, n1, n2;
  long N;
};

inline int get_dims(const usp_symbol* L, Dims* d) {
  if (!L) return fail(USP_ERR_INVALID, "symbol is NULL");
  if (L->ndim < 1 || L->ndim > 3) return fail(USP_ERR_INVALID, "ndim must be 1, 2 or 3");
  for (int a = 0; a < L->ndim; ++a)
    if (!pow2_in_range(L->shape[a]))
      return fail(USP_ERR_UNSUPPORTED_SHAPE, "every axis length must be a power of two in [8, 1024]");
  d->ndim = L->ndim;
  if (L->ndim == 1) {
    d->n0 = 1; d->n1 = 1; d->n2 = L->shape[0];
  } else if (L->ndim == 2) {
    d->n0 = L->shape[0]; d->n1 = 1; d->n2 = L->shape[1];
  } else {
    d->n0 = L->shape[0]; d->n1 = L->shape[1]; d->n2 = L->shape[2];
  }
  d->N = (long)d->n0 * d->n1 * d->n2;
  return 0;
}

inline int make_layout(const usp_symbol* L, int dtype, int flags, Layout* lay, Dims* dims) {
  int rc = get_dims(L, dims);
  if (rc) return rc;
  if (dtype != USP_C64 && dtype != USP_C128) return fail(USP_ERR_INVALID, "dtype must be USP_C64 or USP_C128");
  const bool refine = (flags & USP_FLAG_REFINE) != 0;
  if (refine && dtype != USP_C128) return fail(USP_ERR_INVALID, "refined mode needs USP_C128 buffers");
  if (refine && dims->ndim == 1) return fail(USP_ERR_INVALID, "refined mode is for 2-D / 3-D grids");
  const bool antisym = (flags & USP_FLAG_ANTISYM) != 0;
  if (antisym && (dims->ndim != 1 || refine)) return fail(USP_ERR_INVALID, "the antisymmetrised form is for 1-D handles");
  if (flags & ~(USP_FLAG_REFINE | USP_FLAG_ANTISYM)) return fail(USP_ERR_INVALID, "unknown flag");
  // the first-derivative term and its Nyquist convention exist for 1-D symbols
  // only: the multi-axis passes apply c0 + c2 |p|^2
  if (dims->ndim >= 2 && (L->a1[0] != 0.0 || L->a1[1] != 0.0 || L->nyquist_zero))
    return fail(USP_ERR_INVALID, "a1 and nyquist_zero must be 0 for 2-D and 3-D symbols");
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const long N = dims->N;
  if (dims->ndim >= 2) {
    const size_t ts = (dtype == USP_C128 && !refine) ? 16 : 8;
    lay->t = take(N * ts);
    lay->S = take(N * 16);
    if (refine) {
      lay->B32 = take(N * 8);
      lay->r32 = take(N * 8);
      lay->d32 = take(N * 8);
    }
  }
  if (antisym) {  // adjoint-gather table
    lay->adj_j = take(sizeof(int) * N * usp::kAdjMax);
    lay->adj_w = take(16 * N * usp::kAdjMax);
  }
  // one row of per-block partials per pending iteration, plus a residual row and a norm row
  lay->nblk = (long)dims->n0 * dims->n1 + 4096;
  lay->partials = take(sizeof(double) * lay->nblk * (kRows + 2));
  lay->hist = take(sizeof(double) * kHist);
  lay->scal = take(64 * sizeof(double));
  lay->hist_true = take(2 * sizeof(double) * kHist);
  lay->info = take(64);
  for (int l = 3; l <= 10; ++l) {
    const int n = 1 << l;
    if (n == dims->n0 || n == dims->n1 || n == dims->n2) {
      lay->twf[l] = take(sizeof(float2) * n);
      lay->twd[l] = take(sizeof(double2) * n);
    }
  }
  lay->total = off;
  return 0;
}

}  // namespace usp_detail

using namespace usp_detail;

struct usp_op_s {
  Dims d;
  int dtype = 0, flags = 0;
  bool refine = false;
  hipStream_t st = nullptr;
  usp_symbol sym;
  const void* B = nullptr;
  bool has_gather = false;
  usp_gather g{};
  char* ws = nullptr;
  Layout lay;
  void* t = nullptr;
  double2* S = nullptr;
  float2 *B32 = nullptr, *r32 = nullptr, *d32 = nullptr;
  double* partials = nullptr;
  long pitch = 0;          // row pitch of partials (doubles)
  int pending = 0;         // per-iteration rows written since the last finalisation
  int pending_first = 0;   // iteration index of the first pending row
  bool pending_f32 = false;  // the pending rows hold complex64 iterations' FP32 partials
  int xblocks = 0;         // blocks of the last complex64/128 contiguous-axis launch (row width)
  double* hist = nullptr;
  double* scal = nullptr;
  double* hist_true = nullptr;
  usp::Solve1DInfo* info = nullptr;
  bool antisym = false;
  int* adj_j = nullptr;   // adjoint gather table (antisymmetrised form)
  void* adj_w = nullptr;
  float2* twf[11] = {nullptr};
  double2* twd[11] = {nullptr};
  // symbol multiplier constants
  double sa0[2], sa1[2], sa2[2];
  usp_plan plan{};
  // per-pass event timing (usp_profile)
  std::vector<hipEvent_t>* prof = nullptr;  // array of USP_NPASS vectors of (start, stop) events
  int kind = 0;
};

