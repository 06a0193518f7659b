// Batched persistent solver: many independent 2-D problems of uneven sizes in
// one launch.  Each workgroup takes a problem from a ticket counter and runs
// the whole refined solve on it -- complex64 iterations of Algorithm 1
// (Sec. 2.1) with the FP64 residual recomputed and accumulated every k
// iterations -- then takes the next problem, until the queue is empty.  The
// passes use the same device bodies as the single-problem kernels, looping
// over line groups and column tiles inside the workgroup; a problem's
// intermediate arrays are only touched by its own workgroup, so barriers
// inside the workgroup order all accesses and no cross-workgroup
// synchronisation or fence exists.  Every loop is bounded (maxit).
#pragma once
#include "passes.hpp"

namespace usp {

constexpr int kBatchThreads = 512;

struct BatchProblem {
  int n;              // 2-D grid n x n (axis 0 rows, axis 1 contiguous)
  int maxit;
  int k;              // refinement interval
  int x_is_guess;
  double alpha, tol;
  double sa, sx;      // (2 pi/(n h0))^2, (2 pi/(n h1))^2
  double s0r, s0i;    // s * a0
  double s2r, s2i;    // s * a2
  const double2* y64;
  const double2* B64;
  double2* x64;
  float2* t;
  float2* r32;
  float2* d32;
  float2* B32;
  double2* S;
  const float2* twf;  // length-n twiddle tables
  const double2* twd;
};

struct BatchResult {
  int iterations;
  int status;         // 0 converged, 1 maxit, 2 stagnated, -5 non-finite
  double rho;         // last true residual ||y - A x||/||y||
  unsigned long long t_start, t_done;  // wall-clock ticks
};

constexpr int cmin(int a, int b) { return a < b ? a : b; }

// column-tile widths of the strided passes inside the batched solver: at most
// 16 columns, at most the number of columns N, at most the participating
// threads (256 for the FP64 passes, kBatchThreads for the complex64 ones)
template <int N> constexpr int batch_w128() { return cmin(cmin(256 / (N / PassPlan<N>::E), 16), N); }
template <int N> constexpr int batch_w64() { return cmin(cmin(kBatchThreads / (N / PassPlan<N>::E), 16), N); }

// LDS bytes the batched solver needs for side length n
template <int N> constexpr long batch_lds_bytes() {
  constexpr int E = PassPlan<N>::E, T = N / E;
  constexpr int L128 = 256 / T, L64 = kBatchThreads / T;
  constexpr int W128 = batch_w128<N>(), W64 = batch_w64<N>();
  constexpr long a = (long)L128 * LdsRow<double2>::padded(N) * 16, b = (long)L64 * LdsRow<float2>::padded(N) * 8;
  constexpr long c = (long)N * (W128 + 1) * 16, d = (long)N * (W64 + 1) * 8;
  constexpr long w = a > b ? (a > c ? (a > d ? a : d) : (c > d ? c : d)) : (b > c ? (b > d ? b : d) : (c > d ? c : d));
  return (long)N * 24 + w;
}

template <int N, int FL>
__device__ __noinline__ void batch_solve(const BatchProblem& P, BatchResult* res, char* smem, double* scratch) {
  constexpr int E = PassPlan<N>::E, T = N / E;
  constexpr int L128 = 256 / T, L64 = kBatchThreads / T;
  constexpr int W128 = batch_w128<N>(), W64 = batch_w64<N>();
  const int tid = threadIdx.x;
  const unsigned long long t0 = wall_clock64();
  float2* twf = reinterpret_cast<float2*>(smem);
  double2* twd = reinterpret_cast<double2*>(smem + N * 8);
  char* work = smem + N * 24;
  for (int i = tid; i < N; i += kBatchThreads) {
    twf[i] = P.twf[i];
    twd[i] = P.twd[i];
  }
  const long NN = (long)N * N;
  double yy = 0.0;
  for (long i = tid; i < NN; i += kBatchThreads) {
    P.B32[i] = cvt<float2>(P.B64[i]);
    if (!P.x_is_guess) P.x64[i] = mk<double2>(0.0, 0.0);
    yy += cabs2(P.y64[i]);
  }
  yy = block_sum(yy, scratch);  // its barriers also order the stores above

  SymArgs sr;  // residual: l(p)/NN
  sr.sa = P.sa;
  sr.sm = 0.0;
  sr.sx = P.sx;
  sr.n1 = 1;
  sr.log2_n2 = __builtin_ctz(N);
  sr.c0r = P.s0r;
  sr.c0i = P.s0i;
  sr.c2r = P.s2r;
  sr.c2i = P.s2i;
  sr.scale = 1.0 / (double)NN;
  SymArgs si = sr;  // iteration: 1/(NN (l(p) + 1))
  si.c0r += 1.0;

  int it = 0, status = 1, since_best = 0, ran = 0;
  double rho = 0.0, best = 1e300, rho_prev = 0.0;
  const float2* dcorr = nullptr;
  for (;;) {
    // FP64 residual r = y - A (x + d); x += d; r32 = complex64(r)
    for (int l0 = 0; l0 < N; l0 += L128)
      xpass_body<double2, double2, N, X_RFWD, 0, L128>(P.S, P.x64, P.y64, P.B64, dcorr, nullptr, twd,
                                                        reinterpret_cast<double2*>(work), 0.0, l0, N, 0);
    __syncthreads();
    for (int c0 = 0; c0 < N; c0 += W128)
      spass_body<double2, N, W128, S_SYMA>(P.S, nullptr, twd, reinterpret_cast<double2*>(work), N, sr, c0, 0);
    __syncthreads();
    double rr = 0.0;
    for (int l0 = 0; l0 < N; l0 += L128)
      rr += xpass_body<double2, double2, N, X_RINV, 0, L128>(P.S, P.x64, P.y64, P.B64, nullptr, P.r32, twd,
                                                             reinterpret_cast<double2*>(work), 0.0, l0, N, 0);
    rr = block_sum(rr, scratch);
    rho = sqrt(rr / yy);
    if (!(rho == rho)) { status = -5; break; }
    if (rho < P.tol) { status = 0; break; }
    if (rho < 0.99 * best) {
      best = rho;
      since_best = 0;
    } else if (++since_best >= 8) {
      status = 2;
      break;
    }
    if (it >= P.maxit) { status = 1; break; }
    // complex64 inner iterations on A d = r from d = 0: k, or fewer when the
    // residual's rate over the last cycle predicts the crossing of tol within
    // half a cycle (the rule of the grouped schedule)
    int nb = P.k;
    if (ran > 0 && rho > 0.0 && rho < rho_prev) {
      const double lrate = log(rho / rho_prev) / ran;
      const double need = log(P.tol / rho) / lrate;
      if (need < 0.5 * nb) nb = max(1, (int)ceil(1.05 * need) + 1);
    }
    const int m = max(1, min(nb, P.maxit - it));
    rho_prev = rho;
    ran = m;
    for (long i = tid; i < NN; i += kBatchThreads) P.d32[i] = mk<float2>(0.0, 0.0);
    for (int l0 = 0; l0 < N; l0 += L64)
      xpass_body<float2, float2, N, X_FIRST, 0, L64>(P.t, P.d32, P.r32, P.B32, nullptr, nullptr, twf,
                                                      reinterpret_cast<float2*>(work), 0.0, l0, N, 0);
    __syncthreads();
    for (int j = 0; j < m; ++j) {
      for (int c0 = 0; c0 < N; c0 += W64)
        spass_body<float2, N, W64, S_SYM>(P.t, nullptr, twf, reinterpret_cast<float2*>(work), N, si, c0, 0);
      __syncthreads();
      for (int l0 = 0; l0 < N; l0 += L64)
        xpass_body<float2, float2, N, X_FUSED, FL, L64>(P.t, P.d32, P.r32, P.B32, nullptr, nullptr, twf,
                                                         reinterpret_cast<float2*>(work), P.alpha, l0, N, 1);
      __syncthreads();
    }
    it += m;
    dcorr = P.d32;
  }
  if (tid == 0) {
    res->iterations = it;
    res->status = status;
    res->rho = rho;
    res->t_start = t0;
    res->t_done = wall_clock64();
  }
  __syncthreads();
}

template <int FL>
__global__ void __launch_bounds__(kBatchThreads)
k_batch(const BatchProblem* __restrict__ probs, int nprob, unsigned* __restrict__ ticket,
        BatchResult* __restrict__ out) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double scratch[64];
  __shared__ int cur;
  for (int guard = 0; guard <= nprob; ++guard) {
    if (threadIdx.x == 0) cur = (int)atomicAdd(ticket, 1u);
    __syncthreads();
    const int p = cur;
    __syncthreads();
    if (p >= nprob) break;
    const BatchProblem P = probs[p];
    switch (P.n) {
      case 8: batch_solve<8, FL>(P, out + p, smem, scratch); break;
      case 16: batch_solve<16, FL>(P, out + p, smem, scratch); break;
      case 32: batch_solve<32, FL>(P, out + p, smem, scratch); break;
      case 64: batch_solve<64, FL>(P, out + p, smem, scratch); break;
      case 128: batch_solve<128, FL>(P, out + p, smem, scratch); break;
      case 256: batch_solve<256, FL>(P, out + p, smem, scratch); break;
      case 512: batch_solve<512, FL>(P, out + p, smem, scratch); break;
      case 1024: batch_solve<1024, FL>(P, out + p, smem, scratch); break;
      default:
        if (threadIdx.x == 0) out[p].status = -1;
        break;
    }
  }
}

__global__ void k_reset_ticket(unsigned* ticket) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ticket = 0u;
}

}  // namespace usp
