// Grouped batched solver: every launch covers the tiles of all active problems
// of a batch (blockIdx.x -> (problem, first line or column)), so the whole chip
// works on the batch while problem sizes differ.  One refinement cycle is
//   FIRST (t = F_x r32, d32 = 0), k x [SYM, FUSED]   -- complex64 iterations
//   RFWD, SYMA, RINV, FINAL                          -- FP64 residual, decision
// with per-problem convergence decided on the device (FINAL sets done flags
// and timestamps); blocks of finished problems return at once.  Launch
// boundaries order all accesses: there is no cross-workgroup synchronisation.
#pragma once
#include "batch.hpp"

namespace usp {

struct GTask {
  int p;      // problem index
  int start;  // first line (contiguous-axis passes) or first column (strided passes)
  int slot;   // index of this task among its problem's tasks (partial-sum column)
  int pad;
};

struct GState {
  int done;        // 1 when finished
  int status;      // 0 converged, 1 maxit, 2 stagnated, -5 non-finite
  int iterations;
  int since_best;
  double best;
  double rho;
  double ynorm2;
  unsigned long long t_start, t_done;
  double rho_prev; // FP64 residual before the last cycle
  int budget;      // inner iterations of the next cycle (at most kmax)
  int kmax;        // refinement interval k
};

constexpr int kGX = 256;   // threads of the contiguous-axis group kernels
constexpr int kGS64 = 512; // threads of the complex64 strided group kernel
constexpr int kGS128 = 256;

template <int N> constexpr int g_lpb() { return kGX / (N / PassPlan<N>::E); }
// NW = 1 (variant bit 3): column tiles half as wide, in blocks of kGS64 / 2
// threads (more, smaller blocks per CU)
template <int N, int NW = 0> constexpr int g_w64() { return cmin(cmin(kGS64 / (N / PassPlan<N>::E), 16), N) >> NW; }
template <int N> constexpr int g_w128() { return cmin(cmin(kGS128 / (N / PassPlan<N>::E), 8), N); }
// complex64 t of the 1024^2 problems is kept in column tiles of g_w64 (the
// column pass reads 64 KB blocks instead of 64-byte row segments)
template <int N, int NW = 0> constexpr int g_tile() { return N == 1024 ? g_w64<N, NW>() : 0; }

template <class C> __device__ __forceinline__ void copy_tw(C* tws, const C* tw, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) tws[i] = tw[i];
  __syncthreads();
}

// GMODE: 0 init (B32, x = 0, |y|^2), 1 FIRST, 2 FUSED, 3 RFWD (first residual),
// 4 RINV, 5 RFWD after inner iterations (x += d first).  j: index of a FUSED
// launch within the cycle; problems whose cycle budget is spent skip it.
template <int GMODE, int FL, int NW = 0>
__global__ void __launch_bounds__(kGX)
k_gx(const GTask* __restrict__ tasks, const BatchProblem* __restrict__ probs, const GState* __restrict__ st,
     double* __restrict__ part, long pitch, int j) {
  constexpr bool F64 = (GMODE == 3 || GMODE == 4 || GMODE == 5);
  using C = typename std::conditional<F64, double2, float2>::type;
  __shared__ C lds[kGX * 17];
  __shared__ C tws[1024];
  __shared__ double scratch[64];
  const GTask tk = tasks[blockIdx.x];
  if (GMODE != 0 && st[tk.p].done) return;  // whole block; the state is not yet set during init
  if (GMODE == 2 && j >= st[tk.p].budget) return;
  const BatchProblem P = probs[tk.p];
  double acc = 0.0;
  auto run = [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    constexpr int LPB = g_lpb<N>();
    if (GMODE == 0) {
      const long n0 = (long)tk.start * N, n1 = n0 + (long)LPB * N;
      for (long i = n0 + threadIdx.x; i < n1 && i < (long)N * N; i += kGX) {
        P.B32[i] = cvt<float2>(P.B64[i]);
        if (!P.x_is_guess) P.x64[i] = mk<double2>(0.0, 0.0);
        acc += cabs2(P.y64[i]);
      }
      return;
    }
    if constexpr (F64) {
      copy_tw(reinterpret_cast<double2*>(tws), P.twd, N);
      if (GMODE == 3 || GMODE == 5) {
        const float2* dc = GMODE == 5 ? P.d32 : nullptr;
        xpass_body<double2, double2, N, X_RFWD, 0, LPB>(P.S, P.x64, P.y64, P.B64, dc, nullptr,
                                                        reinterpret_cast<double2*>(tws),
                                                        reinterpret_cast<double2*>(lds), 0.0, tk.start, N, 0);
      } else {
        acc = xpass_body<double2, double2, N, X_RINV, 0, LPB>(P.S, P.x64, P.y64, P.B64, nullptr, P.r32,
                                                              reinterpret_cast<double2*>(tws),
                                                              reinterpret_cast<double2*>(lds), 0.0, tk.start, N, 0);
      }
    } else {
      copy_tw(reinterpret_cast<float2*>(tws), P.twf, N);
      if (GMODE == 1) {
        xpass_body<float2, float2, N, X_FIRST, 0, LPB, g_tile<N, NW>()>(P.t, P.d32, P.r32, P.B32, nullptr, nullptr,
                                                       reinterpret_cast<float2*>(tws), reinterpret_cast<float2*>(lds),
                                                       0.0, tk.start, N, 2);
      } else {
        xpass_body<float2, float2, N, X_FUSED, FL, LPB, g_tile<N, NW>()>(P.t, P.d32, P.r32, P.B32, nullptr, nullptr,
                                                        reinterpret_cast<float2*>(tws),
                                                        reinterpret_cast<float2*>(lds), P.alpha, tk.start, N, 1);
      }
    }
  };
  switch (P.n) {
    case 8: run(std::integral_constant<int, 8>{}); break;
    case 16: run(std::integral_constant<int, 16>{}); break;
    case 32: run(std::integral_constant<int, 32>{}); break;
    case 64: run(std::integral_constant<int, 64>{}); break;
    case 128: run(std::integral_constant<int, 128>{}); break;
    case 256: run(std::integral_constant<int, 256>{}); break;
    case 512: run(std::integral_constant<int, 512>{}); break;
    case 1024: run(std::integral_constant<int, 1024>{}); break;
    default: break;
  }
  if (GMODE == 0 || GMODE == 4) {
    const double s = block_sum(acc, scratch);
    if (threadIdx.x == 0) part[(long)tk.p * pitch + tk.slot] = s;
  }
}

// strided pass along axis 0 of every task's problem: SYM (complex64,
// 1/(N (l + 1))) or SYMA (complex128, l(p)/N); j as in k_gx for SYM
template <int GMODE, int NW = 0>
__global__ void __launch_bounds__(GMODE == 0 ? (kGS64 >> NW) : kGS128)
k_gs(const GTask* __restrict__ tasks, const BatchProblem* __restrict__ probs, const GState* __restrict__ st, int j) {
  constexpr bool F64 = (GMODE == 1);
  using C = typename std::conditional<F64, double2, float2>::type;
  constexpr int LDSN = (F64 || NW) ? 1024 * 5 : 1024 * 9;
  __shared__ C lds[LDSN];
  __shared__ C tws[1024];
  // consecutive column tiles (which share cache lines when a tile row is
  // narrower than a line) on one XCD: blocks are dealt to the 8 XCDs in turn
  const int nb = gridDim.x, nb8 = nb - nb % 8, bb = blockIdx.x;
  const GTask tk = tasks[bb < nb8 ? (bb % 8) * (nb8 / 8) + bb / 8 : bb];
  if (st[tk.p].done) return;
  if (GMODE == 0 && j >= st[tk.p].budget) return;
  const BatchProblem P = probs[tk.p];
  SymArgs sym;
  sym.sa = P.sa;
  sym.sm = 0.0;
  sym.sx = P.sx;
  sym.n1 = 1;
  sym.log2_n2 = __builtin_ctz(P.n);
  sym.c0r = P.s0r + (F64 ? 0.0 : 1.0);
  sym.c0i = P.s0i;
  sym.c2r = P.s2r;
  sym.c2i = P.s2i;
  sym.scale = 1.0 / ((double)P.n * P.n);
  auto run = [&](auto NC) {
    constexpr int N = decltype(NC)::value;
    if constexpr (F64) {
      constexpr int W = g_w128<N>();
      static_assert(N * (W + 1) <= LDSN, "LDS tile");
      spass_body<double2, N, W, S_SYMA>(P.S, P.twd, reinterpret_cast<double2*>(tws),
                                        reinterpret_cast<double2*>(lds), N, sym, tk.start, 0);
    } else {
      constexpr int W = g_w64<N, NW>();
      static_assert(N * (W + 1) <= LDSN, "LDS tile");
      static_assert(W * (N / PassPlan<N>::E) <= (kGS64 >> NW), "block threads");
      spass_body<float2, N, W, S_SYM, (g_tile<N, NW>() > 0)>(P.t, P.twf, reinterpret_cast<float2*>(tws),
                                                         reinterpret_cast<float2*>(lds), N, sym, tk.start, 0);
    }
  };
  switch (P.n) {
    case 8: run(std::integral_constant<int, 8>{}); break;
    case 16: run(std::integral_constant<int, 16>{}); break;
    case 32: run(std::integral_constant<int, 32>{}); break;
    case 64: run(std::integral_constant<int, 64>{}); break;
    case 128: run(std::integral_constant<int, 128>{}); break;
    case 256: run(std::integral_constant<int, 256>{}); break;
    case 512: run(std::integral_constant<int, 512>{}); break;
    case 1024: run(std::integral_constant<int, 1024>{}); break;
    default: break;
  }
}

// One block per problem.  INIT: |y|^2 and the state, m = the refinement
// interval k.  Otherwise: the residual decision after the cycle that just ran
// (m > 0; m = 0 for the check of the initial x), converged / stagnated / maxit
// / non-finite, with the problem's finishing timestamp, and the next cycle's
// budget: k, or fewer when the residual's rate over the last cycle predicts
// the crossing of tol within half a cycle (the margin of the single-problem
// solve).
template <bool INIT>
__global__ void __launch_bounds__(256)
k_gfinal(const BatchProblem* __restrict__ probs, GState* __restrict__ st, const double* __restrict__ part, long pitch,
         const int* __restrict__ nslots, int m) {
  __shared__ double scratch[64];
  const int p = blockIdx.x;
  if (!INIT && st[p].done) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nslots[p]; i += blockDim.x) acc += part[(long)p * pitch + i];
  const double s = block_sum(acc, scratch);
  if (threadIdx.x != 0) return;
  GState g = st[p];
  if (INIT) {
    g.done = 0;
    g.status = 1;
    g.iterations = 0;
    g.since_best = 0;
    g.best = 1e300;
    g.rho = 1.0;
    g.ynorm2 = s;
    g.t_start = wall_clock64();
    g.t_done = g.t_start;
    g.rho_prev = 1.0;
    g.kmax = m > 0 ? m : 1;
    g.budget = g.kmax;
    st[p] = g;
    return;
  }
  const int ran = m > 0 ? g.budget : 0;
  g.iterations += ran;
  const double rho = sqrt(s / g.ynorm2);
  g.rho = rho;
  int fin = -100;
  if (!(rho == rho)) fin = -5;
  else if (rho < probs[p].tol) fin = 0;
  else {
    if (rho < 0.99 * g.best) {
      g.best = rho;
      g.since_best = 0;
    } else if (++g.since_best >= 8) {
      fin = 2;
    }
    if (fin == -100 && g.iterations >= probs[p].maxit) fin = 1;
  }
  if (fin != -100) {
    g.done = 1;
    g.status = fin;
    g.t_done = wall_clock64();
  } else {
    int nb = g.kmax;
    if (ran > 0 && rho > 0.0 && rho < g.rho_prev) {
      const double lrate = log(rho / g.rho_prev) / ran;   // log of the per-iteration factor
      const double need = log(probs[p].tol / rho) / lrate;
      if (need < 0.5 * nb) nb = max(1, (int)ceil(1.05 * need) + 1);
    }
    g.budget = max(1, min(nb, probs[p].maxit - g.iterations));
  }
  g.rho_prev = rho;
  st[p] = g;
}

}  // namespace usp
