// Device building blocks: complex arithmetic, in-register DFTs, Stockham stages
// staged through LDS, and deterministic block reductions.
//
// FFT convention (forward): X[k] = sum_n x[n] exp(-2 pi i n k / N), unnormalised;
// the inverse uses exp(+2 pi i n k / N) and no 1/N (callers fold 1/N into the
// spectral multiplier).  This is the transform F of the Fourier inverse of L + I
// (Helmholtz section, Eq. laplacian_inverse).
//
// Register layout shared by every stage: thread t of a line owns E elements, and
// register e holds line position t + T*e (T = N/E threads per line).  A Stockham
// stage of radix R with span Ns performs E/R butterflies per thread (butterfly
// j = t + m*T reads positions j + k*N/R and writes (j/Ns)*Ns*R + j%Ns + q*Ns),
// so the first stage reads and the last stage writes exactly the register
// layout above: loads and stores go straight between HBM and registers, and
// only the intermediate exchanges use LDS.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace usp {

template <class C> struct real_of;
template <> struct real_of<float2> { using type = float; };
template <> struct real_of<double2> { using type = double; };

template <class C> __device__ __forceinline__ C mk(double x, double y) {
  C c;
  c.x = (typename real_of<C>::type)x;
  c.y = (typename real_of<C>::type)y;
  return c;
}
template <class C> __device__ __forceinline__ C cadd(C a, C b) { C c; c.x = a.x + b.x; c.y = a.y + b.y; return c; }
template <class C> __device__ __forceinline__ C csub(C a, C b) { C c; c.x = a.x - b.x; c.y = a.y - b.y; return c; }
template <class C> __device__ __forceinline__ C cmul(C a, C b) {
  C c;
  c.x = a.x * b.x - a.y * b.y;
  c.y = a.x * b.y + a.y * b.x;
  return c;
}
template <class C> __device__ __forceinline__ C cconj(C a) { a.y = -a.y; return a; }
template <class C> __device__ __forceinline__ C cscale(C a, typename real_of<C>::type s) { a.x *= s; a.y *= s; return a; }
template <class C> __device__ __forceinline__ double cabs2(C a) { return (double)a.x * a.x + (double)a.y * a.y; }
// |a|^2 in the precision of the field (FP32 for complex64, FP64 for complex128),
// one explicit fused multiply-add so the rounding does not depend on how the
// compiler schedules the surrounding code
template <class C> __device__ __forceinline__ typename real_of<C>::type cnorm2(C a) { return fma(a.y, a.y, a.x * a.x); }

// conversion between storage and compute precision
template <class D, class S> __device__ __forceinline__ D cvt(S s) {
  D d;
  d.x = (typename real_of<D>::type)s.x;
  d.y = (typename real_of<D>::type)s.y;
  return d;
}

// 1/z for complex z (conj(z)/|z|^2).  Single precision takes the hardware
// reciprocal (1 ulp) instead of the correctly rounded divide, whose
// scale-and-fixup sequence was about a tenth of the instructions of the
// complex64 symbol pass; double precision divides.
template <class C> __device__ __forceinline__ C crecip(C z) {
  using R = typename real_of<C>::type;
  R d = z.x * z.x + z.y * z.y;
  R inv;
  if constexpr (std::is_same<R, float>::value)
    inv = __builtin_amdgcn_rcpf(d);
  else
    inv = R(1) / d;
  C r;
  r.x = z.x * inv;
  r.y = -z.y * inv;
  return r;
}

// cos(2 pi m / 16) and sin(2 pi m / 16)
__host__ __device__ constexpr double cos16(int m) {
  m &= 15;
  return m == 0 ? 1.0 : m == 1 ? 0.92387953251128675613 : m == 2 ? 0.70710678118654752440
       : m == 3 ? 0.38268343236508977173 : m == 4 ? 0.0 : m == 5 ? -0.38268343236508977173
       : m == 6 ? -0.70710678118654752440 : m == 7 ? -0.92387953251128675613 : m == 8 ? -1.0
       : m == 9 ? -0.92387953251128675613 : m == 10 ? -0.70710678118654752440
       : m == 11 ? -0.38268343236508977173 : m == 12 ? 0.0 : m == 13 ? 0.38268343236508977173
       : m == 14 ? 0.70710678118654752440 : 0.92387953251128675613;
}
__host__ __device__ constexpr double sin16(int m) { return cos16(m - 4); }

// In-register DFT of length R (power of two, R <= 16) by recursive even/odd
// splitting.  DIR = -1: forward, DIR = +1: inverse (no scaling).
template <int R, int DIR> struct Dft {
  template <class C> __device__ static __forceinline__ void run(C (&a)[R]) {
    C e[R / 2], o[R / 2];
#pragma unroll
    for (int k = 0; k < R / 2; ++k) { e[k] = a[2 * k]; o[k] = a[2 * k + 1]; }
    Dft<R / 2, DIR>::run(e);
    Dft<R / 2, DIR>::run(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const int m = k * (16 / R);
      C t;
      if (m == 0) {
        t = o[k];
      } else if (m == 4) {  // multiply by DIR*i
        t.x = -DIR * o[k].y;
        t.y = DIR * o[k].x;
      } else {
        const C w = mk<C>(cos16(m), DIR * sin16(m));
        t = cmul(o[k], w);
      }
      a[k] = cadd(e[k], t);
      a[k + R / 2] = csub(e[k], t);
    }
  }
};
template <int DIR> struct Dft<1, DIR> {
  template <class C> __device__ static __forceinline__ void run(C (&)[1]) {}
};

// LDS line accessors --------------------------------------------------------
// Contiguous line: positions padded by one slot every 16 to spread the
// stride-16 writes of radix-16 stages over the banks.
template <class C> struct LdsRow {
  C* base;
  __device__ __forceinline__ C& operator[](int p) const { return base[p + (p >> 4)]; }
  // position a + k, k a compile-time offset of the unrolled loops:
  // (a + k) >> 4 = (a >> 4) + (k >> 4) when (a mod 16) + (k mod 16) < 16,
  // which holds for every access of the pass and line plans below, so the
  // thread's part is computed once and k stays an immediate offset
  __device__ __forceinline__ C& at(int a, int k) const { return base[a + (a >> 4) + k + (k >> 4)]; }
  static constexpr int padded(int n) { return n + (n >> 4); }
};
// Column of a [pos][W] tile (strided passes): pitch W + 1.
template <class C, int W> struct LdsCol {
  C* base;
  __device__ __forceinline__ C& operator[](int p) const { return base[p * (W + 1)]; }
  __device__ __forceinline__ C& at(int a, int k) const { return (*this)[a + k]; }
};
// Column of a [pos][W] tile with pitch W and one spare row every 16
// positions (N (W + W / 16) slots): the stride-16 writes of a radix-16 stage
// (positions 16 j + q) and the stride-T reads that follow spread over all
// banks, which the pitch W + 1 does not give them when W <= 8, and the
// address stays affine in the unrolled index.
template <class C, int W> struct LdsColP {
  C* base;
  __device__ __forceinline__ C& operator[](int p) const { return base[(p + (p >> 4)) * W]; }
  // (a + k) >> 4 = (a >> 4) + (k >> 4) when (a mod 16) + (k mod 16) < 16,
  // which holds for every access of the 16 x 16 x 4 plan (stage 1 writes
  // 16 j + q, stage 2 writes (j mod 16) + 256 (j / 16) + 16 q, reads t + 64 e):
  // the thread's part is computed once and k stays an immediate offset
  __device__ __forceinline__ C& at(int a, int k) const { return base[(a + (a >> 4)) * W + (k + (k >> 4)) * W]; }
};

// One Stockham stage.  `tw` is the forward twiddle table exp(-2 pi i k / N),
// k < N (in LDS or global).  `sync` is a functor executing the barrier used to
// separate the LDS write and read phases (block-wide).
template <class C, int N, int E, int R, int Ns, int DIR, class Line, class TwT, class Sync>
__device__ __forceinline__ void fft_stage(C (&v)[E], int t, const Line& line, const TwT* tw, Sync sync) {
  constexpr int T = N / E;
  constexpr int M = E / R;
  constexpr bool LAST = (Ns * R == N);
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int j = t + m * T;
    C a[R];
#pragma unroll
    for (int k = 0; k < R; ++k) a[k] = v[m + k * M];
    if (Ns > 1) {
      const int jm = j & (Ns - 1);
#pragma unroll
      for (int k = 1; k < R; ++k) {
        C w = cvt<C>(tw[(jm * k) * (N / (Ns * R))]);
        if (DIR > 0) w = cconj(w);
        a[k] = cmul(a[k], w);
      }
    }
    Dft<R, DIR>::run(a);
    if (LAST) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[m + q * M] = a[q];
    } else {
      const int base = (j / Ns) * Ns * R + (j & (Ns - 1));
#pragma unroll
      for (int q = 0; q < R; ++q) line.at(base, q * Ns) = a[q];
    }
  }
  if (!LAST) {
    sync();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = line.at(t, T * e);
    sync();
  }
}

// Radix plans.  Each plan lists its radices; E (elements per thread) is the
// largest radix and every radix divides it.
template <int... Rs> struct Plan {};

template <class C, int N, int E, int DIR, int Ns, class P> struct FftRun;
template <class C, int N, int E, int DIR, int Ns> struct FftRun<C, N, E, DIR, Ns, Plan<>> {
  template <class Line, class TwT, class Sync>
  __device__ static __forceinline__ void run(C (&)[E], int, const Line&, const TwT*, Sync) {}
};
template <class C, int N, int E, int DIR, int Ns, int R0, int... Rest>
struct FftRun<C, N, E, DIR, Ns, Plan<R0, Rest...>> {
  template <class Line, class TwT, class Sync>
  __device__ static __forceinline__ void run(C (&v)[E], int t, const Line& line, const TwT* tw, Sync sync) {
    fft_stage<C, N, E, R0, Ns, DIR>(v, t, line, tw, sync);
    FftRun<C, N, E, DIR, Ns * R0, Plan<Rest...>>::run(v, t, line, tw, sync);
  }
};

// Plans for the pass kernels (E <= 16).
template <int N> struct PassPlan;
template <> struct PassPlan<8> { using P = Plan<8>; static constexpr int E = 8; };
template <> struct PassPlan<16> { using P = Plan<16>; static constexpr int E = 16; };
template <> struct PassPlan<32> { using P = Plan<8, 4>; static constexpr int E = 8; };
template <> struct PassPlan<64> { using P = Plan<8, 8>; static constexpr int E = 8; };
template <> struct PassPlan<128> { using P = Plan<16, 8>; static constexpr int E = 16; };
template <> struct PassPlan<256> { using P = Plan<16, 16>; static constexpr int E = 16; };
template <> struct PassPlan<512> { using P = Plan<16, 16, 2>; static constexpr int E = 16; };
template <> struct PassPlan<1024> { using P = Plan<16, 16, 4>; static constexpr int E = 16; };

// Plans for the single-workgroup 1-D solver (E = 4: many threads per line).
template <int N> struct LinePlan;
template <> struct LinePlan<8> { using P = Plan<4, 2>; static constexpr int E = 4; };
template <> struct LinePlan<16> { using P = Plan<4, 4>; static constexpr int E = 4; };
template <> struct LinePlan<32> { using P = Plan<4, 4, 2>; static constexpr int E = 4; };
template <> struct LinePlan<64> { using P = Plan<4, 4, 4>; static constexpr int E = 4; };
template <> struct LinePlan<128> { using P = Plan<4, 4, 4, 2>; static constexpr int E = 4; };
template <> struct LinePlan<256> { using P = Plan<4, 4, 4, 4>; static constexpr int E = 4; };
template <> struct LinePlan<512> { using P = Plan<4, 4, 4, 4, 2>; static constexpr int E = 4; };
template <> struct LinePlan<1024> { using P = Plan<4, 4, 4, 4, 4>; static constexpr int E = 4; };

struct BlockSync {
  __device__ __forceinline__ void operator()() const { __syncthreads(); }
};
// Exchange barrier for a line held by a single wave: the LDS performs one
// wave's accesses in issue order, so only the compiler must keep the writes
// before the reads (and the reads before the next stage's writes).
struct WaveSync {
  __device__ __forceinline__ void operator()() const {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
};
// Exchange barrier for lines of T threads: wave-local when no line straddles
// a wave (T divides 64), block-wide otherwise.
template <int T> constexpr bool line_in_wave() { return (64 % T) == 0; }
template <int T> using LineSync = typename std::conditional<line_in_wave<T>(), WaveSync, BlockSync>::type;

// Reductions ----------------------------------------------------------------
// R is float (norms of complex64 iterations) or double (FP64 residuals).
template <class R> __device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of one value per thread over the block; result valid in every thread.
// `scratch` must hold 64 values (static LDS).  Deterministic: fixed shuffle
// tree inside each wave, waves added in index order.  Blocks smaller than one
// wave add through LDS serially.
template <class R> __device__ __forceinline__ R block_sum(R v, R* scratch) {
  const int nt = blockDim.x;
  if (nt < 64) {
    __syncthreads();
    scratch[threadIdx.x] = v;
    __syncthreads();
    R s = R(0);
    for (int i = 0; i < nt; ++i) s += scratch[i];
    __syncthreads();
    return s;
  }
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = nt >> 6;
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  R s = R(0);
  for (int w = 0; w < nw; ++w) s += scratch[w];
  __syncthreads();
  return s;
}

// Per-block partial of a grid reduction: the block's sum goes to row[block].
// Rows are summed in block order by k_sum_rows in a later launch, so the result
// is deterministic and no cross-block fence or atomic is needed (a device-scope
// fence writes back the whole L2 on this chip).
template <class R> __device__ __forceinline__ void block_partial(R v, R* scratch, R* row) {
  const R s = block_sum(v, scratch);
  if (row && threadIdx.x == 0) row[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = s;
}

}  // namespace usp
