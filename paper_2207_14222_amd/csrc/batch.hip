// Batched solve of many independent, uneven-size 2-D problems (host side).
//
// Two schedules (usp_solve_batched `variant` bit 2; bit 3 halves the column
// tiles of the grouped schedule):
//  * grouped (default): each launch covers the tiles of every active problem
//    (group.hpp); a refinement cycle is FIRST, k x [SYM, FUSED], RFWD, SYMA,
//    RINV, FINAL, with per-problem convergence, status and timestamps decided
//    on the device.  With use_graph the cycle is captured once in a hipGraph
//    and replayed; the task lists are compacted (and the graph re-captured)
//    when the active work has shrunk by a quarter.
//  * persistent: ONE launch in which each workgroup solves whole problems
//    taken from a ticket counter (batch.hpp); no cross-workgroup waits.
#include <hip/hip_runtime.h>

#include "group.hpp"
#include "op.hpp"

using namespace usp;

namespace {

long batch_lds_for(int n) {
  long b = 0;
  with_n(n, [&](auto NC) { b = batch_lds_bytes<decltype(NC)::value>(); });
  return b;
}

int g_lpb_rt(int n) {
  int v = 0;
  with_n(n, [&](auto NC) { v = g_lpb<decltype(NC)::value>(); });
  return v;
}
int g_w64_rt(int n, int nw) {
  int v = 0;
  with_n(n, [&](auto NC) { v = nw ? g_w64<decltype(NC)::value, 1>() : g_w64<decltype(NC)::value, 0>(); });
  return v;
}
int g_w128_rt(int n) {
  int v = 0;
  with_n(n, [&](auto NC) { v = g_w128<decltype(NC)::value>(); });
  return v;
}

template <int FL>
void launch_persistent(hipStream_t st, const BatchProblem* table, int nprob, unsigned* ticket, BatchResult* res,
                       long lds, int grid) {
  hipLaunchKernelGGL(k_reset_ticket, dim3(1), dim3(64), 0, st, ticket);
  hipLaunchKernelGGL((k_batch<FL>), dim3(grid), dim3(kBatchThreads), (size_t)lds, st, table, nprob, ticket, res);
}

int persistent_fl(int fl, hipStream_t st, const BatchProblem* table, int nprob, unsigned* ticket, BatchResult* res,
                  long lds, int grid) {
  hipError_t e;
  switch (fl) {
    case 1: e = hipFuncSetAttribute((const void*)k_batch<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); break;
    case 2: e = hipFuncSetAttribute((const void*)k_batch<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); break;
    case 3: e = hipFuncSetAttribute((const void*)k_batch<3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); break;
    default: e = hipFuncSetAttribute((const void*)k_batch<0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); break;
  }
  if (e != hipSuccess) return fail(USP_ERR_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  switch (fl) {
    case 1: launch_persistent<1>(st, table, nprob, ticket, res, lds, grid); break;
    case 2: launch_persistent<2>(st, table, nprob, ticket, res, lds, grid); break;
    case 3: launch_persistent<3>(st, table, nprob, ticket, res, lds, grid); break;
    default: launch_persistent<0>(st, table, nprob, ticket, res, lds, grid); break;
  }
  LAUNCHCHK("k_batch");
  return 0;
}

// workspace layout of a batch
struct BLayout {
  size_t table, res, ticket, state, xt, s64, s128, nslots, part, total;
  long max_tasks, pitch;
};

BLayout batch_layout(const usp_batch_item* items, int nprob) {
  BLayout L{};
  long sumn = 0, maxn = 8;
  for (int i = 0; i < nprob; ++i) {
    const long n = items[i].op ? items[i].op->d.n2 : 8;
    sumn += n;
    maxn = std::max(maxn, n);
  }
  L.max_tasks = sumn;
  L.pitch = maxn;
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = align_up(off + b);
    return o;
  };
  L.table = take(sizeof(BatchProblem) * nprob);
  L.res = take(sizeof(BatchResult) * nprob);
  L.ticket = take(256);
  L.state = take(sizeof(GState) * nprob);
  L.xt = take(sizeof(GTask) * L.max_tasks);
  L.s64 = take(sizeof(GTask) * L.max_tasks);
  L.s128 = take(sizeof(GTask) * L.max_tasks);
  L.nslots = take(sizeof(int) * nprob);
  L.part = take(sizeof(double) * nprob * L.pitch);
  L.total = off;
  return L;
}

int validate_items(const usp_batch_item* items, int nprob) {
  for (int i = 0; i < nprob; ++i) {
    const usp_op op = items[i].op;
    if (!op || !items[i].y_dev || !items[i].x_dev) return fail(USP_ERR_INVALID, "NULL item field");
    if (op->d.ndim != 2 || op->d.n0 != op->d.n2 || !op->refine)
      return fail(USP_ERR_INVALID, "batched items must be square 2-D operators prepared with USP_FLAG_REFINE");
    if (!(items[i].alpha > 0.0) || items[i].maxit < 0) return fail(USP_ERR_INVALID, "alpha > 0, maxit >= 0");
  }
  return 0;
}

BatchProblem make_problem(const usp_batch_item& it, int k) {
  const usp_op op = it.op;
  BatchProblem P{};
  const int n = op->d.n0;
  P.n = n;
  P.maxit = it.maxit;
  P.k = k;
  P.x_is_guess = it.x_is_guess;
  P.alpha = it.alpha;
  P.tol = it.tol;
  P.sa = std::pow(2.0 * M_PI / (n * op->sym.spacing[0]), 2);
  P.sx = std::pow(2.0 * M_PI / (n * op->sym.spacing[1]), 2);
  P.s0r = op->sa0[0];
  P.s0i = op->sa0[1];
  P.s2r = op->sa2[0];
  P.s2i = op->sa2[1];
  P.y64 = (const double2*)it.y_dev;
  P.B64 = (const double2*)op->B;
  P.x64 = (double2*)it.x_dev;
  P.t = (float2*)op->t;
  P.r32 = op->r32;
  P.d32 = op->d32;
  P.B32 = op->B32;
  P.S = op->S;
  P.twf = op->twf[ilog2(n)];
  P.twd = op->twd[ilog2(n)];
  return P;
}

// task lists of the active problems
struct Tasks {
  std::vector<GTask> xt, s64, s128;
};
Tasks build_tasks(const std::vector<BatchProblem>& tab, const std::vector<char>& active, int nw) {
  Tasks T;
  for (int p = 0; p < (int)tab.size(); ++p) {
    if (!active[p]) continue;
    const int n = tab[p].n;
    const int lpb = g_lpb_rt(n), w64 = g_w64_rt(n, nw), w128 = g_w128_rt(n);
    int slot = 0;
    for (int l = 0; l < n; l += lpb) T.xt.push_back(GTask{p, l, slot++, 0});
    for (int c = 0; c < n; c += w64) T.s64.push_back(GTask{p, c, 0, 0});
    for (int c = 0; c < n; c += w128) T.s128.push_back(GTask{p, c, 0, 0});
  }
  return T;
}

template <int FL, int NW>
int launch_inner_cycle(hipStream_t st, const BatchProblem* dtab, GState* dst, double* part, long pitch,
                       const GTask* xt, int nx, const GTask* s64, int ns64, const GTask* s128, int ns128,
                       const int* nslots, int nprob, int k) {
  // complex64 inner iterations on A d = r from d = 0
  // (problems whose cycle budget is below k skip the remaining launches)
  hipLaunchKernelGGL((k_gx<1, 0, NW>), dim3(nx), dim3(kGX), 0, st, xt, dtab, dst, part, pitch, 0);
  for (int j = 0; j < k; ++j) {
    hipLaunchKernelGGL((k_gs<0, NW>), dim3(ns64), dim3(kGS64 >> NW), 0, st, s64, dtab, dst, j);
    hipLaunchKernelGGL((k_gx<2, FL, NW>), dim3(nx), dim3(kGX), 0, st, xt, dtab, dst, part, pitch, j);
  }
  // FP64 residual of x + d (x += d) and the per-problem decision
  hipLaunchKernelGGL((k_gx<5, 0>), dim3(nx), dim3(kGX), 0, st, xt, dtab, dst, part, pitch, 0);
  hipLaunchKernelGGL((k_gs<1>), dim3(ns128), dim3(kGS128), 0, st, s128, dtab, dst, 0);
  hipLaunchKernelGGL((k_gx<4, 0>), dim3(nx), dim3(kGX), 0, st, xt, dtab, dst, part, pitch, 0);
  hipLaunchKernelGGL((k_gfinal<false>), dim3(nprob), dim3(256), 0, st, dtab, dst, part, pitch, nslots, k);
  return 0;
}

int inner_cycle_fl(int fl, int nw, hipStream_t st, const BatchProblem* dtab, GState* dst, double* part, long pitch,
                   const GTask* xt, int nx, const GTask* s64, int ns64, const GTask* s128, int ns128,
                   const int* nslots, int nprob, int k) {
#define USP_CYCLE(F, W) launch_inner_cycle<F, W>(st, dtab, dst, part, pitch, xt, nx, s64, ns64, s128, ns128, nslots, \
                                                 nprob, k)
  switch (fl + 4 * (nw ? 1 : 0)) {
    case 1: USP_CYCLE(1, 0); break;
    case 2: USP_CYCLE(2, 0); break;
    case 3: USP_CYCLE(3, 0); break;
    case 4: USP_CYCLE(0, 1); break;
    case 5: USP_CYCLE(1, 1); break;
    case 6: USP_CYCLE(2, 1); break;
    case 7: USP_CYCLE(3, 1); break;
    default: USP_CYCLE(0, 0); break;
  }
#undef USP_CYCLE
  LAUNCHCHK("grouped cycle");
  return 0;
}

int solve_grouped(const usp_batch_item* items, int nprob, int k, int fl, int nw, char* w, const BLayout& L,
                  hipStream_t st,
                  int use_graph, usp_batch_result* results, double* elapsed_ms, int clk_khz) {
  std::vector<BatchProblem> tab(nprob);
  for (int i = 0; i < nprob; ++i) tab[i] = make_problem(items[i], k);
  BatchProblem* dtab = (BatchProblem*)(w + L.table);
  GState* dst = (GState*)(w + L.state);
  GTask* dxt = (GTask*)(w + L.xt);
  GTask* ds64 = (GTask*)(w + L.s64);
  GTask* ds128 = (GTask*)(w + L.s128);
  int* dns = (int*)(w + L.nslots);
  double* part = (double*)(w + L.part);
  std::vector<int> nslots(nprob);
  for (int p = 0; p < nprob; ++p) {
    const int lpb = g_lpb_rt(tab[p].n);
    nslots[p] = (tab[p].n + lpb - 1) / lpb;  // tasks of the contiguous-axis passes
  }
  std::vector<char> active(nprob, 1);
  Tasks T = build_tasks(tab, active, nw);
  HIPCHK(hipMemcpy(dtab, tab.data(), sizeof(BatchProblem) * nprob, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dns, nslots.data(), sizeof(int) * nprob, hipMemcpyHostToDevice));
  auto upload = [&]() -> int {
    HIPCHK(hipMemcpy(dxt, T.xt.data(), sizeof(GTask) * T.xt.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ds64, T.s64.data(), sizeof(GTask) * T.s64.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ds128, T.s128.data(), sizeof(GTask) * T.s128.size(), hipMemcpyHostToDevice));
    return 0;
  };
  int rc;
  if ((rc = upload())) return rc;
  hipStream_t cs = st;
  if (use_graph) HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, st));
  if (cs != st) HIPCHK(hipStreamWaitEvent(cs, e0, 0));
  // init (B32, x = 0, |y|^2), then the first FP64 residual and decision
  hipLaunchKernelGGL((k_gx<0, 0>), dim3(T.xt.size()), dim3(kGX), 0, cs, dxt, dtab, dst, part, L.pitch, 0);
  hipLaunchKernelGGL((k_gfinal<true>), dim3(nprob), dim3(256), 0, cs, dtab, dst, part, L.pitch, dns, k);
  hipLaunchKernelGGL((k_gx<3, 0>), dim3(T.xt.size()), dim3(kGX), 0, cs, dxt, dtab, dst, part, L.pitch, 0);
  hipLaunchKernelGGL((k_gs<1>), dim3(T.s128.size()), dim3(kGS128), 0, cs, ds128, dtab, dst, 0);
  hipLaunchKernelGGL((k_gx<4, 0>), dim3(T.xt.size()), dim3(kGX), 0, cs, dxt, dtab, dst, part, L.pitch, 0);
  hipLaunchKernelGGL((k_gfinal<false>), dim3(nprob), dim3(256), 0, cs, dtab, dst, part, L.pitch, dns, 0);
  LAUNCHCHK("grouped init");
  std::vector<GState> hs(nprob);
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  size_t captured_x = 0;
  long cycles = 0, max_cycles = 0;
  for (int p = 0; p < nprob; ++p) max_cycles = std::max<long>(max_cycles, tab[p].maxit / std::max(k, 1) + 2);
  for (;;) {
    HIPCHK(hipMemcpyAsync(hs.data(), dst, sizeof(GState) * nprob, hipMemcpyDeviceToHost, cs));
    HIPCHK(hipStreamSynchronize(cs));
    size_t active_x = 0;
    int nact = 0;
    for (int p = 0; p < nprob; ++p) {
      active[p] = !hs[p].done;
      nact += active[p];
      if (active[p]) active_x += nslots[p];
    }
    if (nact == 0 || cycles++ > max_cycles) break;
    const bool compact = !use_graph || !exec || active_x * 4 <= captured_x * 3;
    if (compact) {
      T = build_tasks(tab, active, nw);
      if ((rc = upload())) break;
    }
    if (use_graph) {
      if (compact || !exec) {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        rc = inner_cycle_fl(fl, nw, cs, dtab, dst, part, L.pitch, dxt, (int)T.xt.size(), ds64, (int)T.s64.size(), ds128,
                            (int)T.s128.size(), dns, nprob, k);
        hipError_t ec = hipStreamEndCapture(cs, &graph);
        if (!rc && ec != hipSuccess) rc = fail(USP_ERR_HIP, std::string("capture: ") + hipGetErrorString(ec));
        if (!rc && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
          rc = fail(USP_ERR_HIP, "hipGraphInstantiate failed");
        if (rc) break;
        captured_x = active_x;
      }
      if (hipGraphLaunch(exec, cs) != hipSuccess) {
        rc = fail(USP_ERR_HIP, "hipGraphLaunch failed");
        break;
      }
    } else {
      if ((rc = inner_cycle_fl(fl, nw, cs, dtab, dst, part, L.pitch, dxt, (int)T.xt.size(), ds64, (int)T.s64.size(),
                               ds128, (int)T.s128.size(), dns, nprob, k)))
        break;
    }
  }
  if (exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  HIPCHK(hipEventRecord(e1, cs));
  HIPCHK(hipEventSynchronize(e1));
  if (cs != st) {
    HIPCHK(hipStreamWaitEvent(st, e1, 0));
    hipStreamDestroy(cs);
  }
  float ms = 0.f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  if (elapsed_ms) *elapsed_ms = ms;
  unsigned long long tmin = ~0ull;
  for (const GState& g : hs) tmin = std::min(tmin, g.t_start);
  int worst = USP_OK;
  for (int p = 0; p < nprob; ++p) {
    const GState& g = hs[p];
    const int status = g.done ? g.status : USP_MAXIT;
    if (results) {
      results[p].iterations = g.iterations;
      results[p].status = status;
      results[p].rho = g.rho;
      results[p].t_done_ms = clk_khz > 0 ? (double)(g.t_done - tmin) / clk_khz : 0.0;
    }
    if (status < 0) worst = status;
    else if (worst >= 0 && status > worst) worst = status;
  }
  if (worst < 0) return fail(worst, "a batched problem produced non-finite values");
  return worst;
}

int solve_persistent(const usp_batch_item* items, int nprob, int k, int fl, char* w, const BLayout& L, hipStream_t st,
                     int use_graph, usp_batch_result* results, double* elapsed_ms, int clk_khz, int ncu) {
  // table in largest-first order
  std::vector<int> order(nprob);
  for (int i = 0; i < nprob; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return items[a].op->d.N > items[b].op->d.N; });
  std::vector<BatchProblem> tab(nprob);
  long lds = 0;
  for (int j = 0; j < nprob; ++j) {
    tab[j] = make_problem(items[order[j]], k);
    lds = std::max(lds, batch_lds_for(tab[j].n));
  }
  BatchProblem* dtab = (BatchProblem*)(w + L.table);
  BatchResult* dres = (BatchResult*)(w + L.res);
  unsigned* ticket = (unsigned*)(w + L.ticket);
  HIPCHK(hipMemcpyAsync(dtab, tab.data(), sizeof(BatchProblem) * nprob, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  const int grid = std::min(nprob, std::max(ncu, 1));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int rc = 0;
  if (use_graph) {
    hipStream_t cs;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIPCHK(hipEventRecord(e0, st));
    HIPCHK(hipStreamWaitEvent(cs, e0, 0));
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    rc = persistent_fl(fl, cs, dtab, nprob, ticket, dres, lds, grid);
    hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (!rc && ec != hipSuccess) rc = fail(USP_ERR_HIP, std::string("capture: ") + hipGetErrorString(ec));
    if (!rc && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
      rc = fail(USP_ERR_HIP, "hipGraphInstantiate failed");
    if (!rc) {
      HIPCHK(hipEventRecord(e0, cs));
      HIPCHK(hipGraphLaunch(exec, cs));
      HIPCHK(hipEventRecord(e1, cs));
      HIPCHK(hipStreamWaitEvent(st, e1, 0));
      HIPCHK(hipEventSynchronize(e1));
    }
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    hipStreamDestroy(cs);
  } else {
    HIPCHK(hipEventRecord(e0, st));
    rc = persistent_fl(fl, st, dtab, nprob, ticket, dres, lds, grid);
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
  }
  float ms = 0.f;
  if (!rc) hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  if (elapsed_ms) *elapsed_ms = ms;
  std::vector<BatchResult> hres(nprob);
  HIPCHK(hipMemcpy(hres.data(), dres, sizeof(BatchResult) * nprob, hipMemcpyDeviceToHost));
  unsigned long long tmin = ~0ull;
  for (const BatchResult& r : hres) tmin = std::min(tmin, r.t_start);
  int worst = USP_OK;
  for (int j = 0; j < nprob; ++j) {
    const BatchResult& r = hres[j];
    if (results) {
      usp_batch_result& o = results[order[j]];
      o.iterations = r.iterations;
      o.status = r.status;
      o.rho = r.rho;
      o.t_done_ms = clk_khz > 0 ? (double)(r.t_done - tmin) / clk_khz : 0.0;
    }
    if (r.status < 0) worst = r.status;
    else if (worst >= 0 && r.status > worst) worst = r.status;
  }
  if (worst < 0) return fail(worst, "a batched problem failed (non-finite values or unsupported size)");
  return worst;
}

}  // namespace

extern "C" {

int usp_batch_workspace_bytes(const usp_batch_item* items, int nprob, size_t* bytes) {
  if (!items || nprob < 1 || !bytes) return fail(USP_ERR_INVALID, "items, nprob >= 1 and bytes required");
  int rc = validate_items(items, nprob);
  if (rc) return rc;
  *bytes = batch_layout(items, nprob).total;
  return 0;
}

int usp_solve_batched(const usp_batch_item* items, int nprob, int refine_every, int variant, void* ws,
                      size_t ws_bytes, void* stream, int use_graph, usp_batch_result* results, double* elapsed_ms) {
  if (!items || nprob < 1 || !ws || refine_every < 1 || variant < 0 || variant > 15 || (variant & 12) == 12)
    return fail(USP_ERR_INVALID, "invalid argument (variant 0..11 or 8..11 with bit 2 clear)");
  int rc = validate_items(items, nprob);
  if (rc) return rc;
  const BLayout L = batch_layout(items, nprob);
  if (ws_bytes < L.total) return fail(USP_ERR_WORKSPACE, "batch workspace too small: need " + std::to_string(L.total));
  if (((uintptr_t)ws) & 255) return fail(USP_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  int dev = 0, ncu = 0, clk_khz = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, dev));
  const int fl = variant & 3;
  if (variant & 4)
    return solve_persistent(items, nprob, refine_every, fl, (char*)ws, L, (hipStream_t)stream, use_graph, results,
                            elapsed_ms, clk_khz, ncu);
  return solve_grouped(items, nprob, refine_every, fl, (variant >> 3) & 1, (char*)ws, L, (hipStream_t)stream,
                       use_graph, results, elapsed_ms, clk_khz);
}

int usp_autotune_batched(const usp_batch_item* items, int nprob, int refine_every, void* ws, size_t ws_bytes,
                         void* stream, int* best_variant) {
  if (!items || nprob < 1 || !best_variant) return fail(USP_ERR_INVALID, "invalid argument");
  std::vector<usp_batch_item> short_items(items, items + nprob);
  for (auto& it : short_items) {
    it.maxit = std::min(it.maxit, 2 * refine_every);
    it.tol = 0.0;
    it.x_is_guess = 0;
  }
  double best = INFINITY;
  *best_variant = 0;
  for (int v = 0; v < 12; ++v) {   // grouped 0-3, persistent 4-7, grouped with narrow column tiles 8-11
    double ms = 0.0;
    int rc = usp_solve_batched(short_items.data(), nprob, refine_every, v, ws, ws_bytes, stream, 1, nullptr, &ms);
    if (rc < 0) return rc;
    if (ms < best) {
      best = ms;
      *best_variant = v;
    }
  }
  return 0;
}

}  // extern "C"
