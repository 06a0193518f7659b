/*
 * usp.h -- C ABI of the MI355X (gfx950) universal-split-preconditioner solver.
 *
 * Method: Vettenburg & Vellekoop, "A universal matrix-free split preconditioner
 * for the fixed-point iterative solution of non-symmetric linear systems"
 * (arXiv 2207.14222).  A canonical system A x = y with A = L + V, ||V|| < 1,
 * A accretive (Sec. 2, Theorem 1) is solved by the preconditioned fixed-point
 * iteration with the forward problem eliminated (Sec. 2.1, Algorithm 1):
 *
 *     Delta = B [ (L + I)^-1 (B x + y) - x ],   x <- x + alpha Delta,   B = I - V,
 *
 * with (L + I)^-1 applied through the analytic Fourier symbol of L
 * (Eq. laplacian_inverse): F^-1 diag(1/(l(p) + 1)) F on a periodic grid.
 *
 * Conventions (all entry points):
 *   - Return value: 0 = OK / converged; > 0 = solver outcome (USP_MAXIT,
 *     USP_STAGNATED, USP_DIVERGED: the paper's "m", "s", "d" of Table 1);
 *     < 0 = error (USP_ERR_*).  The message of the last error on the calling
 *     thread is returned by usp_last_error().  No C++ exception crosses the ABI.
 *   - Device buffers ("_dev") are plain device pointers owned by the caller,
 *     C-ordered (last axis contiguous), complex interleaved (re, im), 8-byte
 *     aligned at least; dtype USP_C64 = float2 elements, USP_C128 = double2.
 *   - The library never allocates device memory: every scratch array lives in a
 *     caller-provided workspace of usp_workspace_bytes() bytes.
 *   - All device work is issued on the stream given to usp_prepare_operator
 *     (a hipStream_t passed as void*; NULL = default stream).  Solves are
 *     synchronous with respect to their host outputs.  An operator handle is
 *     not thread-safe; use one handle per stream.
 *   - Grid sizes: ndim 1: n in {8, ..., 1024} (power of two, single-workgroup
 *     solver); ndim 2 or 3: every axis in {8, ..., 1024} (power of two).
 */
#ifndef USP_H
#define USP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status and error codes */
#define USP_OK 0
#define USP_MAXIT 1
#define USP_STAGNATED 2
#define USP_DIVERGED 3
#define USP_ERR_INVALID (-1)
#define USP_ERR_UNSUPPORTED_SHAPE (-2)
#define USP_ERR_NOT_CONTRACTIVE (-3)
#define USP_ERR_HIP (-4)
#define USP_ERR_NAN (-5)
#define USP_ERR_WORKSPACE (-6)

/* element types */
#define USP_C64 0
#define USP_C128 1

/* prepare flags */
#define USP_FLAG_REFINE 1 /* complex64 inner iterations, FP64 outer refinement (needs USP_C128 buffers) */
#define USP_FLAG_ANTISYM 2 /* 1-D: solve the antisymmetrised system (Sec. 2.2) on x = [x~; x~'] (2N values) */

/* bias kinds for usp_smallest_circle */
#define USP_BIAS_COMPLEX 0
#define USP_BIAS_REAL 1

/*
 * Fourier symbol of L (Sec. 2.2 canonical form; Sec. 3.1 Helmholtz, 3.2
 * diffusion, 3.3 pantograph):
 *     l(p) = s * (a0 + a2 |p|^2 + a1 * i * p_0)        (a1 term: ndim == 1 only)
 * on the FFT grid p_k = 2 pi fftfreq(n_k, h_k).  When nyquist_zero is set, the
 * first-derivative term i p is zero at the Nyquist index (keeps d/dt
 * skew-Hermitian).  Complex coefficients are (re, im) pairs.  A 2-D or 3-D
 * symbol with a1 != 0 or nyquist_zero set is rejected (USP_ERR_INVALID).
 *   Helmholtz:  s = 1/c, a0 = kbar^2, a2 = -1            (c = i R / 0.95)
 *   diffusion:  s = 1/c, a0 = mubar - i omega/v, a2 = D  (c = R / 0.95)
 *   pantograph: s = 1/c, a0 = abar, a1 = 1               (c real)
 */
typedef struct {
  int ndim;           /* 1, 2 or 3 */
  int shape[3];       /* C order; shape[ndim-1] is the contiguous axis */
  double spacing[3];  /* grid spacing h per axis */
  double s[2];
  double a0[2];
  double a1[2];
  double a2[2];
  int nyquist_zero;
} usp_symbol;

/* Pantograph dilation gather (Sec. 3.3, ndim == 1 only): V adds
 *     (G x)_j = g0_j x[idx_j] + g1_j x[min(idx_j + 1, n - 1)].
 * idx_dev: int32[n]; g0_dev, g1_dev: complex[n] of the operator's dtype.
 * Device arrays, caller-owned, must outlive the handle. */
typedef struct {
  const int32_t* idx_dev;
  const void* g0_dev;
  const void* g1_dev;
} usp_gather;

typedef struct usp_op_s* usp_op;

/* Launch plan of the complex64 iteration passes (2-D / 3-D grids).  Every plan
 * computes bit-identical results; only speed differs.
 *   x_prefetch  1: the fused contiguous-axis pass loads x, B, y before its
 *               inverse FFT (more registers, more loads in flight)
 *   x_stream    1: the fused pass reads x, B, y and writes x with non-temporal
 *               (streaming) accesses so the temporary spectrum stays cached
 *   w_mid       column-tile width (elements, 4/8/16/32; 0 = default) of the
 *               middle-axis passes (3-D)
 *   w_sym       column-tile width of the symbol pass (first axis)
 *   r_load      FP64 residual's last pass: bit 0 loads x, B, y before its
 *               inverse FFT, bit 1 reads them with non-temporal accesses */
typedef struct {
  int x_prefetch;
  int w_mid;
  int w_sym;
  int x_stream;
  int r_load;
} usp_plan;

/* Workspace size for an operator.  dtype: USP_C64 or USP_C128; flags: 0 or
 * USP_FLAG_REFINE (requires USP_C128).  Errors: INVALID, UNSUPPORTED_SHAPE. */
int usp_workspace_bytes(const usp_symbol* L, int dtype, int flags, size_t* bytes);

/* Prepare an operator handle (Sec. 2.1: the iteration needs B = I - V and the
 * symbol of L).
 *   B_dev      diagonal of B = 1 - v (N elements of dtype), caller-owned, must
 *              outlive the handle.  Validated: max |1 - B| must be < 1
 *              (||V|| < 1, Theorem 1), else USP_ERR_NOT_CONTRACTIVE (diagonal
 *              part only when a gather is present).
 *   gather     NULL, or the pantograph gather (ndim == 1).
 *   workspace  device buffer of usp_workspace_bytes() bytes (>= 256-B aligned);
 *              owned by the caller, used exclusively by this handle.
 *   stream     hipStream_t or NULL.
 * In refined mode B_dev is complex128; the library writes a complex64 copy of
 * B into the workspace for the inner iterations. */
int usp_prepare_operator(const usp_symbol* L, int dtype, int flags, const void* B_dev, const usp_gather* gather,
                         void* workspace_dev, size_t workspace_bytes, void* stream, usp_op* out);

/* Algorithm 1 (Sec. 2.1) until ||y - A x|| / ||y|| < tol.
 *   y_dev, x_dev   right-hand side and solution (dtype of the handle; complex128
 *                  in refined mode).  x_dev is read as the initial guess when
 *                  x_is_guess != 0, otherwise the iteration starts from x = 0.
 *                  x_is_guess == 2 (2-D / 3-D): the guess is judged first --
 *                  its FP64 residual is the first hist_true entry, and if it
 *                  is not below ||y|| the guess is discarded and the solve
 *                  starts from x = 0 (for learned or otherwise untrusted
 *                  guesses).  On return x_dev holds the last iterate.
 *   alpha          step size (> 0; (0, 1] is always contractive, Corollary 1).
 *   check_every    true residual evaluated (in FP64) every check_every
 *                  iterations; in refined mode this is the refinement interval
 *                  k (residual recomputed and accumulated in FP64 every k steps),
 *                  except that a cycle is shortened to the number of steps the
 *                  current rate of ||Delta|| (last 10 iterations) predicts for
 *                  reaching tol when that is under half the cycle.
 *   iters_out      iterations performed.
 *   hist_pre       host array, may be NULL: ||Delta_i||^2 for i < hist_pre_cap.
 *   hist_true      host array, may be NULL: pairs (iteration, ||y - A x||/||y||)
 *                  for each check, up to hist_true_cap pairs; n_true_out gets
 *                  the number of checks performed.
 * Returns USP_OK (converged), USP_MAXIT, USP_STAGNATED (no 1% improvement of
 * the true residual over 8 checks), USP_DIVERGED, or an error. */
int usp_solve(usp_op op, const void* y_dev, void* x_dev, int x_is_guess, double alpha, double tol, int maxit,
              int check_every, int* iters_out, double* hist_pre, int hist_pre_cap, double* hist_true,
              int hist_true_cap, int* n_true_out);

/* Test hook: exactly K iterations of Algorithm 1 from x_dev (in/out; x_is_guess
 * as in usp_solve).  hist_pre as in usp_solve.  Not available in refined mode. */
int usp_iterate(usp_op op, const void* y_dev, void* x_dev, int x_is_guess, double alpha, int K, double* hist_pre,
                int hist_pre_cap);

/* True relative residual ||y - A x|| / ||y|| evaluated in FP64 (A = L + V,
 * canonical form, Sec. 2.2).  rnorm_out / ynorm_out may be NULL. */
int usp_residual(usp_op op, const void* y_dev, const void* x_dev, double* rel_out, double* rnorm_out,
                 double* ynorm_out);

/* Per-pass timing with hipEvents on the handle's stream (2-D / 3-D grids).
 * Runs the first pass and K iterations of Algorithm 1 from x = 0 on y_dev /
 * x_dev (x_dev is overwritten) and one FP64 residual evaluation, with an event
 * pair around every launch, then K more iterations bracketed by one event pair.
 * In refined mode the iterations are the complex64 inner ones (on workspace
 * copies; x_dev is the complex128 solution, only read) after one FP64 residual.
 * pass_ms[USP_NPASS]: average milliseconds per launch of each pass kind (0 if
 * the kind was not launched), indexed by USP_PASS_*; iter_ms (may be NULL):
 * average milliseconds per whole iteration. */
#define USP_NPASS 11
#define USP_PASS_X_FUSED 0   /* inverse FFT (contiguous axis), update, norm, next forward FFT */
#define USP_PASS_M_FWD 1     /* forward FFT along the middle axis (3-D) */
#define USP_PASS_SYM 2       /* forward FFT, 1/(N (l + 1)), inverse FFT along the first axis */
#define USP_PASS_M_INV 3     /* inverse FFT along the middle axis (3-D) */
#define USP_PASS_X_FIRST 4   /* B x + y and its forward FFT (first iteration) */
#define USP_PASS_R_FWD 5     /* FP64 residual: forward FFT of x (contiguous axis) */
#define USP_PASS_R_MFWD 6
#define USP_PASS_R_SYM 7     /* FP64 residual: forward FFT, l(p)/N, inverse FFT */
#define USP_PASS_R_MINV 8
#define USP_PASS_R_INV 9     /* FP64 residual: inverse FFT, r = y - A x, ||r||^2 */
#define USP_PASS_REDUCE 10   /* ordered sum of per-block partial norms */
int usp_profile(usp_op op, const void* y_dev, void* x_dev, double alpha, int K, double* pass_ms, double* iter_ms);

/* Read / set the launch plan of a handle (see usp_plan).  Invalid widths:
 * USP_ERR_INVALID; widths that do not fit an axis fall back to the largest
 * valid smaller width at launch. */
int usp_get_plan(usp_op op, usp_plan* out);
int usp_set_plan(usp_op op, const usp_plan* plan);

/* Autotuner: times `reps` iterations (best of two) for every candidate plan on
 * y_dev / x_dev (x_dev overwritten; in refined mode the workspace copies are
 * used) and keeps the fastest in the handle, then times one FP64 residual of
 * x_dev for each r_load and keeps the fastest; best_out may be NULL.  Results
 * of all candidates are identical, so tuning never changes a solution. */
int usp_autotune(usp_op op, const void* y_dev, void* x_dev, double alpha, int reps, usp_plan* best_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * true residual of usp_residual computed without an operator handle or a
 * workspace, every temporary (twiddle tables, partial sums, the FP64 spectrum)
 * in a static device array of USP_STATIC_SCRATCH_BYTES that each GPU holds
 * until the process ends.  L: the symbol (as for usp_prepare_operator; no
 * gather term), dtype USP_C64 or USP_C128 for B_dev, y_dev, x_dev (device,
 * contiguous, C order, caller-owned).  Outputs as usp_residual.  Grids whose
 * temporaries exceed the array (2-D / 3-D: about 16 bytes per point plus
 * partial rows; 128^3 fits, 256^3 does not): USP_ERR_WORKSPACE.  Runs on
 * `stream`, which must belong to the current device, and synchronises it.
 * Allocates nothing: no hipMalloc, hipFree or allocating library call.
 * Calls that overlap on one GPU share its array and race; serialise them. */
#define USP_STATIC_SCRATCH_BYTES (64 * 1024 * 1024)
int usp_residual_static(const usp_symbol* L, int dtype, const void* B_dev, const void* y_dev, const void* x_dev,
                        double* rel_out, double* rnorm_out, double* ynorm_out, void* stream);

/* Measurement hook (not part of the method): copy `bytes` bytes from src_dev
 * to dst_dev on `stream` with non-temporal 16-byte loads and stores, the
 * streaming ceiling that the pass kernels' HBM rates are compared with.  Both
 * pointers 16-byte aligned, bytes a multiple of 16, buffers not overlapping
 * (USP_ERR_INVALID otherwise).  Asynchronous. */
int usp_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream);

/* ---- batched persistent solve (many uneven-size 2-D problems) ----------- */

/* One problem of a batch: a square 2-D operator prepared with
 * USP_FLAG_REFINE (its workspace holds the problem's scratch), the
 * complex128 right-hand side and solution buffers, and the solve settings. */
typedef struct {
  usp_op op;
  const void* y_dev;
  void* x_dev;
  int x_is_guess;
  double alpha;
  double tol;
  int maxit;
} usp_batch_item;

typedef struct {
  int iterations;    /* complex64 iterations performed */
  int status;        /* 0 converged, 1 maxit, 2 stagnated, < 0 error */
  double rho;        /* last ||y - A x||/||y|| (FP64) */
  double t_done_ms;  /* device time from the first workgroup's start to this problem's end */
} usp_batch_result;

/* Device workspace (problem table, task lists, states, partial sums) for a batch. */
int usp_batch_workspace_bytes(const usp_batch_item* items, int nprob, size_t* bytes);

/* Solve every item with the refined method (complex64 iterations of
 * Algorithm 1, FP64 residual recomputed and accumulated every refine_every
 * iterations, stop at ||y - A x||/||y|| < tol).  A problem's cycle is cut to
 * what remains of its maxit, and to the number of iterations that the rate
 * of its FP64 residual over the previous cycle predicts for reaching tol when
 * that is under half of refine_every.  variant: bits 0-1 select the fused-pass access
 * plan (bit 0 prefetch, bit 1 streaming); bit 2 selects the schedule:
 *   0 grouped: every launch covers the tiles of all active problems (the whole
 *     chip works on the batch); per-problem convergence, status and
 *     timestamps are decided on the device; with use_graph = 1 one refinement
 *     cycle is captured in a hipGraph and replayed (re-captured when the
 *     active work shrinks by a quarter);
 *   4 persistent: ONE launch (captured in a hipGraph when use_graph = 1) in
 *     which each workgroup takes whole problems, largest first, from a ticket
 *     counter and solves them alone; workgroups never wait for each other;
 * bit 3 (grouped schedule only; variants 8-11): the column pass works on
 * tiles half as wide (4 columns for 1024^2 problems, 8 for the others) in
 * blocks of 256 threads instead of 512.  Every variant gives the same
 * solution to rounding; variants 12-15 are invalid.
 * Graphs run on a private default-priority stream ordered after `stream`.
 * results (host, may be NULL; in item order) and elapsed_ms (device time) are
 * filled in.  Returns the worst status (errors < 0 first). */
int usp_solve_batched(const usp_batch_item* items, int nprob, int refine_every, int variant, void* workspace_dev,
                      size_t workspace_bytes, void* stream, int use_graph, usp_batch_result* results,
                      double* elapsed_ms);

/* Autotuner of the batched solve: runs 2 * refine_every iterations of every
 * problem with each variant (0..11) and returns the fastest (overwrites x_dev). */
int usp_autotune_batched(const usp_batch_item* items, int nprob, int refine_every, void* workspace_dev,
                         size_t workspace_bytes, void* stream, int* best_variant);

/* Destroy a handle (frees host memory only). */
int usp_destroy(usp_op op);

/* Message of the last error on this thread ("" if none). */
const char* usp_last_error(void);

/* ---- canonicalisation helpers (Sec. 2.2, 3.1, 3.2) ---------------------- */

/* Centre and radius of the smallest disc containing n complex points (host
 * array of 2n doubles).  kind USP_BIAS_COMPLEX: unrestricted centre (the
 * smallest-circle problem of Sec. 3.1); USP_BIAS_REAL: centre restricted to the
 * real axis (real bias, Sec. 4.1).  centre_out: 2 doubles. */
int usp_smallest_circle(const double* pts_host, size_t n, int kind, double* centre_out, double* radius_out);

/* B and y of a canonical problem with diagonal V (Sec. 2.2):
 *     B = 1 - (q - bias)/c,   y = src_scale * S / c
 * q_dev, S_dev: complex128[n] device arrays (k^2 or mu_a, and the raw source);
 * B_dev, y_dev: outputs of dtype (either may be NULL).  Helmholtz: q = k^2,
 * src_scale = -1; diffusion: q = mu_a (+0i), src_scale = +1.  Runs on `stream`. */
int usp_canonical_fields(const void* q_dev, const void* S_dev, size_t n, const double* bias, const double* c,
                         double src_scale, int dtype, void* B_dev, void* y_dev, void* stream);

/* Helmholtz canonical form (Sec. 3.1, Eq. laplacian_inverse): raw problem
 * (laplacian + k^2) psi = -S.  Computes kbar^2 (smallest-circle centre of the n
 * values k2_host, complex or real-axis per bias_kind) and c = i R / vnorm, or
 * takes both from `given` = {kbar^2 re, im, c re, im} (required for a
 * homogeneous medium, R = 0).  grid: ndim/shape/spacing to copy; sym_out gets
 * s = 1/c, a0 = kbar^2, a2 = -1.  c_out, bias_out: 2 doubles each.  Host only.
 * Then usp_canonical_fields(k^2, S, bias, c, -1, ...) gives B and y on device. */
int usp_canonical_helmholtz(const double* k2_host, size_t n, int bias_kind, const double* given, double vnorm,
                            const usp_symbol* grid, usp_symbol* sym_out, double* c_out, double* bias_out);

/* Constant-D frequency-domain diffusion (Sec. 3.2, scalar form):
 * A0 = -D laplacian + mu_a - i omega/v.  mubar = midrange of mu_a (smallest
 * circle of a real set), c = R / vnorm.  sym_out: s = 1/c,
 * a0 = mubar - i omega/v, a2 = D.  Then usp_canonical_fields(mu_a, S, mubar, c,
 * +1, ...).  Host only. */
int usp_canonical_diffusion(const double* mu_host, size_t n, double D, double omega_over_v, double vnorm,
                            const usp_symbol* grid, usp_symbol* sym_out, double* c_out, double* bias_out);

/* Shifted Schrodinger operator (Sec. 4, Eq. schrodinger; unit mass, natural
 * units): H + shift = -1/2 laplacian + V + shift on the grid, canonicalised as
 * the constant-D diffusion operator with D = 1/2, mu = V + shift, omega = 0.
 * V_host: n real potential values.  c = (max V - min V)/(2 vnorm);
 * sym_out: s = 1/c, a0 = midrange(V) + shift, a2 = 1/2; bias_out = the field
 * bias midrange(V) for usp_canonical_fields(V, S, bias, c, +1, ...), which
 * gives B = 1 - (V - midrange(V))/c.  Energies: E = c lam - shift.  A constant
 * V (R = 0) or a non-finite value: USP_ERR_INVALID / USP_ERR_NAN.  Host only. */
int usp_canonical_schrodinger(const double* V_host, size_t n, double shift, double vnorm, const usp_symbol* grid,
                              usp_symbol* sym_out, double* c_out, double* bias_out);

/* Pantograph canonical form (Sec. 3.3, Eq. pantograph-A) on t_j = t0 + j h:
 * A x = c^-1 [(d/dt + a) x + b x(lam t)], y = c^-1 [b x0(lam t) + x0(t0) delta(t - t0)],
 * the delta sampled as x0(t0)/h at j = 0.  Inputs (host, n complex = 2n doubles):
 * a, b, x0_lam_t (x0(lam t_j) where lam t_j < t0, else 0), x0_t0 (2 doubles).
 * abar = smallest-circle centre of a; the dilation is a linear-interpolation
 * gather S; c = (sup|a - abar| + sup|b| ||S||_2)/vnorm (real), which bounds
 * ||V|| by vnorm.  Outputs (host): sym_out (s = 1/c, a0 = abar, a1 = 1,
 * nyquist_zero = 1), B_out = 1 - (a - abar)/c, gather idx_out / g0_out / g1_out
 * (usp_gather layout), y_out, c_out, bias_out (2 doubles each).  For the
 * antisymmetrised form (USP_FLAG_ANTISYM) the caller clears
 * sym_out->nyquist_zero: with a zero derivative at the Nyquist index the
 * alternating grid vector is almost in the null space of A (the interpolation
 * gather nearly annihilates it) and the iteration stalls. */
int usp_canonical_pantograph(const double* a, const double* b, int n, double lam, double t0, double h,
                             const double* x0_lam_t, const double* x0_t0, double vnorm, usp_symbol* sym_out,
                             double* B_out, int32_t* idx_out, double* g0_out, double* g1_out, double* y_out,
                             double* c_out, double* bias_out);

/* ---- steady diffusion in flux form with a tensor coefficient ------------
 *
 * Sec. 3.2 (Eq. diffusion-equation-matrix-form) keeps the flux J as an unknown:
 * div J + mu u = S and D^-1 J + grad u = 0 on a periodic 2-D or 3-D grid
 * (shape n[0..ndim), the last axis contiguous), spacing h, spectral
 * derivatives whose Nyquist mode is zero.  Unknown x = [u; J_x; J_y (; J_z)],
 * stored component-major as 1 + ndim planes of n[0]*..*n[ndim-1] complex
 * values (complex64 or complex128 per dtype); flux component k pairs with
 * axis ndim - k (J_x with the contiguous axis).  D is given per voxel in the
 * same (x, y, z) order.  L keeps the derivatives and the biases mubar
 * (smallest circle of {mu}) and Dibar (smallest circle of each element of
 * {D^-1}); V = blockdiag(mu - mubar, D^-1 - Dibar) per voxel.  The system is
 * equilibrated by a diagonal S = diag(s) and scaled by a real c so that
 * ||V|| = vnorm:
 *     A = S A~ S / c,   y = S [source; 0 ..] / sqrt(c),   [u; J] = S x / sqrt(c). */
typedef struct {
  int ndim;             /* 2 or 3 */
  int n[3];             /* grid sides (n[2] = 1 in 2-D) */
  double h;
  double s[4];          /* equilibration: u, then J_x, J_y (, J_z) */
  double c;             /* overall scale (real, > 0) */
  double mubar[2];      /* re, im */
  double dibar[9][2];   /* Dibar row-major ndim x ndim in (x, y, z) order (re, im) */
} usp_flux_symbol;

/* Canonical flux form (host).  Inputs, row-major over the grid of `shape`
 * (ndim entries, each >= 2), n voxels: mu (n complex, 2n doubles), D (per
 * voxel the ndim x ndim tensor row-major: ndim^2 n complex), source (n
 * complex).  Circles of a constant set are the value itself with radius 0.
 * The radii dV = blockdiag(R_mu, [R_ab]) are equilibrated symmetrically
 * (s_i <- s_i / sqrt(max_j s_i dV_ij s_j), 50 sweeps; zero rows keep
 * s_i = 1); then c = max over voxels of the spectral norm of S V~ S, divided
 * by vnorm (1 if that is 0).  Outputs (host): sym_out; bu_out (n complex) =
 * 1 - s0^2 (mu - mubar)/c; b2_out (ndim^2 n complex, per voxel row-major) =
 * I - S' (D^-1 - Dibar) S' / c with S' = diag(s_1 ..); y_out ((1 + ndim) n
 * complex).  Returns USP_ERR_INVALID for NULL pointers, ndim not 2 or 3, a
 * side < 2, h <= 0, vnorm outside (0, 1) or a singular D, USP_ERR_NAN for
 * non-finite input. */
int usp_canonical_flux(const double* mu_host, const double* D_host, const double* source_host, int ndim,
                       const int* shape, double h, double vnorm, usp_flux_symbol* sym_out, double* bu_out,
                       double* b2_out, double* y_out);

/* Device workspace of a flux-form solve (every side a power of two in [8, 1024]). */
int usp_flux_workspace_bytes(const usp_flux_symbol* sym, int dtype, size_t* bytes);

/* Algorithm 1 on the flux-form system: per iteration t = B x + y, u = (L + I)^-1 t
 * (FFTs of the 1 + ndim planes; per Fourier mode the inverse of the
 * (1 + ndim) x (1 + ndim) block I + S L~(p) S / c), Delta = B (u - x),
 * x += alpha Delta.  bu_dev (n complex), b2_dev (ndim^2 n complex), y_dev and
 * x_dev ((1 + ndim) n complex) are device
 * arrays of dtype; x_is_guess != 0 reads x as the starting point, else x
 * starts at 0.  Every check_every iterations (and at maxit) the FP64 relative
 * residual ||y - A x|| / ||y|| is computed; below tol the solve stops with
 * USP_OK.  ||Delta_i||^2 goes to hist_pre (up to hist_pre_cap values),
 * (iteration, rho) pairs to hist_true (up to hist_true_cap pairs).  Returns
 * USP_OK, USP_MAXIT, USP_DIVERGED (||Delta|| grew 3 times in a row above its
 * first value) or an error.  Workspace: 256-byte aligned, at least
 * usp_flux_workspace_bytes.  Synchronises `stream` before returning. */
int usp_flux_solve(const usp_flux_symbol* sym, int dtype, const void* bu_dev, const void* b2_dev, const void* y_dev,
                   void* x_dev, int x_is_guess, double alpha, double tol, int maxit, int check_every, void* ws_dev,
                   size_t ws_bytes, void* stream, int* iters_out, double* hist_pre, int hist_pre_cap,
                   double* hist_true, int hist_true_cap, int* n_true_out);

/* Device workspace of usp_flux_solve_refined. */
int usp_flux_refined_workspace_bytes(const usp_flux_symbol* sym, size_t* bytes);

/* Mixed-precision flux-form solve (the refinement of Sec. 2.1 applied to the
 * system of usp_flux_solve): bu_dev, b2_dev, y_dev, x_dev are complex128
 * device arrays laid out as for usp_flux_solve.  Each cycle computes the
 * FP64 residual r = y - A x (its relative norm is a hist_true entry; below
 * tol the solve stops with USP_OK), then runs up to refine_every complex64
 * iterations of Algorithm 1 on A d = r from d = 0 (on workspace copies of
 * B and r) and adds d to x in FP64.  The last cycle is cut to the number of
 * iterations that the rate of ||Delta|| over the last 10 iterations predicts
 * for reaching tol, when that is under half of refine_every.  x_is_guess:
 * 0 starts from x = 0; 1 reads x; 2 reads x and discards it (restart from 0)
 * if its residual is not below ||y||.  hist_pre gets the inner iterations'
 * ||Delta||^2.  Returns USP_OK, USP_MAXIT, USP_STAGNATED (no 1% residual
 * improvement over 8 cycles), USP_DIVERGED or an error.  Workspace: 256-byte
 * aligned, at least usp_flux_refined_workspace_bytes.  Synchronises `stream`
 * before returning. */
int usp_flux_solve_refined(const usp_flux_symbol* sym, const void* bu_dev, const void* b2_dev, const void* y_dev,
                           void* x_dev, int x_is_guess, double alpha, double tol, int maxit, int refine_every,
                           void* ws_dev, size_t ws_bytes, void* stream, int* iters_out, double* hist_pre,
                           int hist_pre_cap, double* hist_true, int hist_true_cap, int* n_true_out);

/* FP64 relative residual ||y - A x|| / ||y|| of the flux-form system. */
int usp_flux_residual(const usp_flux_symbol* sym, int dtype, const void* bu_dev, const void* b2_dev,
                      const void* y_dev, const void* x_dev, void* ws_dev, size_t ws_bytes, void* stream,
                      double* rel_out);

/* ---- Krylov drivers on the preconditioned system ---------------------------
 *
 * The comparison of Sec. 4 (Table 1b) runs Krylov methods on the same
 * preconditioned operator.  With the forward problem eliminated (Sec. 2.1)
 * and step size 1 the preconditioned system is P x = b with
 *     P v = B [v - (L + I)^-1 (B v)],     b = B (L + I)^-1 y,
 * so Algorithm 1 is x <- x + alpha (b - P x).  P v costs one pass sequence of
 * the iteration (the same FFT passes).  Methods:
 *   USP_KRYLOV_BICGSTAB  BiCGSTAB (van der Vorst 1992), shadow vector r_0;
 *                        true residual checked every check_every iterations.
 *   USP_KRYLOV_GMRES     GMRES(restart) (Saad and Schultz 1986): Arnoldi with
 *                        classical Gram-Schmidt applied twice, Givens
 *                        rotations; x updated and the true residual checked at
 *                        the end of each cycle; a cycle ends early when its
 *                        residual estimate, scaled by the ratio of true to
 *                        preconditioned residual at the last check, is below tol.
 * Stopping: ||y - A x||/||y|| < tol in FP64 (as usp_solve).  The handle must be
 * plain (not USP_FLAG_REFINE), 2-D or 3-D, without a gather; the vectors are
 * the handle's dtype, dot products and scalars are double. */
#define USP_KRYLOV_BICGSTAB 1
#define USP_KRYLOV_GMRES 2
#define USP_KRYLOV_CG 3       /* Hermitian handles (real symbol and B); P is then Hermitian (positive definite when A is) */

/* Workspace (device, 256-B aligned, caller-owned) of usp_solve_krylov for a
 * method (restart: GMRES cycle length in [1, 64]; ignored for BiCGSTAB):
 * BiCGSTAB 6 vectors, GMRES restart + 3 vectors, plus partial sums.
 * Errors: INVALID (refined handle, unknown method, restart), UNSUPPORTED_SHAPE
 * (1-D or gather). */
int usp_krylov_workspace_bytes(usp_op op, int method, int restart, size_t* bytes);

/* Test hook: w = P v (rhs 0) or w = b = B (L + I)^-1 v (rhs 1), one pass
 * sequence of the iteration (Sec. 2.1's eliminated form, step size 1).  Same
 * handle restrictions and workspace as usp_solve_krylov with
 * USP_KRYLOV_BICGSTAB (only its partial-sum area is used).  Synchronises. */
int usp_apply_precond(usp_op op, const void* v_dev, void* w_dev, int rhs, void* workspace_dev, size_t workspace_bytes);

/* Solve A x = y with a Krylov method on P x = b.  x_dev: initial guess when
 * x_is_guess, else started from 0; the solution on return.  iters_out:
 * operator applications counted as iterations (BiCGSTAB: iterations, each
 * applies P twice; GMRES: Arnoldi steps).  hist_est (may be NULL): GMRES:
 * squared residual estimate ||b - P x||^2 after each Arnoldi step; BiCGSTAB:
 * ||r||^2 of the recurrence at each check (index = iteration - 1).  hist_true
 * (may be NULL): (iteration, ||y - A x||/||y||) pairs per check; n_true_out:
 * number of checks.  Returns USP_OK, USP_MAXIT, USP_STAGNATED (no 1% progress
 * over 8 checks, or a BiCGSTAB breakdown), or a negative error.  Runs on the
 * handle's stream; synchronous with respect to the host outputs. */
int usp_solve_krylov(usp_op op, int method, int restart, const void* y_dev, void* x_dev, int x_is_guess, double tol,
                     int maxit, int check_every, void* workspace_dev, size_t workspace_bytes, int* iters_out,
                     double* hist_est, int hist_est_cap, double* hist_true, int hist_true_cap, int* n_true_out);

/* ---- eigenmodes (Sec. 4, Eq. schrodinger) -----------------------------------
 *
 * Lowest eigenpairs of a Hermitian canonical operator A (real symbol and real
 * B: e.g. H + Abar = -1/2 laplacian + V + Abar prepared with
 * usp_canonical_diffusion, D = 1/2, mu = V + Abar, omega = 0; then
 * E = c lam - Abar).  Shift-invert Lanczos: the Krylov space of A^-1, each
 * product A^-1 v by CG on the preconditioned system (to inner_tol relative
 * residual of A w = v, at most inner_maxit iterations), full
 * reorthogonalisation (classical Gram-Schmidt twice), thick restart keeping
 * nev + (ncv - nev)/2 Ritz vectors (the Hermitian counterpart of an
 * implicit restart).  A Ritz pair has converged when ||A u - lam u|| /
 * ||lam u|| (FP64 residual passes) is below tol. */
#define USP_EIGS_MAX_NEV 16
#define USP_EIGS_MAX_NCV 64

/* Workspace of usp_eigs: the CG vectors, ncv + 1 basis vectors, one work
 * vector and ncv restart vectors of the handle's dtype.  nev in [1, 16],
 * ncv in [nev + 2, 64]. */
int usp_eigs_workspace_bytes(usp_op op, int nev, int ncv, size_t* bytes);

/* v0_dev: start vector (N values, not all zero).  evecs_dev: nev vectors of
 * N values (contiguous), unit norm, for evals_out (host, ascending
 * eigenvalues of A); resid_out (host) their relative residuals.  Returns
 * USP_OK when all nev pairs converged within max_restarts restarts, else
 * USP_MAXIT (the best pairs are returned); USP_ERR_INVALID for a
 * non-Hermitian handle.  restarts_out: restarts used; inner_iters_out: CG
 * iterations summed over all inner solves (each one application of P). */
int usp_eigs(usp_op op, int nev, int ncv, const void* v0_dev, double tol, int max_restarts, double inner_tol,
             int inner_maxit, void* evecs_dev, double* evals_out, double* resid_out, void* ws_dev, size_t ws_bytes,
             int* restarts_out, int* inner_iters_out);

/* Host helper: eigenvalues (ascending, w_out[n]) and orthonormal eigenvectors
 * (columns of z_out, n x n complex row-major, 2 n^2 doubles) of the Hermitian
 * part of the n x n complex matrix a (row-major, 2 n^2 doubles), by cyclic
 * Jacobi rotations; n <= 256.  Used for the Rayleigh-Ritz step of usp_eigs. */
int usp_hermitian_eig(int n, const double* a, double* w_out, double* z_out);

/* ---- learned initial guess: 3-D convolutional network kernels ----------
 *
 * A learned x0 (a network mapping the refractive-index map to the field) is
 * an extension of the method: the fixed-point iteration (Algorithm 1)
 * starts from it and is the judge of its error, falling back to x0 = 0 when
 * ||y - A x0|| >= ||y||.  Activations are bf16 (16-bit words,
 * round-to-nearest-even) in 16-channel planes: a tensor with C channels (C
 * a multiple of 16; inputs padded) over V = D*H*W voxels (x fastest) holds
 * element (v, c) at ((c / 16) * V + v) * 16 + c % 16, so concatenation along
 * channels is placing planes one after the other.  Conv weights
 * [COUT][TAPS][CIN] bf16 with an fp32 master copy, repacked for the kernels
 * by usp_nn_pack_weights; biases fp32.  All calls run on `stream`
 * (asynchronous unless stated) and allocate nothing.
 */

/* Repack bf16 weights w [cout][taps][cin] (the forward layer's) into the
 * fragment order usp_nn_conv3d reads: transposed 0 for the forward
 * convolution (cin -> cout), 1 for the input gradient (cout -> cin).  27
 * taps are packed as 14 tap pairs (the 28th tap zero) for the 32-deep bf16
 * matrix-core product: the packed array has 28 * cin * cout bf16; 1 tap:
 * cin * cout.  cin, cout multiples of 16, taps 1 or 27, else USP_ERR_INVALID. */
int usp_nn_pack_weights(const void* w_dev, void* packed_dev, int cout, int taps, int cin, int transposed, void* stream);

/* 3x3x3 (taps 27, zero padding 1) or 1x1x1 (taps 1) convolution as an
 * implicit GEMM on the bf16 matrix cores with fp32 accumulation, from cin to
 * cout channels with weights packed by usp_nn_pack_weights:
 *   sign +1: out[v][co] = act(bias[co] + sum_{tap,ci} in[v + off(tap)][ci] w[co][tap][ci])
 *            (packing with transposed 0 of the layer's weights);
 *   sign -1: input gradient of a layer whose forward direction is cout -> cin,
 *            out[v][ci] = sum_{tap,co} g[v - off(tap)][co] w[co][tap][ci]
 *            (packing with transposed 1; no bias, no ReLU).
 * relu: apply max(0, .); bias may be NULL.  bf16 output: all cout channels
 * as planes (cstore must equal cout); out_f32: fp32 rows [V][cstore] of the
 * first cstore channels.  V must be a multiple of 16 and at most 2^30.
 * Schedule (results agree to rounding): grids of at least 2^18 voxels with
 * W % 64 == 0 and H % 4 == 0 (or W % 16 == 0 and H % 16 == 0) stage each
 * 16-channel input brick in LDS; other grids read operands from global memory.
 * Supported (cin, cout, taps): the network's layer shapes (16,16), (16,32),
 * (32,16), (32,32), (32,64), (64,32), (64,64), (64,128), (128,64), (192,64),
 * (64,192), (96,32), (32,96), (48,16), (16,48) with 27 taps and (16,16)
 * with 1 tap; others: USP_ERR_UNSUPPORTED_SHAPE. */
int usp_nn_conv3d(const void* in_dev, const void* wpacked_dev, const float* bias_dev, void* out_dev, int out_f32,
                  int cstore, int D, int H, int W, int cin, int cout, int taps, int sign, int relu, void* stream);

/* Weight (and bias) gradient of usp_nn_conv3d (sign +1):
 *   dw[co][tap][ci] = sum_v in[v + off(tap)][ci] g[v][co],  db[co] = sum_v g[v][co]
 * (fp32, deterministic: per-chunk partials in ws, added in a fixed order).
 * db may be NULL.  ws: usp_nn_wgrad_workspace bytes.  Schedule: 3x3x3
 * convolutions on grids with W % 32 == 0 copy in and g to voxel-blocked rows
 * in ws (in zero-padded in y and z) and sweep chunks of rows along y with all
 * 27 taps per wave (db from the same sweep); other shapes sum per row chunk
 * and tap group from the planes. */
int usp_nn_wgrad_workspace(int D, int H, int W, int cin, int cout, int taps, size_t* bytes);
int usp_nn_conv3d_wgrad(const void* in_dev, const void* g_dev, float* dw_dev, float* db_dev, void* ws_dev,
                        size_t ws_bytes, int D, int H, int W, int cin, int cout, int taps, void* stream);

/* 2x2x2 average pooling of a D x H x W grid (even sides; backward 0: in
 * fine, out coarse; backward 1: in = coarse gradient, out = fine gradient). */
int usp_nn_pool2(const void* in_dev, void* out_dev, int D, int H, int W, int C, int backward, void* stream);

/* Nearest upsampling by 2 to a D x H x W grid, written to channels
 * [c0, c0 + C) of an output with Ctot channels (backward 1: in = fine
 * gradient with Ctot channels, out = coarse gradient of those C channels).
 * c0 and C multiples of 16. */
int usp_nn_upsample2(const void* in_dev, void* out_dev, int D, int H, int W, int C, int Ctot, int c0, int backward,
                     void* stream);

/* dst[v][d0 + c] = src[v][s0 + c] for c < C (concatenation / split; whole
 * planes: s0, d0, C multiples of 16). */
int usp_nn_channel_copy(const void* src_dev, int Cs, int s0, void* dst_dev, int Cd, int d0, int C, long V, void* stream);

/* out = g * (y > 0) (y: post-ReLU activation); accumulate 1: out += that. */
int usp_nn_relu_backward(const void* y_dev, const void* g_dev, void* out_dev, long n, int accumulate, void* stream);

/* dst += src (bf16, n elements). */
int usp_nn_add(void* dst_dev, const void* src_dev, long n, void* stream);

/* Network input from the complex refractive index n + i kappa (complex64
 * [D][H][W]), one plane of 16 bf16 channels: 0 (Re n - n_bg)/n_span,
 * 1 kappa/kappa_max, 2 = 1 on the source plane z == plane, 3 and 4 the real
 * and imaginary parts of the source's Gaussian beam
 * exp(-((x - W/2)^2 + (y - H/2)^2)/w0^2) carried along z with
 * exp(i k0h S(z)), S(z) the trapezoidal sum of n + i kappa between the
 * source plane and z (k0h = wavenumber times grid step), 5..15 zero.
 * 0 <= plane < D, n_span, kappa_max, w0 > 0, else USP_ERR_INVALID. */
int usp_nn_features(const void* nidx_dev, void* out_dev, int D, int H, int W, double n_bg, double n_span,
                    double kappa_max, int plane, double k0h, double w0, void* stream);

/* Relative squared L2 loss ||scale p - x||^2 / ||x||^2 between the prediction
 * p (fp32 [V][2], Re/Im) and the target field x (complex64 [V]); grad (may be
 * NULL) receives its gradient with respect to p as bf16 [V][16] (channels
 * >= 2 zero).  ws: 32 KiB.  With loss_out the call synchronises and writes
 * the loss there; with loss_out NULL it does not synchronise and leaves the
 * loss (a double) at byte offset 16384 of ws, valid once the stream reaches it. */
int usp_nn_loss(const float* pred_dev, const void* target_dev, float scale, long V, void* grad_dev, void* ws_dev,
                double* loss_out, void* stream);

/* Adam step (Kingma & Ba) on n fp32 parameters with moments m, v; step >= 1;
 * wb (may be NULL) receives the bf16 copy. */
int usp_nn_adam(float* w_dev, const float* g_dev, float* m_dev, float* v_dev, void* wb_dev, long n, float lr, float b1,
                float b2, float eps, int step, void* stream);

/* fp32 -> bf16 (n elements). */
int usp_nn_to_bf16(const float* a_dev, void* b_dev, long n, void* stream);

/* x[v] = scale (p[v][0] + i p[v][1]) as complex128 (the initial guess). */
int usp_nn_pred_to_field(const float* pred_dev, float scale, void* x_dev, long V, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* USP_H */
