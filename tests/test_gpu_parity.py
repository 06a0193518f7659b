"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (relative L2):
* complex128: 1e-10 (solutions) / 1e-11 (fixed-K iterates, same arithmetic up to
  rounding order);
* complex64 fixed-K iterates: 3e-5 -- FP32 rounding (unit 6e-8) of each pass,
  amplified by log2(N)-deep FFTs and carried through a contraction;
* complex64 + FP64 refinement, solution: 1e-6.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import gpu_helmholtz, oracle_helmholtz, rel, to_np
from oracle import canon, operators, richardson as R
from paper_2207_14222_amd import media

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


# ---------------------------------------------------------------- canonical form
def test_canonical_fields_match_oracle():
    _need_gpu()
    p = media.helmholtz_spheres(shape=(16, 32, 8), count=6, width=3, w0=3.0, plane=2)
    _announce("canonical fields 16x32x8 c128")
    cp, _ = oracle_helmholtz(p)
    can, op = gpu_helmholtz(p, "c128")
    assert rel(to_np(can.B), cp.B) < 1e-14
    assert rel(to_np(can.y), cp.y) < 1e-14
    assert abs(can.c - cp.c) < 1e-12 * abs(cp.c)


# ---------------------------------------------------------------- 1-D single workgroup
def test_1d_config1_c128_solution():
    """1-D random medium N = 256, complex128, tol 1e-10, check every iteration:
    the GPU's iterate equals the oracle's after the same number of iterations
    (1e-10), and both solved until the residual is below 1e-13 match the dense
    LU solution to 1e-10."""
    _need_gpu()
    p = media.helmholtz_1d()
    _announce("1d N=256 c128 solve")
    cp, op_o = oracle_helmholtz(p)
    ref = R.solve(op_o, cp.y, 0.8, 1e-10, 5000, 1)
    can, op = gpu_helmholtz(p, "c128")
    res = op.solve(can.y, alpha=0.8, tol=1e-10, maxit=5000, check_every=1)
    assert res.converged
    assert abs(res.iterations - ref.iterations) <= 1
    x = to_np(res.x)
    xk, _ = R.iterate(op_o, cp.y, 0.8, res.iterations)
    assert rel(x, xk) < 1e-10
    # residual history matches the oracle's
    k = min(len(ref.hist_true), len(res.hist_true)) - 1
    np.testing.assert_allclose(res.hist_true[:k, 1], [h[1] for h in ref.hist_true[:k]], rtol=1e-6, atol=1e-14)
    np.testing.assert_allclose(np.sqrt(res.hist_pre[:k]), ref.hist_pre[:k], rtol=1e-9, atol=1e-14)
    # to stagnation: both against dense LU
    xs = R.solve_direct(op_o, cp.y)
    ref13 = R.solve(op_o, cp.y, 0.8, 1e-13, 5000, 1)
    assert ref13.converged and rel(ref13.x, xs) < 1e-10
    res13 = op.solve(can.y, alpha=0.8, tol=1e-13, maxit=5000, check_every=1)
    assert res13.converged
    assert rel(to_np(res13.x), xs) < 1e-10
    assert rel(to_np(res13.x), ref13.x) < 1e-10


@pytest.mark.parametrize("n", [8, 64, 1024])
@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_1d_iterates(n, dt):
    _need_gpu()
    p = media.helmholtz_1d(n=n, width=max(n // 8, 1), sigma=2.0)
    _announce(f"1d iterate N={n} {dt}")
    cp, op_o = oracle_helmholtz(p)
    K = 25
    xo, ho = R.iterate(op_o, cp.y, 0.9, K)
    can, op = gpu_helmholtz(p, dt)
    x, h = op.iterate(can.y, alpha=0.9, K=K)
    tol = 1e-11 if dt == "c128" else 3e-5
    assert rel(to_np(x), xo) < tol
    np.testing.assert_allclose(np.sqrt(h), ho, rtol=tol * 10)


# ---------------------------------------------------------------- multi-pass 2-D / 3-D
# every axis position with lengths 8 to 1024; the 256-long axes run the
# complex128 pass instantiations of the benchmark's FP64 residual and of its
# plain complex128 solve
SHAPES = [(16, 16), (8, 1024), (1024, 8), (32, 64), (256, 16), (8, 8, 8), (16, 32, 64), (64, 8, 16), (8, 16, 512),
          (128, 8, 8), (256, 8, 8), (8, 256, 8), (8, 8, 256)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_multipass_iterates_c128(shape):
    _need_gpu()
    cnt = 4
    p = media.helmholtz_spheres(shape=shape, count=cnt, width=2, w0=2.0, plane=1, seed=7)
    _announce(f"iterate c128 {shape}")
    cp, op_o = oracle_helmholtz(p)
    K = 12
    xo, ho = R.iterate(op_o, cp.y, 0.8, K)
    can, op = gpu_helmholtz(p, "c128")
    x, h = op.iterate(can.y, alpha=0.8, K=K)
    assert rel(to_np(x), xo) < 1e-11
    np.testing.assert_allclose(np.sqrt(h), ho, rtol=1e-10)
    rho, _, _ = op.residual(can.y, x)
    assert abs(rho - R.relative_residual(op_o, xo, cp.y)) < 1e-10 * rho


@pytest.mark.parametrize("shape", [(32, 32), (16, 32, 64), (8, 16, 512)], ids=lambda s: "x".join(map(str, s)))
def test_multipass_iterates_c64(shape):
    _need_gpu()
    p = media.helmholtz_spheres(shape=shape, count=4, width=2, w0=2.0, plane=1, seed=8)
    _announce(f"iterate c64 {shape}")
    cp, op_o = oracle_helmholtz(p)
    K = 12
    xo, ho = R.iterate(op_o, cp.y, 0.8, K)
    can, op = gpu_helmholtz(p, "c64")
    x, h = op.iterate(can.y, alpha=0.8, K=K)
    assert rel(to_np(x), xo) < 3e-5
    np.testing.assert_allclose(np.sqrt(h), ho, rtol=3e-4)


def test_iterate_from_guess_continues_exactly():
    """Resuming from a saved x equals running straight through (memoryless iteration)."""
    _need_gpu()
    p = media.helmholtz_spheres(shape=(16, 16, 32), count=3, width=2, w0=2.0, plane=1, seed=9)
    _announce("resume c128 16x16x32")
    can, op = gpu_helmholtz(p, "c128")
    x20, _ = op.iterate(can.y, alpha=0.8, K=20)
    x10, _ = op.iterate(can.y, alpha=0.8, K=10)
    x10b, _ = op.iterate(can.y, x=x10.clone(), alpha=0.8, K=10)
    assert rel(to_np(x10b), to_np(x20)) < 1e-13


def test_solve_3d_c128_matches_oracle_solution():
    _need_gpu()
    p = media.helmholtz_spheres(shape=(32, 32, 32), count=6, width=4, w0=4.0, plane=4, seed=3)
    _announce("solve c128 32^3")
    cp, op_o = oracle_helmholtz(p)
    ref = R.solve(op_o, cp.y, 0.8, 1e-12, 5000, 10)
    can, op = gpu_helmholtz(p, "c128")
    res = op.solve(can.y, alpha=0.8, tol=1e-12, maxit=5000, check_every=10)
    assert res.converged and res.iterations == ref.iterations
    assert rel(to_np(res.x), ref.x) < 1e-10


def test_refined_c64_matches_oracle_solution():
    _need_gpu()
    p = media.helmholtz_spheres(shape=(32, 32, 32), count=6, width=4, w0=4.0, plane=4, seed=3)
    _announce("refined solve 32^3")
    cp, op_o = oracle_helmholtz(p)
    ref = R.solve(op_o, cp.y, 0.8, 1e-12, 5000, 10)
    can, op = gpu_helmholtz(p, "c128", refine=True)
    res = op.solve(can.y, alpha=0.8, tol=1e-10, maxit=5000, check_every=20)
    assert res.converged
    assert rel(to_np(res.x), ref.x) < 1e-6
    # iteration count close to the plain FP64 iteration's (memoryless, Sec. 2.1)
    ref10 = R.solve(op_o, cp.y, 0.8, 1e-10, 5000, 20)
    assert abs(res.iterations - ref10.iterations) <= 40


def test_plain_c64_solve_reaches_its_floor():
    """Plain complex64 reaches 1e-5 and then stalls near the FP32 floor (reported as stagnated)."""
    _need_gpu()
    p = media.helmholtz_spheres(shape=(32, 32, 32), count=6, width=4, w0=4.0, plane=4, seed=3)
    _announce("plain c64 solve 32^3")
    cp, op_o = oracle_helmholtz(p)
    can, op = gpu_helmholtz(p, "c64")
    res = op.solve(can.y, alpha=0.8, tol=1e-5, maxit=3000, check_every=10)
    assert res.converged
    ref = R.solve(op_o, cp.y, 0.8, 1e-12, 5000, 10)
    assert rel(to_np(res.x), ref.x) < 1e-4


def test_diffusion_iterates_and_solution():
    _need_gpu()
    d = media.diffusion_blobs(shape=(16, 32, 32), sigma=2.0, seed=3)
    _announce("diffusion 16x32x32")
    cp = canon.canonical_diffusion(d.mu_a, d.D, d.omega_over_v, d.source, d.spacing)
    op_o = operators.Operator(cp)
    from paper_2207_14222_amd import solver
    can = solver.canonical_diffusion(d.mu_a, d.D, d.omega_over_v, d.source, d.spacing, dtype=torch.complex128)
    assert rel(to_np(can.B), cp.B) < 1e-14 and rel(to_np(can.y), cp.y) < 1e-14
    op = solver.Operator(can.symbol, can.B)
    xo, _ = R.iterate(op_o, cp.y, 1.0, 10)
    x, _ = op.iterate(can.y, alpha=1.0, K=10)
    assert rel(to_np(x), xo) < 1e-11
    ref = R.solve(op_o, cp.y, 1.0, 1e-11, 2000, 5)
    res = op.solve(can.y, alpha=1.0, tol=1e-11, maxit=2000, check_every=5)
    assert res.converged and rel(to_np(res.x), ref.x) < 1e-10


def test_not_contractive_is_rejected():
    _need_gpu()
    from paper_2207_14222_amd import _lib, solver
    p = media.helmholtz_spheres(shape=(8, 8, 8), count=2, width=1, w0=1.0, plane=1)
    can = solver.canonical_helmholtz(p.k2, p.source, p.spacing, dtype=torch.complex128)
    B = can.B.clone()
    B[0, 0, 0] = -0.5 + 0j   # |v| = 1.5
    with pytest.raises(_lib.UspError) as ei:
        solver.Operator(can.symbol, B)
    assert ei.value.code == _lib.USP_ERR_NOT_CONTRACTIVE


def test_nan_is_reported():
    _need_gpu()
    from paper_2207_14222_amd import _lib
    p = media.helmholtz_spheres(shape=(8, 16, 8), count=2, width=1, w0=1.0, plane=1)
    can, op = gpu_helmholtz(p, "c64")
    y = can.y.clone()
    y[1, 1, 1] = complex(float("nan"), 0.0)
    with pytest.raises(_lib.UspError) as ei:
        op.solve(y, alpha=0.8, tol=1e-6, maxit=50, check_every=5)
    assert ei.value.code == _lib.USP_ERR_NAN


def test_launch_plans_are_bit_identical_and_autotune_picks_one():
    """Every autotuner candidate computes the same bits; the tuner keeps a valid plan."""
    _need_gpu()
    p = media.helmholtz_spheres(shape=(64, 32, 64), count=5, width=3, w0=3.0, plane=2, seed=12)
    _announce("plans c64 64x32x64")
    can, op = gpu_helmholtz(p, "c64")
    ref = None
    for pf in (0, 1, 2, 3):
        for wm in (8, 16, 32):
            for ws in (8, 16, 32):
                op.set_plan(pf & 1, wm, ws, pf >> 1)
                x, h = op.iterate(can.y, alpha=0.8, K=6)
                xn = x.cpu()
                if ref is None:
                    ref = (xn, h)
                else:
                    assert torch.equal(xn, ref[0]), (pf, wm, ws)
                    assert np.array_equal(h, ref[1])
    xt = torch.zeros_like(can.y)
    best = op.autotune(can.y, xt, alpha=0.8, reps=3)
    assert best["w_sym"] in (8, 16, 32) and best["x_prefetch"] in (0, 1) and best["r_load"] in (0, 1, 2, 3)
    x, _ = op.iterate(can.y, alpha=0.8, K=6)
    assert torch.equal(x.cpu(), ref[0])


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_residual_load_plans_are_bit_identical(dt):
    """Every load plan of the FP64 residual's last pass gives the same bits, and the
    residual equals the oracle's."""
    _need_gpu()
    p = media.helmholtz_spheres(shape=(32, 16, 256), count=5, width=3, w0=3.0, plane=2, seed=13)
    _announce(f"residual load plans {dt} 32x16x256")
    cp, op_o = oracle_helmholtz(p)
    can, op = gpu_helmholtz(p, dt)
    x, _ = op.iterate(can.y, alpha=0.8, K=7)
    rhos = []
    for rl in range(4):
        op.set_plan(1, 0, 0, 1, rl)
        rhos.append(op.residual(can.y, x))
    assert all(r == rhos[0] for r in rhos), rhos
    # complex64 handles hold B and y rounded to FP32: the oracle's residual of
    # the same x then differs at the level of that rounding
    rho_o = R.relative_residual(op_o, to_np(x), cp.y)
    assert abs(rhos[0][0] - rho_o) < (1e-10 if dt == "c128" else 1e-5) * rho_o


@pytest.mark.parametrize("bval", [5.0, -5.0])
def test_pantograph_solution_and_iterates(bval):
    """Pantograph (lambda = 0.5, N = 1024, complex128) with the non-diagonal gather in V."""
    _need_gpu()
    from paper_2207_14222_amd import solver
    pp = media.pantograph(n=1024, b_value=bval)
    _announce(f"pantograph b={bval}")
    cp = canon.canonical_pantograph(pp.a, pp.b, pp.lam, pp.t0, pp.h, pp.x0_at_lam_t, pp.x0_t0)
    op_o = operators.Operator(cp)
    can = solver.canonical_pantograph(pp.a, pp.b, pp.lam, pp.t0, pp.h, pp.x0_at_lam_t, pp.x0_t0)
    op = solver.Operator(can.symbol, can.B, gather=can.gather)
    xo, ho = R.iterate(op_o, cp.y, 0.9, 15)
    x, h = op.iterate(can.y, alpha=0.9, K=15)
    assert rel(to_np(x), xo) < 1e-10
    ref = R.solve(op_o, cp.y, 0.9, 1e-10, 5000, 1)
    res = op.solve(can.y, alpha=0.9, tol=1e-10, maxit=5000, check_every=1)
    assert res.converged and abs(res.iterations - ref.iterations) <= 1
    # the same number of iterations: equal iterates
    xk, _ = R.iterate(op_o, cp.y, 0.9, res.iterations)
    assert rel(to_np(res.x), xk) < 1e-10
    # both until the residual is below 1e-13: the dense LU solution
    xs = np.linalg.solve(op_o.dense_A(), cp.y)
    ref13 = R.solve(op_o, cp.y, 0.9, 1e-13, 5000, 1)
    assert ref13.converged and rel(ref13.x, xs) < 1e-10
    res13 = op.solve(can.y, alpha=0.9, tol=1e-13, maxit=5000, check_every=1)
    assert res13.converged
    assert rel(to_np(res13.x), xs) < 1e-10
    assert rel(to_np(res13.x), ref13.x) < 1e-10


def test_stream_copy_is_exact_and_validates():
    """The measurement copy kernel copies every byte (ragged tail of the grid-stride
    loop included) and rejects misaligned or overlapping buffers."""
    _need_gpu()
    from paper_2207_14222_amd import _lib, solver
    _announce("stream copy")
    for n in (1, 7, 4099, (1 << 20) + 3):
        a = torch.randn(n, dtype=torch.complex128, device="cuda")
        b = torch.zeros_like(a)
        solver.stream_copy(a, b)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    a = torch.randn(64, dtype=torch.complex128, device="cuda")
    with pytest.raises(_lib.UspError):
        solver.stream_copy(a[0:32], a[16:48])   # overlapping
    f = torch.zeros(9, dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.UspError):
        solver.stream_copy(f[1:5], torch.zeros(4, dtype=torch.float32, device="cuda"))      # not 16-byte aligned
