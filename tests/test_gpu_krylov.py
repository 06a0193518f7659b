"""GPU parity of the Krylov drivers (BiCGSTAB, GMRES(m) on the eliminated
preconditioned operator) against the FP64 oracle, through the C ABI.

Tolerances (relative L2): complex128 fixed-K iterates 1e-10 (same recurrences;
GMRES orthogonalises with classical Gram-Schmidt twice where the oracle uses
modified Gram-Schmidt, equal up to rounding); complex128 solutions 1e-9 against
the oracle's direct solution at tol 1e-11; complex64 fixed-K iterates 1e-4
(FP32 passes, Krylov recurrences amplify rounding more than the contraction)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from helpers import gpu_helmholtz, oracle_helmholtz, rel, to_np
from oracle import krylov as K
from oracle import richardson as R
from paper_2207_14222_amd import media

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _problems():
    return {
        "2d": media.helmholtz_disks(n=32, seed=4003, count=6, width=4, w0=4.0, row=4),
        "3d": media.helmholtz_spheres(shape=(16, 32, 8), count=6, width=3, w0=3.0, plane=2),
    }


@pytest.mark.parametrize("grid", ["2d", "3d"])
@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_bicgstab_iterates(grid, dt):
    _need_gpu()
    p = _problems()[grid]
    _announce(f"bicgstab iterates {grid} {dt}")
    cp, op_o = oracle_helmholtz(p)
    ref = K.bicgstab(op_o, cp.y, tol=0.0, maxit=8)
    can, op = gpu_helmholtz(p, dt)
    res = op.krylov(can.y, method="bicgstab", tol=0.0, maxit=8, check_every=8)
    assert res.iterations == 8
    assert rel(to_np(res.x), ref.x) < (1e-10 if dt == "c128" else 1e-4)
    assert abs(res.hist_true[-1, 1] - ref.hist_true[-1][1]) <= (1e-9 if dt == "c128" else 1e-4) * ref.hist_true[-1][1]


@pytest.mark.parametrize("grid", ["2d", "3d"])
@pytest.mark.parametrize("m,maxit", [(5, 12), (20, 20), (3, 3)])
def test_gmres_iterates_c128(grid, m, maxit):
    _need_gpu()
    p = _problems()[grid]
    _announce(f"gmres({m}) iterates {grid} maxit {maxit}")
    cp, op_o = oracle_helmholtz(p)
    ref = K.gmres(op_o, cp.y, m, tol=0.0, maxit=maxit)
    can, op = gpu_helmholtz(p, "c128")
    res = op.krylov(can.y, method="gmres", restart=m, tol=0.0, maxit=maxit)
    assert res.iterations == maxit
    assert rel(to_np(res.x), ref.x) < 1e-10
    # residual estimates after every Arnoldi step
    est = np.sqrt(res.hist_pre[:maxit])
    np.testing.assert_allclose(est, [e for _, e in ref.hist_est], rtol=1e-8)
    # one true-residual check per cycle
    assert len(res.hist_true) == len(ref.hist_true)


def test_gmres_c64_iterates():
    _need_gpu()
    p = _problems()["3d"]
    _announce("gmres(5) iterates 3d c64")
    cp, op_o = oracle_helmholtz(p)
    ref = K.gmres(op_o, cp.y, 5, tol=0.0, maxit=10)
    can, op = gpu_helmholtz(p, "c64")
    res = op.krylov(can.y, method="gmres", restart=5, tol=0.0, maxit=10)
    assert rel(to_np(res.x), ref.x) < 1e-4


@pytest.mark.parametrize("method,m", [("bicgstab", 0), ("gmres", 5), ("gmres", 20)])
def test_krylov_solution_c128(method, m):
    _need_gpu()
    p = _problems()["3d"]
    _announce(f"{method}({m}) solve 3d c128")
    cp, op_o = oracle_helmholtz(p)
    xs = R.solve(op_o, cp.y, 0.9, 1e-13, 20000, 50).x   # fixed point to the rounding floor
    can, op = gpu_helmholtz(p, "c128")
    res = op.krylov(can.y, method=method, restart=max(m, 1), tol=1e-11, maxit=3000, check_every=5)
    assert res.converged, res.status_name
    assert rel(to_np(res.x), xs) < 1e-9
    # the oracle's driver needs about as many steps
    ref = K.bicgstab(op_o, cp.y, 1e-11, 3000, 5) if method == "bicgstab" else K.gmres(op_o, cp.y, m, 1e-11, 3000)
    assert ref.converged
    slack = 5 if method == "bicgstab" else m
    assert abs(res.iterations - ref.iterations) <= slack
    # and fewer operator applications than the fixed point at alpha = 0.8
    fp = op.solve(can.y, alpha=0.8, tol=1e-11, maxit=20000, check_every=5)
    applies = 2 * res.iterations if method == "bicgstab" else res.iterations
    assert applies < fp.iterations


def test_krylov_initial_guess_and_rejections():
    _need_gpu()
    from paper_2207_14222_amd import _lib as L, solver
    p = _problems()["2d"]
    _announce("krylov guess / rejections 2d")
    can, op = gpu_helmholtz(p, "c128")
    r0 = op.krylov(can.y, method="bicgstab", tol=1e-10, maxit=2000, check_every=1)
    assert r0.converged
    # starting from the solution: converged at the first check
    r1 = op.krylov(can.y, x=r0.x.clone(), method="gmres", restart=10, tol=1e-9, maxit=100)
    assert r1.converged and r1.iterations <= 1
    r2 = op.krylov(can.y, x=r0.x.clone(), method="bicgstab", tol=1e-9, maxit=100, check_every=1)
    assert r2.converged and r2.iterations <= 1
    with pytest.raises(L.UspError):
        op.krylov(can.y, method="gmres", restart=0)
    with pytest.raises(L.UspError):
        op.krylov(can.y, method="gmres", restart=65)
    canr = solver.canonical_helmholtz(p.k2, p.source, p.spacing, dtype=torch.complex128)
    opr = solver.Operator(canr.symbol, canr.B, refine=True)
    with pytest.raises(L.UspError):
        opr.krylov(canr.y, method="bicgstab")
    # workspace too small
    import ctypes as ct
    nb = ct.c_size_t()
    assert L.lib().usp_krylov_workspace_bytes(op.handle, L.USP_KRYLOV_BICGSTAB, 0, ct.byref(nb)) == 0
    ws = torch.empty(nb.value - 4096, dtype=torch.uint8, device="cuda")
    it = ct.c_int()
    x = torch.empty_like(can.y)
    rc = L.lib().usp_solve_krylov(op.handle, L.USP_KRYLOV_BICGSTAB, 0, ct.c_void_p(can.y.data_ptr()),
                                  ct.c_void_p(x.data_ptr()), 0, 1e-6, 10, 1, ct.c_void_p(ws.data_ptr()),
                                  ws.numel(), ct.byref(it), None, 0, None, 0, None)
    assert rc == L.USP_ERR_WORKSPACE


@pytest.mark.parametrize("grid", ["2d", "3d"])
def test_apply_precond_matches_oracle(grid):
    _need_gpu()
    p = _problems()[grid]
    _announce(f"apply_precond {grid} c128")
    cp, op_o = oracle_helmholtz(p)
    can, op = gpu_helmholtz(p, "c128")
    rng = np.random.default_rng(3)
    v = rng.standard_normal(op_o.shape) + 1j * rng.standard_normal(op_o.shape)
    w = op.apply_precond(torch.from_numpy(v).cuda())
    assert rel(to_np(w), K.precond_apply(op_o, v)) < 1e-13
    b = op.apply_precond(can.y, rhs=True)
    assert rel(to_np(b), K.precond_rhs(op_o, cp.y)) < 1e-13
