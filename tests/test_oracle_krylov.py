"""Pins for the Krylov drivers of the oracle (CPU):
* the preconditioned operator P and right-hand side b against Algorithm 1
  (one step is x + alpha (b - P x)) and against dense matrices;
* GMRES without restart terminates, on a constant-V grid (P diagonal in
  Fourier space), after exactly as many iterations as P has distinct
  eigenvalues, and not one earlier;
* GMRES's minimal-residual property: within a cycle its preconditioned
  residual is never above that of the fixed-point iteration with the same
  number of operator applications, and never increases;
* BiCGSTAB's defining orthogonalities (<r^, s> = 0 by the choice of alpha,
  <t, r_new> = 0 by the choice of omega);
* BiCGSTAB and restarted GMRES reach the dense LU solution."""
import numpy as np
import pytest

from oracle import canon, krylov, operators, richardson
from paper_2207_14222_amd import media


def _disks(n=16, seed=4001):
    p = media.helmholtz_disks(n=n, seed=seed, count=3, width=3, w0=3.0, row=3)
    cp = canon.canonical_helmholtz(p.k2, p.source, p.spacing)
    return cp, operators.Operator(cp)


def test_precond_operator_matches_algorithm_1_and_dense():
    cp, op = _disks()
    rng = np.random.default_rng(0)
    x = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    b = krylov.precond_rhs(op, cp.y)
    xn, _ = richardson.step(op, x, cp.y, 0.7)
    assert np.allclose(xn, x + 0.7 * (b - krylov.precond_apply(op, x)), atol=1e-13, rtol=0)
    # dense: P = B (I - (L + I)^-1 B) and P = B (L + I)^-1 A (the eliminated and the plain forms)
    N = x.size
    Bd = op.dense_B()
    LIinv = np.linalg.inv(op.dense_L() + np.eye(N))
    Pd = op._dense(lambda v: krylov.precond_apply(op, v))
    assert np.allclose(Pd, Bd @ (np.eye(N) - LIinv @ Bd), atol=1e-12)
    assert np.allclose(Pd, Bd @ LIinv @ op.dense_A(), atol=1e-12)


def _homogeneous(shape=(8, 8), n=1.2 + 0.05j):
    p = media.helmholtz_homogeneous(shape, nidx=n)
    # a given bias away from k^2 so that V = v0 != 0 is constant
    kbar = p.k2.flat[0] - 2.0
    cp = canon.canonical_helmholtz(p.k2, p.source, p.spacing, given=(kbar, 3.0j))
    return cp, operators.Operator(cp)


def test_gmres_terminates_at_the_number_of_distinct_eigenvalues():
    """A right-hand side made of plane waves on q distinct |p|^2 shells lies in a
    q-dimensional invariant space of P: GMRES is exact after q steps, not before."""
    cp, op = _homogeneous()
    b0 = 1.0 - op.v.flat[0]
    lam = b0 * (1.0 - b0 / (op.l + 1.0))       # P = F^-1 diag(lam) F on this grid
    modes = [(0, 0), (1, 0), (1, 2), (3, 2), (0, 4)]   # |k|^2 = 0, 1, 5, 13, 16
    assert len({round(float(abs(lam[m])), 12) for m in modes}) == len(modes)
    rng = np.random.default_rng(1)
    yhat = np.zeros(op.shape, dtype=complex)
    for m in modes:
        yhat[m] = rng.standard_normal() + 1j * rng.standard_normal()
    y = np.fft.ifftn(yhat)
    b = krylov.precond_rhs(op, y)
    q = len(modes)
    res_q = krylov.gmres(op, y, m=32, tol=0.0, maxit=q)
    res_q1 = krylov.gmres(op, y, m=32, tol=0.0, maxit=q - 1)
    rq = np.linalg.norm(b - krylov.precond_apply(op, res_q.x)) / np.linalg.norm(b)
    rq1 = np.linalg.norm(b - krylov.precond_apply(op, res_q1.x)) / np.linalg.norm(b)
    assert rq < 1e-12
    assert rq1 > 1e-6


def test_gmres_minimal_residual_against_fixed_point():
    cp, op = _disks()
    b = krylov.precond_rhs(op, cp.y)
    prev = np.inf
    for j in range(1, 13):
        g = krylov.gmres(op, cp.y, m=20, tol=0.0, maxit=j)
        rg = np.linalg.norm(b - krylov.precond_apply(op, g.x))
        assert abs(g.hist_est[-1][1] - rg) <= 1e-9 * np.linalg.norm(b)   # Givens estimate = true value
        assert rg <= prev * (1 + 1e-12)
        prev = rg
        for alpha in (0.6, 0.8, 1.0):
            xf, _ = richardson.iterate(op, cp.y, alpha, j)
            assert rg <= np.linalg.norm(b - krylov.precond_apply(op, xf)) * (1 + 1e-10)


def test_bicgstab_orthogonalities():
    cp, op = _disks()
    b = krylov.precond_rhs(op, cp.y)
    r = b.copy()
    rhat = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(r)
    p = np.zeros_like(r)
    x = np.zeros_like(r)
    for _ in range(6):
        rho_new = np.vdot(rhat, r)
        p = r + (rho_new / rho) * (alpha / omega) * (p - omega * v)
        v = krylov.precond_apply(op, p)
        alpha = rho_new / np.vdot(rhat, v)
        s = r - alpha * v
        assert abs(np.vdot(rhat, s)) <= 1e-12 * np.linalg.norm(rhat) * np.linalg.norm(s) + 1e-14
        t = krylov.precond_apply(op, s)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        assert abs(np.vdot(t, r)) <= 1e-12 * np.linalg.norm(t) * np.linalg.norm(r) + 1e-14
        rho = rho_new
    # the library-style driver produces the same iterate
    res = krylov.bicgstab(op, cp.y, tol=0.0, maxit=6)
    assert np.allclose(res.x, x, atol=1e-13 * np.linalg.norm(x))
    # and r is the true preconditioned residual of x
    assert np.allclose(r, b - krylov.precond_apply(op, x), atol=1e-11 * np.linalg.norm(b))


@pytest.mark.parametrize("method", ["bicgstab", "gmres5", "gmres20"])
def test_krylov_reaches_lu_solution(method):
    cp, op = _disks()
    xs = np.linalg.solve(op.dense_A(), cp.y.ravel()).reshape(op.shape)
    if method == "bicgstab":
        res = krylov.bicgstab(op, cp.y, 1e-12, 500, 1)
    else:
        res = krylov.gmres(op, cp.y, int(method[5:]), 1e-12, 2000)
    assert res.converged
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) < 1e-10
    # fewer iterations than the fixed point at alpha = 0.8 on this problem
    fp = richardson.solve(op, cp.y, 0.8, 1e-12, 5000, 1)
    assert res.iterations < fp.iterations
