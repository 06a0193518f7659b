"""Pins for the oracle's operators and Algorithm 1 (paper Sec. 2.1, Eq. laplacian_inverse)."""
import math

import numpy as np
import pytest

from oracle import canon, operators, richardson as R, theory
from paper_2207_14222_amd import media

K0 = media.K0


def naive_dft(x):
    n = x.shape[0]
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n) @ x


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32, 64])
def test_fft_matches_naive_dft(n):
    rng = np.random.default_rng(n)
    x = rng.normal(size=n) + 1j * rng.normal(size=n)
    assert np.allclose(np.fft.fft(x), naive_dft(x), rtol=0, atol=1e-12 * n)
    assert np.allclose(np.fft.ifft(naive_dft(x)), x, atol=1e-13 * n)


@pytest.mark.parametrize("shape", [(8,), (4, 8), (2, 4, 8), (8, 4, 2)])
def test_oracle_fftn_matches_naive_dft(shape):
    """The oracle's multi-dimensional transform (library FFT, threaded) against a
    naive DFT matrix applied along every axis, forward and inverse."""
    rng = np.random.default_rng(len(shape))
    x = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    ref = x
    for ax in range(len(shape)):
        n = shape[ax]
        j = np.arange(n)
        W = np.exp(-2j * np.pi * np.outer(j, j) / n)
        ref = np.moveaxis(np.tensordot(W, np.moveaxis(ref, ax, 0), axes=(1, 0)), 0, ax)
    N = x.size
    assert np.allclose(operators.fftn(x), ref, rtol=0, atol=1e-12 * N)
    assert np.allclose(operators.ifftn(ref), x, rtol=0, atol=1e-13 * N)


def test_wavenumbers():
    for n, h in ((8, 0.25), (7, 0.5), (16, 1.0)):
        p = operators.wavenumbers(n, h)
        expect = [2 * math.pi * (k if k < (n + 1) // 2 else k - n) / (n * h) for k in range(n)]
        assert np.allclose(p, expect, atol=1e-14)


def _helm_homog(shape, nidx, kbar2, c, h=0.25):
    k2 = np.full(shape, (K0 * nidx) ** 2)
    return canon.canonical_helmholtz(k2, np.zeros(shape), (h,) * len(shape), given=(kbar2, c))


@pytest.mark.parametrize("shape", [(16,), (8, 8), (4, 8, 4)])
def test_LI_inverse_on_plane_waves(shape):
    """(L + I)^-1 e^{i p.r} = c / (-|p|^2 + kbar^2 + c) e^{i p.r}  (Eq. laplacian_inverse)."""
    h = 0.25
    kbar2, c = 40.0 + 3.0j, 11.0j
    cp = _helm_homog(shape, 1.1, kbar2, c, h)
    op = operators.Operator(cp)
    rng = np.random.default_rng(0)
    grids = np.meshgrid(*[np.arange(n) * h for n in shape], indexing="ij")
    for _ in range(5):
        m = [int(rng.integers(0, n)) for n in shape]
        p = [2 * math.pi * (mi if mi < n / 2 else mi - n) / (n * h) for mi, n in zip(m, shape)]
        w = np.exp(1j * sum(pi * g for pi, g in zip(p, grids)))
        p2 = sum(pi * pi for pi in p)
        assert np.allclose(op.apply_LI_inv(w), c / (-p2 + kbar2 + c) * w, atol=1e-12)
        assert np.allclose(op.apply_L(w), (-p2 + kbar2) / c * w, atol=1e-11)


@pytest.mark.parametrize("dtype_K", [(1.0, 30), (0.8, 50), (0.5, 7)])
def test_constant_V_closed_form(dtype_K):
    """Constant v = v0: every Fourier mode evolves independently with
    x_K(p) = (1 - m^K) y(p)/(l + v0),  m = 1 - alpha b0 (l + v0)/(l + 1),
    derived from the two lines of Algorithm 1 with B = b0 = 1 - v0."""
    alpha, K = dtype_K
    shape = (8, 6, 4)
    nidx = 1.2 + 0.1j
    k2 = (K0 * nidx) ** 2
    kbar2 = k2.real - 5.0
    c = 1j * abs(k2 - kbar2) / 0.9
    cp = _helm_homog(shape, nidx, kbar2, c)
    rng = np.random.default_rng(1)
    y = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    op = operators.Operator(cp)
    xK, _ = R.iterate(op, y, alpha, K)
    v0 = (k2 - kbar2) / c
    b0 = 1 - v0
    grids = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(n, 0.25) for n in shape], indexing="ij")
    p2 = sum(g ** 2 for g in grids)
    l = (-p2 + kbar2) / c
    m = 1 - alpha * b0 * (l + v0) / (l + 1)
    expect = np.fft.ifftn((1 - m ** K) * np.fft.fftn(y) / (l + v0))
    assert np.linalg.norm(xK - expect) <= 1e-12 * np.linalg.norm(expect)


def test_config1_solution_matches_dense_lu():
    """1-D random medium, N = 256: Algorithm 1 to ||r||/||y|| < 1e-12 equals numpy.linalg.solve."""
    p = media.helmholtz_1d()
    cp = canon.canonical_helmholtz(p.k2, p.source, p.spacing)
    op = operators.Operator(cp)
    res = R.solve(op, cp.y, 0.8, 1e-12, 20000, 1)
    assert res.converged
    A = op.dense_A()
    xs = np.linalg.solve(A, cp.y)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(res.x - xs) <= 1e-12 * kappa * np.linalg.norm(xs)


@pytest.mark.parametrize("shape", [(16, 16), (8, 8, 8)])
def test_small_grid_solution_matches_dense_lu(shape):
    pr = media.helmholtz_spheres(shape=shape, count=3, width=2, w0=2.0, plane=1, seed=5)
    cp = canon.canonical_helmholtz(pr.k2, pr.source, pr.spacing)
    op = operators.Operator(cp)
    res = R.solve(op, cp.y, 0.8, 1e-13, 20000, 5)
    xs = R.solve_direct(op, cp.y)
    assert np.linalg.norm(res.x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_monotone_update_norm_and_error():
    """||Delta_i|| and ||x_i - x*|| decrease monotonically (||M|| < 1, appendix)."""
    p = media.helmholtz_1d(n=128, width=16)
    cp = canon.canonical_helmholtz(p.k2, p.source, p.spacing)
    op = operators.Operator(cp)
    xs = R.solve_direct(op, cp.y)
    x = np.zeros_like(xs)
    errs, dn = [], []
    for _ in range(300):
        x, d = R.step(op, x, cp.y, 0.8)
        dn.append(np.linalg.norm(d))
        errs.append(np.linalg.norm(x - xs))
    dn, errs = np.array(dn), np.array(errs)
    live = dn > 1e-13 * dn[0]
    assert np.all(np.diff(dn[live]) < 0)
    live = errs > 1e-12 * errs[0]
    assert np.all(np.diff(errs[live]) < 0)


def test_refined_equals_plain_iterates():
    """Richardson keeps a single vector (Sec. 2.1), so restarting on A d = y - A x from d = 0
    every k steps reproduces the plain iterates."""
    p = media.helmholtz_1d(n=128, width=16)
    cp = canon.canonical_helmholtz(p.k2, p.source, p.spacing)
    op = operators.Operator(cp)
    xp, _ = R.iterate(op, cp.y, 0.8, 60)
    rr = R.solve_refined(op, cp.y, 0.8, 1e-300, 60, inner=20)
    assert rr.iterations == 60
    assert np.linalg.norm(rr.x - xp) <= 1e-13 * np.linalg.norm(xp)


def test_eliminated_form_identity():
    """alpha B [I - (L + I)^-1 B] == Gamma^-1 A with Gamma^-1 = alpha B (L + I)^-1 (Sec. 2.1)."""
    p = media.helmholtz_spheres(shape=(4, 4, 4), count=2, width=1, w0=1.0, plane=1)
    cp = canon.canonical_helmholtz(p.k2, p.source, p.spacing)
    op = operators.Operator(cp)
    A, L, B = op.dense_A(), op.dense_L(), op.dense_B()
    I = np.eye(A.shape[0])
    for alpha in (0.5, 1.0):
        lhs = alpha * B @ (I - np.linalg.solve(L + I, B))
        rhs = alpha * B @ np.linalg.solve(L + I, A)
        assert np.allclose(lhs, rhs, atol=1e-13)
        assert np.allclose(theory.eliminated(A, B, alpha), rhs, atol=1e-13)


def test_gaussian_source_matches_free_space_green_function():
    """Homogeneous absorbing medium (n = 1 + 0.1 i), Gaussian source of width sigma:
    outside the source psi = (2 pi sigma^2)^{3/2} e^{-k^2 sigma^2/2} e^{ikr}/(4 pi r)
    (radial-source form of the outgoing Green function of laplacian + k^2, Sec. 3.1),
    summed over the nearest periodic images."""
    N, h, sig = 48, 0.25, 0.4
    k = K0 * (1 + 0.1j)
    k2 = k * k
    g = (np.arange(N) - N // 2) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    r0 = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    S = np.exp(-r0 ** 2 / (2 * sig ** 2)).astype(complex)
    cp = canon.canonical_helmholtz(np.full((N,) * 3, k2), S, (h,) * 3,
                                   given=(k2.real, 1j * abs(k2.imag) / 0.95))
    res = R.solve(operators.Operator(cp), cp.y, 1.0, 1e-9, 5000, 20)
    assert res.converged
    Lb = N * h
    G = np.zeros_like(X, dtype=complex)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                r = np.sqrt((X + a * Lb) ** 2 + (Y + b * Lb) ** 2 + (Z + c * Lb) ** 2)
                with np.errstate(all="ignore"):
                    G += np.exp(1j * k * r) / (4 * np.pi * r)
    G *= (2 * np.pi * sig ** 2) ** 1.5 * np.exp(-k2 * sig ** 2 / 2)
    m = (r0 >= 2.0) & (r0 < 4.0)
    assert np.max(np.abs(res.x[m] - G[m]) / np.abs(G[m])) < 1e-3


def test_point_source_1d_green_function():
    """1-D: psi'' + k^2 psi = -delta has psi = (i/2k) e^{ik|x|}; periodic images summed
    as a geometric series.  The discrete delta is 1/h at one sample."""
    N, h = 256, 0.25
    k = K0 * (1 + 0.05j)
    k2 = k * k
    S = np.zeros(N, complex)
    S[N // 2] = 1 / h
    cp = canon.canonical_helmholtz(np.full(N, k2), S, (h,), given=(k2.real, 1j * abs(k2.imag) / 0.95))
    res = R.solve(operators.Operator(cp), cp.y, 1.0, 1e-12, 5000, 10)
    x = (np.arange(N) - N // 2) * h
    q = np.exp(1j * k * N * h)
    G = (1j / (2 * k)) * (np.exp(1j * k * np.abs(x)) + q * np.exp(-1j * k * np.abs(x))) / (1 - q)
    m = np.abs(x) >= 2
    assert np.max(np.abs(res.x[m] - G[m])) / np.max(np.abs(G[m])) < 1e-2


def test_stopping_rule_and_history():
    p = media.helmholtz_1d(n=64, width=8)
    cp = canon.canonical_helmholtz(p.k2, p.source, p.spacing)
    op = operators.Operator(cp)
    res = R.solve(op, cp.y, 0.8, 1e-6, 5000, 7)
    assert res.converged and res.iterations % 7 == 0
    assert res.hist_true[-1][1] < 1e-6 <= res.hist_true[-2][1]
    assert len(res.hist_pre) == res.iterations
    assert abs(R.relative_residual(op, res.x, cp.y) - res.hist_true[-1][1]) < 1e-15
