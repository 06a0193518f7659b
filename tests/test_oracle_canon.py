"""Pins for the oracle's canonicalisation (paper Sec. 2.2, 3.1-3.3)."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import canon, operators, theory
from paper_2207_14222_amd import media

GOLD = os.path.join(os.path.dirname(__file__), "golden", "mec_cases.txt")


def _parse_pts(s):
    return np.array([complex(*map(float, p.split(","))) for p in s.split()])


def _gold():
    out = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        kind, pts, cen, rad = [f.strip() for f in line.split("|")]
        out.append((kind, _parse_pts(pts), complex(*map(float, cen.split(","))), float(rad)))
    return out


@pytest.mark.parametrize("case", _gold())
def test_mec_golden(case):
    kind, pts, cen, rad = case
    if kind == "complex":
        z, r = canon.smallest_circle(pts)
    else:
        z, r = canon.smallest_real_centre(pts)
    assert abs(z - cen) < 1e-12 and abs(r - rad) < 1e-12


def _brute_force_mec(pts):
    """All 2- and 3-point circles over every point (no hull), the smallest enclosing one."""
    best = math.inf
    for a, b in itertools.combinations(pts, 2):
        z = (a + b) / 2
        r = abs(a - b) / 2
        if np.all(np.abs(pts - z) <= r * (1 + 1e-12)):
            best = min(best, r)
    for a, b, c in itertools.combinations(pts, 3):
        M = np.array([[2 * (b - a).real, 2 * (b - a).imag], [2 * (c - a).real, 2 * (c - a).imag]])
        if abs(np.linalg.det(M)) < 1e-14:
            continue
        rhs = np.array([abs(b) ** 2 - abs(a) ** 2, abs(c) ** 2 - abs(a) ** 2])
        zx, zy = np.linalg.solve(M, rhs)
        z = complex(zx, zy)
        r = abs(z - a)
        if np.all(np.abs(pts - z) <= r * (1 + 1e-12)):
            best = min(best, r)
    return best


@pytest.mark.parametrize("seed", range(6))
def test_mec_vs_brute_force(seed):
    rng = np.random.default_rng(seed)
    pts = rng.normal(size=9) + 1j * rng.normal(size=9) * (0.3 + seed)
    z, r = canon.smallest_circle(pts)
    assert np.max(np.abs(pts - z)) <= r * (1 + 1e-12)
    assert abs(r - _brute_force_mec(pts)) < 1e-12 * max(1, r)


def test_mec_real_centre_is_optimal():
    rng = np.random.default_rng(7)
    pts = rng.normal(size=15) * 3 + 1j * np.abs(rng.normal(size=15))
    b, r = canon.smallest_real_centre(pts)
    assert b.imag == 0
    grid = np.linspace(b.real - 1, b.real + 1, 20001)
    f = np.max(np.abs(pts[None, :] - grid[:, None]), axis=1)
    assert r <= f.min() + 1e-12
    assert abs(r - np.max(np.abs(pts - b))) < 1e-14


def _lap_sum(x, spacing):
    # the Laplacian is a sum of second derivatives: apply each axis to x separately
    total = np.zeros_like(x, dtype=np.complex128)
    for ax in range(x.ndim):
        n, h = x.shape[ax], spacing[ax]
        j = np.arange(n)
        F = np.exp(-2j * np.pi * np.outer(j, j) / n)
        kk = np.where(j < n // 2, j, j - n)
        p = 2 * np.pi * kk / (n * h)
        D2 = np.linalg.inv(F) @ np.diag(-(p ** 2)) @ F
        total += np.moveaxis(np.tensordot(D2, np.moveaxis(x, ax, 0), axes=(1, 0)), 0, ax)
    return total


@pytest.mark.parametrize("shape", [(16,), (8, 6), (4, 6, 8)])
def test_helmholtz_canonical_operator(shape):
    """c A x = laplacian x + k^2 x,  y = -S/c,  max|v| = 0.95,  A accretive (Sec. 3.1)."""
    rng = np.random.default_rng(len(shape))
    nidx = 1.2 + 0.2 * rng.random(shape) + 1j * 0.1 * rng.random(shape)
    k2 = (media.K0 * nidx) ** 2
    S = rng.normal(size=shape) + 0j
    sp = (0.25,) * len(shape)
    cp = canon.canonical_helmholtz(k2, S, sp)
    op = operators.Operator(cp)
    x = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    lhs = cp.c * op.apply_A(x)
    rhs = _lap_sum(x, sp) + k2 * x
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(rhs)
    assert np.allclose(cp.y * cp.c, -S)
    assert abs(np.max(np.abs(cp.v)) - 0.95) < 1e-12
    assert abs(cp.c.real) < 1e-12 * abs(cp.c) and cp.c.imag > 0  # c = i R / 0.95
    A = op.dense_A()
    assert theory.re_part(A) >= -1e-10  # accretive


def test_helmholtz_real_bias():
    p = media.helmholtz_1d(n=64, width=8)
    cp = canon.canonical_helmholtz(p.k2, p.source, p.spacing, bias="real")
    assert cp.bias.imag == 0.0
    assert abs(np.max(np.abs(cp.v)) - 0.95) < 1e-12
    A = operators.Operator(cp).dense_A()
    assert theory.re_part(A) >= -1e-10


def test_diffusion_canonical_operator():
    """c A x = -D laplacian x + mu_a x - i (omega/v) x,  y = S/c,  max|v| = 0.95 (Sec. 3.2)."""
    d = media.diffusion_blobs(shape=(4, 6, 8), sigma=1.0)
    cp = canon.canonical_diffusion(d.mu_a, d.D, d.omega_over_v, d.source, d.spacing)
    op = operators.Operator(cp)
    rng = np.random.default_rng(3)
    x = rng.normal(size=d.shape) + 1j * rng.normal(size=d.shape)
    lhs = cp.c * op.apply_A(x)
    rhs = -d.D * _lap_sum(x, d.spacing) + d.mu_a * x - 1j * d.omega_over_v * x
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(rhs)
    assert abs(np.max(np.abs(cp.v)) - 0.95) < 1e-12
    assert np.isreal(cp.c) and cp.c > 0
    assert theory.re_part(op.dense_A()) >= -1e-10


def test_pantograph_gather_interpolates_linear_functions():
    """(S x)(t_j) = x(lam t_j) exactly for x linear in t (linear interpolation)."""
    n, h, t0 = 64, 0.01, 1.0
    for lam in (0.5, 0.9, 0.37):
        idx, w0, w1 = canon.pantograph_gather(n, lam, t0, h)
        S = canon.gather_matrix(n, idx, w0, w1)
        t = t0 + h * np.arange(n)
        x = 3.0 - 2.0 * t
        valid = lam * t >= t0
        assert np.allclose((S @ x)[valid], (3.0 - 2.0 * lam * t)[valid], atol=1e-12)
        assert np.all((S @ x)[~valid] == 0)


def test_pantograph_canonical_operator():
    """c A x = x' + a x + b x(lam t) with x' the spectral derivative (Nyquist mode 0);
    ||V||_2 <= 0.95 (Sec. 3.3)."""
    n = 32
    pp = media.pantograph(n=n, h=0.2)
    cp = canon.canonical_pantograph(pp.a, pp.b, pp.lam, pp.t0, pp.h, pp.x0_at_lam_t, pp.x0_t0)
    op = operators.Operator(cp)
    j = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(j, j) / n)
    kk = np.where(j < n // 2, j, j - n).astype(float)
    kk[n // 2] = 0.0
    Dt = np.linalg.inv(F) @ np.diag(1j * 2 * np.pi * kk / (n * pp.h)) @ F
    S = canon.gather_matrix(n, *canon.pantograph_gather(n, pp.lam, pp.t0, pp.h))
    A0 = Dt + np.diag(pp.a) + np.diag(pp.b) @ S
    assert np.allclose(cp.c * op.dense_A(), A0, atol=1e-10)
    assert theory.opnorm(op.dense_V()) <= 0.95 + 1e-12
    y0 = pp.b * pp.x0_at_lam_t
    y0[0] += pp.x0_t0 / pp.h
    assert np.allclose(cp.c * cp.y, y0)
