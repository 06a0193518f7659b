"""Pins for the flux-form diffusion oracle (CPU):
* eliminating the flux (Schur complement) gives the scalar equation
  -div(D grad u) + mu u = S with the same spectral derivatives: the u part of the
  dense flux-form solution equals that scalar solution;
* A is accretive and ||V|| = 0.95 (dense spectral norm);
* (L + I)^-1 per Fourier mode equals the dense inverse of L + I;
* an isotropic constant D reduces L~'s block symbol to the scalar diffusion
  symbol D |p|^2 + mubar in the Schur complement;
* the equilibration scales every nonzero row of the radii to maximum 1;
* Algorithm 1 decreases ||Delta|| monotonically and reaches the dense solution;
* the same in 3-D with four components [u; Jx; Jy; Jz] on a non-cubic grid
  (the Schur complement against the scalar equation fixes which flux
  component pairs with which axis)."""
import numpy as np
import pytest

from oracle import flux as F
from oracle import richardson as R
from paper_2207_14222_amd import media


@pytest.fixture(scope="module")
def ring():
    p = media.diffusion_ring(n=16, h=0.6, radius=3.0, width=1.5, abs_rows=3, src_row=2)
    cp = F.canonical_flux(p.mu, p.D, p.source, p.h)
    return p, cp, F.FluxOperator(cp)


def _deriv_matrix(n0, n1, h, axis):
    """Dense spectral derivative (Nyquist mode zero) along an axis of an (n0, n1) grid."""
    N = n0 * n1
    M = np.empty((N, N), dtype=complex)
    e = np.zeros(N, dtype=complex)
    p = F._dspec(n0 if axis == 0 else n1, h)
    for j in range(N):
        e[:] = 0
        e[j] = 1
        f = np.fft.fft(e.reshape(n0, n1), axis=axis)
        f = f * (1j * (p[:, None] if axis == 0 else p[None, :]))
        M[:, j] = np.fft.ifft(f, axis=axis).ravel()
    return M


def test_schur_complement_is_the_scalar_equation(ring):
    p, cp, op = ring
    n0, n1 = cp.shape
    A = op.dense(op.apply_A)
    x = np.linalg.solve(A, cp.y.ravel()).reshape(op.shape)
    u = op.physical(x)[0]
    Gx = _deriv_matrix(n0, n1, p.h, 1)
    Gy = _deriv_matrix(n0, n1, p.h, 0)
    Dxx, Dxy = np.diag(p.D[..., 0, 0].ravel()), np.diag(p.D[..., 0, 1].ravel())
    Dyx, Dyy = np.diag(p.D[..., 1, 0].ravel()), np.diag(p.D[..., 1, 1].ravel())
    # J = -D grad u;  div J + mu u = S
    K = -(Gx @ (Dxx @ Gx + Dxy @ Gy) + Gy @ (Dyx @ Gx + Dyy @ Gy)) + np.diag(p.mu.ravel())
    us = np.linalg.solve(K, p.source.ravel()).reshape(cp.shape)
    assert np.linalg.norm(u - us) / np.linalg.norm(us) < 1e-10


def test_accretive_vnorm_and_block_inverse(ring):
    p, cp, op = ring
    A = op.dense(op.apply_A)
    assert np.linalg.eigvalsh(0.5 * (A + A.conj().T)).min() > -1e-12
    V = op.dense(op.apply_V)
    assert abs(np.linalg.norm(V, 2) - 0.95) < 1e-12
    L = op.dense(op.apply_L)
    LI = op.dense(op.apply_LI_inv)
    assert np.allclose(LI, np.linalg.inv(L + np.eye(L.shape[0])), atol=1e-12)


def test_isotropic_symbol_schur_reduces_to_scalar_diffusion():
    """With D = d I everywhere, the 3x3 symbol's Schur complement on the u row is
    (mubar + d |p'|^2) (scaled), p' the derivative wavenumbers."""
    n, h, d, mu0 = 8, 0.5, 1.7, 0.3
    D = np.zeros((n, n, 2, 2), dtype=complex)
    D[..., 0, 0] = d
    D[..., 1, 1] = d
    mu = np.full((n, n), mu0, dtype=complex)
    mu[0, 0] = 2.0                      # some variation so that c is defined by mu
    cp = F.canonical_flux(mu, D, np.zeros((n, n)), h)
    op = F.FluxOperator(cp)
    Lt = op.lsym * cp.c / (cp.s[:, None] * cp.s[None, :])   # undo the scaling
    p0 = F._dspec(n, h)[:, None]
    p1 = F._dspec(n, h)[None, :]
    schur = Lt[..., 0, 0] - (Lt[..., 0, 1] * Lt[..., 1, 0] / Lt[..., 1, 1] + Lt[..., 0, 2] * Lt[..., 2, 0] / Lt[..., 2, 2])
    assert np.allclose(schur, cp.mubar + d * (p0 ** 2 + p1 ** 2), atol=1e-12)


def test_equilibration():
    dV = np.array([[10.0, 0.0, 0.0], [0.0, 0.48, 0.2], [0.0, 0.2, 0.3]])
    s = F.equilibrate(dV)
    scaled = s[:, None] * dV * s[None, :]
    assert np.allclose(scaled.max(axis=1), 1.0, atol=1e-10)
    s0 = F.equilibrate(np.array([[0.0, 0.0], [0.0, 4.0]]))
    assert s0[0] == 1.0 and abs(s0[1] - 0.5) < 1e-12


def test_fixed_point_monotone_to_dense_solution(ring):
    p, cp, op = ring
    x = np.linalg.solve(op.dense(op.apply_A), cp.y.ravel()).reshape(op.shape)
    res = R.solve(op, cp.y, 1.0, 1e-10, 20000, 10)
    assert res.converged
    d = np.array(res.hist_pre)
    assert np.all(np.diff(d) <= 1e-13 * d[0])
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-8


# ---- 3-D: four components [u; Jx; Jy; Jz] -----------------------------------

@pytest.fixture(scope="module")
def cube():
    p = media.diffusion_tensor_random3(shape=(4, 6, 8), seed=5, h=0.7)
    cp = F.canonical_flux(p.mu, p.D, p.source, p.h)
    return p, cp, F.FluxOperator(cp)


def _deriv_nd(shape, h, axis):
    """Dense spectral derivative (Nyquist mode zero) along one axis of a grid."""
    N = int(np.prod(shape))
    M = np.empty((N, N), dtype=complex)
    e = np.zeros(N, dtype=complex)
    p = F._dspec(shape[axis], h)
    shp = [1] * len(shape)
    shp[axis] = shape[axis]
    p = p.reshape(shp)
    for j in range(N):
        e[:] = 0
        e[j] = 1
        f = np.fft.fft(e.reshape(shape), axis=axis) * (1j * p)
        M[:, j] = np.fft.ifft(f, axis=axis).ravel()
    return M


def test_3d_schur_complement_is_the_scalar_equation(cube):
    """u of the dense 4-component solution solves -div(D grad u) + mu u = S, with the
    flux components in x, y, z order (x the last, contiguous axis)."""
    p, cp, op = cube
    x = np.linalg.solve(op.dense(op.apply_A), cp.y.ravel()).reshape(op.shape)
    u = op.physical(x)[0]
    G = [_deriv_nd(cp.shape, p.h, 2), _deriv_nd(cp.shape, p.h, 1), _deriv_nd(cp.shape, p.h, 0)]   # d/dx, d/dy, d/dz
    K = np.diag(p.mu.ravel()).astype(complex)
    for a in range(3):
        for b in range(3):
            K -= G[a] @ np.diag(p.D[..., a, b].ravel()) @ G[b]
    us = np.linalg.solve(K, p.source.ravel()).reshape(cp.shape)
    assert np.linalg.norm(u - us) / np.linalg.norm(us) < 1e-10


def test_3d_accretive_vnorm_block_inverse_and_convergence(cube):
    p, cp, op = cube
    A = op.dense(op.apply_A)
    assert np.linalg.eigvalsh(0.5 * (A + A.conj().T)).min() > -1e-12
    assert abs(np.linalg.norm(op.dense(op.apply_V), 2) - 0.95) < 1e-12
    L = op.dense(op.apply_L)
    assert np.allclose(op.dense(op.apply_LI_inv), np.linalg.inv(L + np.eye(L.shape[0])), atol=1e-12)
    xs = np.linalg.solve(A, cp.y.ravel()).reshape(op.shape)
    res = R.solve(op, cp.y, 1.0, 1e-10, 20000, 10)
    assert res.converged
    d = np.array(res.hist_pre)
    assert np.all(np.diff(d) <= 1e-13 * d[0])
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) < 1e-8


def test_3d_isotropic_symbol_schur_reduces_to_scalar_diffusion():
    shape, h, dd = (4, 6, 8), 0.5, 1.3
    D = np.zeros(shape + (3, 3), dtype=complex)
    for a in range(3):
        D[..., a, a] = dd
    mu = np.full(shape, 0.4, dtype=complex)
    mu[0, 0, 0] = 2.0
    cp = F.canonical_flux(mu, D, np.zeros(shape), h)
    op = F.FluxOperator(cp)
    Lt = op.lsym * cp.c / (cp.s[:, None] * cp.s[None, :])
    p2 = sum(F._dspec(n, h).reshape([n if i == ax else 1 for i in range(3)]) ** 2 for ax, n in enumerate(shape))
    schur = Lt[..., 0, 0] - sum(Lt[..., 0, k] * Lt[..., k, 0] / Lt[..., k, k] for k in (1, 2, 3))
    assert np.allclose(schur, cp.mubar + dd * p2, atol=1e-12)
