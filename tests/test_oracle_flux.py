"""Pins for the flux-form diffusion oracle (CPU):
* eliminating the flux (Schur complement) gives the scalar equation
  -div(D grad u) + mu u = S with the same spectral derivatives: the u part of the
  dense flux-form solution equals that scalar solution;
* A is accretive and ||V|| = 0.95 (dense spectral norm);
* (L + I)^-1 per Fourier mode equals the dense inverse of L + I;
* an isotropic constant D reduces L~'s block symbol to the scalar diffusion
  symbol D |p|^2 + mubar in the Schur complement;
* the equilibration scales every nonzero row of the radii to maximum 1;
* Algorithm 1 decreases ||Delta|| monotonically and reaches the dense solution."""
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
