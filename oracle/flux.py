"""Diffusion in flux form with a tensor diffusion coefficient (Sec. 3.2, Eq.
diffusion-equation-matrix-form), steady state, on a 2-D periodic grid.

TEST INFRASTRUCTURE (FP64 oracle) -- see ``oracle/__init__.py``.

Fick's two laws, div J + mu u = S and D^-1 J + grad u = 0, on x~ = [u; Jx; Jy]
(x the contiguous axis 1, y axis 0):

    A~ = [[mu, d_x, d_y], [d_x, Di_xx, Di_xy], [d_y, Di_yx, Di_yy]],   y~ = [S; 0; 0],

with Di = D^-1 per voxel and d the spectral derivative (symbol i p, Nyquist
mode zero so that d is skew-Hermitian).  Splitting: L~ keeps the derivatives
and the biases mubar (smallest circle of {mu}) and Dibar (smallest circle of
each element of {Di} separately); V~ = blockdiag(mu - mubar, Di - Dibar).
Scaling (reading of the equilibration step): the radii of the circles form
dV = [[R_mu, 0, 0], [0, R_xx, R_xy], [0, R_yx, R_yy]]; a diagonal s > 0 is
found by symmetric infinity-norm equilibration (s_i <- s_i / sqrt(max_j s_i
dV_ij s_j), 50 sweeps; zero rows keep s_i = 1), then c = max over voxels of
||S V~ S||_2 / 0.95 (S = diag(s)).  The canonical system is

    A = S A~ S / c,   x = sqrt(c) S^-1 [u; J],   y = S y~ / sqrt(c),

so ||V|| = 0.95 and [u; J] = S x / sqrt(c).  L's symbol is S L~(p) S / c, a
3 x 3 block per Fourier mode, and (L + I)^-1 is its per-mode inverse.
Fields are arrays of shape (3, n0, n1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .canon import VNORM, smallest_circle


def _dspec(n, h):
    """Spectral derivative wavenumbers p = 2 pi fftfreq(n, h) with the Nyquist mode zeroed."""
    p = 2.0 * np.pi * np.fft.fftfreq(n, d=h)
    if n % 2 == 0:
        p[n // 2] = 0.0
    return p


def equilibrate(dV, sweeps=50):
    """Symmetric infinity-norm equilibration of a nonnegative matrix: s with
    max_j s_i dV_ij s_j = 1 for every nonzero row (zero rows: s_i = 1)."""
    dV = np.asarray(dV, dtype=float)
    s = np.ones(dV.shape[0])
    for _ in range(sweeps):
        for i in range(dV.shape[0]):
            r = max(s[i] * dV[i, j] * s[j] for j in range(dV.shape[0]))
            if r > 0.0:
                s[i] = s[i] / np.sqrt(r)
    return s


@dataclass
class FluxCanonical:
    shape: tuple         # (n0, n1)
    h: float
    s: np.ndarray        # (3,) equilibration
    c: float             # overall scale
    mubar: complex
    Dibar: np.ndarray    # (2, 2) complex
    Buu: np.ndarray      # (n0, n1) complex: 1 - s0^2 (mu - mubar)/c
    B2: np.ndarray       # (n0, n1, 2, 2): I - S2 (Di - Dibar) S2 / c
    y: np.ndarray        # (3, n0, n1)
    radii: np.ndarray    # dV


def canonical_flux(mu, D, source, h, vnorm=VNORM) -> FluxCanonical:
    """mu (n0, n1), D (n0, n1, 2, 2) (the tensor [[Dxx, Dxy], [Dyx, Dyy]]), source (n0, n1)."""
    mu = np.asarray(mu, dtype=np.complex128)
    D = np.asarray(D, dtype=np.complex128)
    Di = np.linalg.inv(D)
    def circle(vals):   # a constant set is its own centre, radius 0
        vals = vals.ravel()
        if np.all(vals == vals[0]):
            return vals[0], 0.0
        return smallest_circle(vals)

    mubar, Rmu = circle(mu)
    Dibar = np.zeros((2, 2), dtype=np.complex128)
    R2 = np.zeros((2, 2))
    for a in range(2):
        for b in range(2):
            Dibar[a, b], R2[a, b] = circle(Di[..., a, b])
    dV = np.zeros((3, 3))
    dV[0, 0] = Rmu
    dV[1:, 1:] = R2
    s = equilibrate(dV)
    S2 = np.diag(s[1:])
    Vu = s[0] ** 2 * (mu - mubar)
    V2 = S2 @ (Di - Dibar) @ S2
    norms = np.maximum(np.abs(Vu), np.linalg.norm(V2, ord=2, axis=(-2, -1)))
    c = float(norms.max()) / vnorm
    if not c > 0.0:
        c = 1.0
    Buu = 1.0 - Vu / c
    B2 = np.eye(2) - V2 / c
    y = np.zeros((3,) + mu.shape, dtype=np.complex128)
    y[0] = s[0] * np.asarray(source, dtype=np.complex128) / np.sqrt(c)
    return FluxCanonical(shape=mu.shape, h=float(h), s=s, c=c, mubar=mubar, Dibar=Dibar, Buu=Buu, B2=B2, y=y,
                         radii=dV)


class FluxOperator:
    """A = L + V, B = I - V and (L + I)^-1 of the canonical flux-form system."""

    def __init__(self, cp: FluxCanonical):
        self.cp = cp
        n0, n1 = cp.shape
        self.shape = (3, n0, n1)
        p0 = _dspec(n0, cp.h)[:, None] * np.ones((1, n1))
        p1 = np.ones((n0, 1)) * _dspec(n1, cp.h)[None, :]
        s, c = cp.s, cp.c
        Lt = np.zeros((n0, n1, 3, 3), dtype=np.complex128)
        Lt[..., 0, 0] = cp.mubar
        Lt[..., 0, 1] = 1j * p1
        Lt[..., 0, 2] = 1j * p0
        Lt[..., 1, 0] = 1j * p1
        Lt[..., 2, 0] = 1j * p0
        Lt[..., 1:, 1:] = cp.Dibar
        self.lsym = (s[:, None] * s[None, :]) * Lt / c          # S L~(p) S / c per mode
        self.lsym_inv = np.linalg.inv(self.lsym + np.eye(3))

    def _modes(self, x, M):
        xh = np.fft.fft2(x, axes=(1, 2))
        yh = np.einsum("...ij,j...->i...", M, xh)
        return np.fft.ifft2(yh, axes=(1, 2))

    def apply_L(self, x):
        return self._modes(x, self.lsym)

    def apply_LI_inv(self, t):
        return self._modes(t, self.lsym_inv)

    def apply_V(self, x):
        cp = self.cp
        out = np.empty_like(x)
        out[0] = (1.0 - cp.Buu) * x[0]
        V2 = np.eye(2) - cp.B2
        out[1] = V2[..., 0, 0] * x[1] + V2[..., 0, 1] * x[2]
        out[2] = V2[..., 1, 0] * x[1] + V2[..., 1, 1] * x[2]
        return out

    def apply_B(self, x):
        return x - self.apply_V(x)

    def apply_A(self, x):
        return self.apply_L(x) + self.apply_V(x)

    def residual(self, x, y):
        return y - self.apply_A(x)

    def dense(self, fn):
        N = int(np.prod(self.shape))
        M = np.empty((N, N), dtype=np.complex128)
        e = np.zeros(N, dtype=np.complex128)
        for j in range(N):
            e[:] = 0.0
            e[j] = 1.0
            M[:, j] = fn(e.reshape(self.shape)).ravel()
        return M

    def physical(self, x):
        """[u; J] = S x / sqrt(c)."""
        return self.cp.s[:, None, None] * x / np.sqrt(self.cp.c)
