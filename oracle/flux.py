"""Diffusion in flux form with a tensor diffusion coefficient (Sec. 3.2, Eq.
diffusion-equation-matrix-form), steady state, on a periodic 2-D or 3-D grid.

TEST INFRASTRUCTURE (FP64 oracle) -- see ``oracle/__init__.py``.

Fick's two laws, div J + mu u = S and D^-1 J + grad u = 0, on
x~ = [u; J_1; ...; J_d] (d = 2 or 3).  Flux component k pairs with grid axis
d - k: J_1 = J_x with the contiguous (last) axis, J_2 = J_y with the one
before, J_3 = J_z with axis 0 in 3-D.  With d_k the spectral derivative along
that axis (symbol i p, Nyquist mode zero so that d is skew-Hermitian),

    A~ = [[mu, d_1 .. d_d], [d_1 .. d_d (column), D^-1]],   y~ = [S; 0 .. 0],

D = [[D_xx, D_xy, ..], ..] in the (x, y[, z]) order of the flux components and
D^-1 its per-voxel inverse.  Splitting: L~ keeps the derivatives and the
biases mubar (smallest circle of {mu}) and Dibar (smallest circle of each
element of {D^-1} separately); V~ = blockdiag(mu - mubar, D^-1 - Dibar).
Scaling (reading of the equilibration step): the radii of the circles form
dV = blockdiag(R_mu, [R_ab]); a diagonal s > 0 is found by symmetric
infinity-norm equilibration (s_i <- s_i / sqrt(max_j s_i dV_ij s_j), 50
sweeps; zero rows keep s_i = 1), then c = max over voxels of ||S V~ S||_2 /
0.95 (S = diag(s)).  The canonical system is

    A = S A~ S / c,   x = sqrt(c) S^-1 [u; J],   y = S y~ / sqrt(c),

so ||V|| = 0.95 and [u; J] = S x / sqrt(c).  L's symbol is S L~(p) S / c, a
(1 + d) x (1 + d) block per Fourier mode, and (L + I)^-1 is its per-mode
inverse.  Fields are arrays of shape (1 + d,) + grid.
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
    shape: tuple         # grid shape (n0, n1[, n2])
    h: float
    s: np.ndarray        # (1 + d,) equilibration
    c: float             # overall scale
    mubar: complex
    Dibar: np.ndarray    # (d, d) complex
    Buu: np.ndarray      # grid: 1 - s0^2 (mu - mubar)/c
    B2: np.ndarray       # grid + (d, d): I - S' (Di - Dibar) S' / c
    y: np.ndarray        # (1 + d,) + grid
    radii: np.ndarray    # dV

    @property
    def ndim(self):
        return len(self.shape)


def canonical_flux(mu, D, source, h, vnorm=VNORM) -> FluxCanonical:
    """mu (grid), D (grid + (d, d)) in the (x, y[, z]) order of the flux components, source (grid)."""
    mu = np.asarray(mu, dtype=np.complex128)
    D = np.asarray(D, dtype=np.complex128)
    d = mu.ndim
    Di = np.linalg.inv(D)

    def circle(vals):   # a constant set is its own centre, radius 0
        vals = vals.ravel()
        if np.all(vals == vals[0]):
            return vals[0], 0.0
        return smallest_circle(vals)

    mubar, Rmu = circle(mu)
    Dibar = np.zeros((d, d), dtype=np.complex128)
    R2 = np.zeros((d, d))
    for a in range(d):
        for b in range(d):
            Dibar[a, b], R2[a, b] = circle(Di[..., a, b])
    dV = np.zeros((1 + d, 1 + d))
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
    B2 = np.eye(d) - V2 / c
    y = np.zeros((1 + d,) + mu.shape, dtype=np.complex128)
    y[0] = s[0] * np.asarray(source, dtype=np.complex128) / np.sqrt(c)
    return FluxCanonical(shape=mu.shape, h=float(h), s=s, c=c, mubar=mubar, Dibar=Dibar, Buu=Buu, B2=B2, y=y,
                         radii=dV)


class FluxOperator:
    """A = L + V, B = I - V and (L + I)^-1 of the canonical flux-form system."""

    def __init__(self, cp: FluxCanonical):
        self.cp = cp
        d = len(cp.shape)
        self.d = d
        self.shape = (1 + d,) + tuple(cp.shape)
        s, c = cp.s, cp.c
        Lt = np.zeros(tuple(cp.shape) + (1 + d, 1 + d), dtype=np.complex128)
        Lt[..., 0, 0] = cp.mubar
        for k in range(1, d + 1):
            ax = d - k                               # flux component k pairs with axis d - k
            pk = _dspec(cp.shape[ax], cp.h)
            shp = [1] * d
            shp[ax] = cp.shape[ax]
            pk = pk.reshape(shp)
            Lt[..., 0, k] = 1j * pk
            Lt[..., k, 0] = 1j * pk
        Lt[..., 1:, 1:] = cp.Dibar
        self.lsym = (s[:, None] * s[None, :]) * Lt / c          # S L~(p) S / c per mode
        self.lsym_inv = np.linalg.inv(self.lsym + np.eye(1 + d))

    def _modes(self, x, M):
        axes = tuple(range(1, self.d + 1))
        xh = np.fft.fftn(x, axes=axes)
        yh = np.einsum("...ij,j...->i...", M, xh)
        return np.fft.ifftn(yh, axes=axes)

    def apply_L(self, x):
        return self._modes(x, self.lsym)

    def apply_LI_inv(self, t):
        return self._modes(t, self.lsym_inv)

    def apply_V(self, x):
        cp = self.cp
        out = np.empty_like(x)
        out[0] = (1.0 - cp.Buu) * x[0]
        V2 = np.eye(self.d) - cp.B2
        out[1:] = np.einsum("...ab,b...->a...", V2, x[1:])
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
        return self.cp.s.reshape((-1,) + (1,) * self.d) * x / np.sqrt(self.cp.c)
