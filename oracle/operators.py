"""Discrete operators of a canonical problem (paper Sec. 2.1 and Eq. laplacian_inverse).

TEST INFRASTRUCTURE (FP64 oracle) -- see ``oracle/__init__.py``.

Discretisation (the paper's "Fourier-space coordinate vector p" on a regular
grid): periodic grid, unnormalised forward DFT F over all axes, and
p = 2 pi * fftfreq(n, h) per axis.  L = F^-1 diag(l(p)) F with
l(p) = s (a0 + a2 |p|^2 + a1 i p); for the first-derivative (1-D) symbol the
Nyquist mode of i p is set to zero so that d/dt stays skew-Hermitian.
(L + I)^-1 = F^-1 diag(1/(l(p) + 1)) F, which for Helmholtz is exactly
F^-1 c/(-|p|^2 + kbar^2 + c) F.

The multi-dimensional transforms F and F^-1 are a library routine: pocketfft
through ``scipy.fft`` with FFT_WORKERS threads (numpy.fft, the same algorithm
single-threaded, when SciPy is absent).  Both are pinned against a naive DFT
over every axis in the tests.
"""
from __future__ import annotations

import os

import numpy as np

from .canon import Canonical

try:
    import scipy.fft as _sfft
except ImportError:  # pragma: no cover
    _sfft = None

# threads of the library FFT (the host's cores, at most 16)
FFT_WORKERS = max(1, min(16, os.cpu_count() or 1))


def fftn(x):
    """Unnormalised forward DFT over all axes."""
    if _sfft is not None:
        return _sfft.fftn(x, workers=FFT_WORKERS)
    return np.fft.fftn(x)


def ifftn(x):
    """Inverse DFT over all axes, with the 1/N."""
    if _sfft is not None:
        return _sfft.ifftn(x, workers=FFT_WORKERS)
    return np.fft.ifftn(x)


def wavenumbers(n: int, h: float) -> np.ndarray:
    """p_k = 2 pi fftfreq(n, h): k/(n h) 2pi for k < n/2, (k - n)/(n h) 2pi otherwise."""
    return 2.0 * np.pi * np.fft.fftfreq(n, d=h)


def symbol(prob: Canonical) -> np.ndarray:
    """l(p) on the full FFT grid (complex128, same shape as the field)."""
    shape, spacing = prob.shape, prob.spacing
    p2 = np.zeros(shape)
    for ax, (n, h) in enumerate(zip(shape, spacing)):
        p = wavenumbers(n, h)
        sh = [1] * len(shape)
        sh[ax] = n
        p2 = p2 + (p ** 2).reshape(sh)
    l = prob.a0 + prob.a2 * p2
    if prob.a1 != 0:
        if len(shape) != 1:
            raise ValueError("first-derivative symbol is 1-D only")
        p = wavenumbers(shape[0], spacing[0])
        if prob.nyquist_zero and shape[0] % 2 == 0:
            p = p.copy()
            p[shape[0] // 2] = 0.0
        l = l + prob.a1 * 1j * p
    return prob.s * l


class Operator:
    """A = L + V, B = I - V and (L + I)^-1 for a canonical problem."""

    def __init__(self, prob: Canonical):
        self.prob = prob
        self.shape = prob.shape
        self.l = symbol(prob)
        self.v = np.asarray(prob.v, dtype=np.complex128)
        self.has_gather = prob.gi is not None

    # V, B ---------------------------------------------------------------
    def gather(self, x):
        p = self.prob
        idx = p.gi
        nxt = np.minimum(idx + 1, x.shape[0] - 1)
        return p.g0 * x[idx] + p.g1 * x[nxt]

    def apply_V(self, x):
        out = self.v * x
        if self.has_gather:
            out = out + self.gather(x)
        return out

    def apply_B(self, x):
        """B x = x - V x."""
        return x - self.apply_V(x)

    # L, (L + I)^-1, A ----------------------------------------------------
    def apply_L(self, x):
        return ifftn(self.l * fftn(x))

    def apply_LI_inv(self, t):
        """(L + I)^-1 t = F^-1 [ F t / (l + 1) ]   (Eq. laplacian_inverse)."""
        return ifftn(fftn(t) / (self.l + 1.0))

    def apply_A(self, x):
        return self.apply_L(x) + self.apply_V(x)

    def residual(self, x, y):
        """r = y - A x."""
        return y - self.apply_A(x)

    # dense matrices (tiny grids) -----------------------------------------
    def _dense(self, fn):
        N = int(np.prod(self.shape))
        M = np.empty((N, N), dtype=np.complex128)
        e = np.zeros(N, dtype=np.complex128)
        for j in range(N):
            e[:] = 0.0
            e[j] = 1.0
            M[:, j] = fn(e.reshape(self.shape)).ravel()
        return M

    def dense_A(self):
        return self._dense(self.apply_A)

    def dense_L(self):
        return self._dense(self.apply_L)

    def dense_V(self):
        return self._dense(self.apply_V)

    def dense_B(self):
        return self._dense(self.apply_B)
