"""The antisymmetrised canonical form for problems whose numerical range is not
confined to a half plane (Sec. 2.2, Eq. antisymmetrised; applied to the
pantograph in Sec. 3.3).

TEST INFRASTRUCTURE (FP64 oracle) -- see ``oracle/__init__.py``.

From a canonical system A~ x~ = y~ with A~ = L~ + V~ (here: the pantograph,
scale c real), the larger system on x = [x~; x~'] is

    A = [[0, -A~*], [A~, 0]],   L = [[0, -L~*], [L~, 0]],   V = [[0, -V~*], [V~, 0]],
    y = [-y~'; y~]   (y~' = 0 unless an adjoint problem is solved too),

where * is the adjoint (conjugate transpose).  With c real, A is
skew-Hermitian, hence accretive, and ||V|| = ||V~|| <= 0.95, so Algorithm 1
converges for it.  Per Fourier mode L + I is the 2 x 2 block
[[1, -conj(l)], [l, 1]] with l = l~(p); its inverse is
[[1, conj(l)], [-l, 1]] / (1 + |l|^2).  The adjoint of the diagonal part of
V~ is its conjugate; the adjoint of the interpolation gather
(G x)_j = g0_j x[i_j] + g1_j x[i_j + 1] is the scatter
(G* z)_k = sum_j conj(g0_j) z_j [i_j = k] + conj(g1_j) z_j [i_j + 1 = k].
Fields are arrays of shape (2, N): component 0 is x~, component 1 is x~'.
"""
from __future__ import annotations

import numpy as np

from .operators import Operator


class AntisymOperator:
    """A, L, V, B = I - V and (L + I)^-1 of the antisymmetrised form of a 1-D operator."""

    def __init__(self, base: Operator):
        if len(base.shape) != 1:
            raise ValueError("the antisymmetrised form is built here for 1-D operators")
        self.base = base
        self.n = base.shape[0]
        self.shape = (2, self.n)
        self.l = base.l

    # V~ and its adjoint ------------------------------------------------------
    def _gather_adj(self, z):
        p = self.base.prob
        out = np.zeros(self.n, dtype=np.complex128)
        idx = np.asarray(p.gi)
        nxt = np.minimum(idx + 1, self.n - 1)
        np.add.at(out, idx, np.conj(p.g0) * z)
        np.add.at(out, nxt, np.conj(p.g1) * z)
        return out

    def apply_Vt(self, x):
        return self.base.apply_V(x)

    def apply_Vt_adj(self, z):
        out = np.conj(self.base.v) * z
        if self.base.has_gather:
            out = out + self._gather_adj(z)
        return out

    # block operators -----------------------------------------------------------
    def apply_V(self, x):
        return np.stack([-self.apply_Vt_adj(x[1]), self.apply_Vt(x[0])])

    def apply_B(self, x):
        return x - self.apply_V(x)

    def apply_L(self, x):
        F, Fi = np.fft.fft, np.fft.ifft
        return np.stack([-Fi(np.conj(self.l) * F(x[1])), Fi(self.l * F(x[0]))])

    def apply_LI_inv(self, t):
        F, Fi = np.fft.fft, np.fft.ifft
        t0, t1 = F(t[0]), F(t[1])
        l = self.l
        den = 1.0 + np.abs(l) ** 2
        return np.stack([Fi((t0 + np.conj(l) * t1) / den), Fi((-l * t0 + t1) / den)])

    def apply_A(self, x):
        return self.apply_L(x) + self.apply_V(x)

    def residual(self, x, y):
        return y - self.apply_A(x)

    def dense(self, fn):
        N = 2 * self.n
        M = np.empty((N, N), dtype=np.complex128)
        e = np.zeros(N, dtype=np.complex128)
        for j in range(N):
            e[:] = 0.0
            e[j] = 1.0
            M[:, j] = fn(e.reshape(self.shape)).ravel()
        return M


def rhs(y, y_adj=None):
    """y = [-y~'; y~] of the antisymmetrised system (y~' = 0 by default)."""
    y = np.asarray(y, dtype=np.complex128)
    ya = np.zeros_like(y) if y_adj is None else np.asarray(y_adj, dtype=np.complex128)
    return np.stack([-ya, y])
