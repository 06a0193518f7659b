"""Conversion to canonical form (paper Sec. 2.2) and the operator splittings of
Sec. 3.1 (Helmholtz), 3.2 (diffusion, scalar constant-D form) and 3.3 (pantograph).

TEST INFRASTRUCTURE (FP64 oracle) -- see ``oracle/__init__.py``.

Canonical form: the raw problem A0 x = y0 is split as A0 = L0 + V0 with L0 close
to A0; dividing everything by a scalar c gives A = A0/c, L = L0/c, y = y0/c and
V = A - L with ||V|| = 0.95 (Sec. 2.2).  For a diagonal V the operator norm is
max |v|, so c is the radius of the smallest disc enclosing the diagonal entries
of V0, divided by 0.95.  The disc centre (the "bias") is the solution of the
smallest-circle problem (Sec. 3.1).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

VNORM = 0.95  # target ||V|| (Sec. 2.2)


# --------------------------------------------------------------------------
# Smallest enclosing circle of points in the complex plane
# --------------------------------------------------------------------------
def _convex_hull(pts: np.ndarray) -> np.ndarray:
    """Vertices of the convex hull of complex points (Andrew's monotone chain).

    The smallest enclosing circle of a set equals that of its hull vertices,
    because the farthest point of the set from any centre is an extreme point.
    """
    u = np.unique(pts)
    if u.size <= 2:
        return u
    order = np.lexsort((u.imag, u.real))
    p = u[order]

    def cross(o, a, b):
        return (a.real - o.real) * (b.imag - o.imag) - (a.imag - o.imag) * (b.real - o.real)

    lower, upper = [], []
    for q in p:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], q) <= 0:
            lower.pop()
        lower.append(q)
    for q in p[::-1]:
        while len(upper) >= 2 and cross(upper[-2], upper[-1], q) <= 0:
            upper.pop()
        upper.append(q)
    return np.array(lower[:-1] + upper[:-1])


def _circumcircle(a: complex, b: complex, c: complex):
    """Centre and radius of the circle through three non-collinear points."""
    ax, ay, bx, by, cx, cy = a.real, a.imag, b.real, b.imag, c.real, c.imag
    d = 2.0 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
    if abs(d) < 1e-300:
        return None
    a2, b2, c2 = ax * ax + ay * ay, bx * bx + by * by, cx * cx + cy * cy
    ux = (a2 * (by - cy) + b2 * (cy - ay) + c2 * (ay - by)) / d
    uy = (a2 * (cx - bx) + b2 * (ax - cx) + c2 * (bx - ax)) / d
    z = complex(ux, uy)
    return z, abs(z - a)


def smallest_circle(points, use_hull: bool = True):
    """Smallest disc containing all ``points`` (complex), by exhaustive search.

    The optimal disc is determined by two points (as a diameter) or three points
    (circumcircle) of the set.  Every such candidate that contains all points is
    generated and the smallest is returned.  O(h^4) in the number h of hull
    vertices; ``use_hull=False`` searches all distinct points (tiny sets only).
    Returns (centre, radius).
    """
    pts = np.asarray(points, dtype=np.complex128).ravel()
    cand = _convex_hull(pts) if use_hull else np.unique(pts)
    if cand.size == 1:
        return complex(cand[0]), 0.0
    best = (None, math.inf)
    tol = 1e-12

    def encloses(z, r):
        return np.max(np.abs(cand - z)) <= r * (1.0 + tol) + 1e-300

    for a, b in itertools.combinations(cand, 2):
        z = 0.5 * (a + b)
        r = abs(a - b) * 0.5
        if r < best[1] and encloses(z, r):
            best = (z, r)
    for a, b, c in itertools.combinations(cand, 3):
        cc = _circumcircle(complex(a), complex(b), complex(c))
        if cc is None:
            continue
        z, r = cc
        if r < best[1] and encloses(z, r):
            best = (z, r)
    # the radius is re-evaluated against every original point
    z = complex(best[0])
    return z, float(np.max(np.abs(pts - z)))


def smallest_real_centre(points):
    """Real b minimising max |z_j - b| (bias restricted to the real axis, Sec. 4.1).

    The optimum is either the real part of one point (when that point alone is
    farthest) or a point equidistant from two points; all candidates are tried.
    """
    pts = np.asarray(points, dtype=np.complex128).ravel()
    cand = _convex_hull(pts)
    bs = [float(z.real) for z in cand]
    for a, b in itertools.combinations(cand, 2):
        if a.real != b.real:
            bs.append((abs(a) ** 2 - abs(b) ** 2) / (2.0 * (a.real - b.real)))
    best_b, best_r = None, math.inf
    for b in bs:
        r = float(np.max(np.abs(cand - b)))
        if r < best_r:
            best_b, best_r = b, r
    return complex(best_b, 0.0), float(np.max(np.abs(pts - best_b)))


# --------------------------------------------------------------------------
# Canonical problems
# --------------------------------------------------------------------------
@dataclass
class Canonical:
    """A canonical problem  A x = y,  A = L + V,  ||V|| <= 0.95.

    L is the translation-invariant operator with Fourier symbol
    l(p) = s * (a0 + a2 |p|^2 + a1 * i p)   (a1 used in 1-D only),
    V = diag(v) (+ an optional gather term for the pantograph).
    """
    shape: tuple
    spacing: tuple
    s: complex
    a0: complex
    a1: complex
    a2: complex
    v: np.ndarray                    # complex128 diagonal of V
    y: np.ndarray                    # complex128 right-hand side
    c: complex                       # overall scale
    bias: complex                    # L0 offset (k-bar^2, mu-bar, a-bar)
    # pantograph gather:  (G x)_j = g0_j x[gi_j] + g1_j x[gi_j + 1]
    gi: Optional[np.ndarray] = None
    g0: Optional[np.ndarray] = None
    g1: Optional[np.ndarray] = None
    nyquist_zero: bool = False       # first-derivative symbol with the Nyquist mode set to 0
    extra: dict = field(default_factory=dict)

    @property
    def B(self):
        """Diagonal of B = I - V (pantograph: diagonal part only)."""
        return 1.0 - self.v


def canonical_helmholtz(k2, source, spacing, bias: str = "complex", given=None, vnorm=VNORM):
    """Helmholtz splitting (Sec. 3.1).

    Raw problem  (laplacian + k^2) psi = -S.  L0 = laplacian + kbar^2 with kbar^2
    the smallest-circle centre of {k^2(r)} (bias='complex'), the best real centre
    (bias='real'), or ``given=(kbar2, c)``.  c = -R/(0.95 i) = i R / 0.95 with R the
    circle radius, so that max|v| = 0.95 and A = (laplacian + k^2)/c is accretive.
    Fourier symbol of L:  (-|p|^2 + kbar^2)/c  ->  s = 1/c, a0 = kbar^2, a2 = -1.
    """
    k2 = np.asarray(k2, dtype=np.complex128)
    if given is not None:
        kbar2, c = complex(given[0]), complex(given[1])
    else:
        if bias == "complex":
            kbar2, R = smallest_circle(k2)
        elif bias == "real":
            kbar2, R = smallest_real_centre(k2)
        else:
            raise ValueError(bias)
        if R <= 0.0:
            raise ValueError("homogeneous medium: pass given=(kbar2, c)")
        c = -R / (vnorm * 1j)
    v = (k2 - kbar2) / c
    y = -np.asarray(source, dtype=np.complex128) / c
    return Canonical(shape=k2.shape, spacing=tuple(spacing), s=1.0 / c, a0=kbar2, a1=0.0, a2=-1.0,
                     v=v, y=y, c=c, bias=kbar2)


def canonical_diffusion(mu_a, D, omega_over_v, source, spacing, vnorm=VNORM):
    """Scalar frequency-domain diffusion with constant D (Sec. 3.2, Eq. diffusion with
    D constant and e^{-i omega t} time dependence).

    A0 = -D laplacian + mu_a(r) - i omega/v.  L0 = -D laplacian + mubar - i omega/v with
    mubar the centre of the smallest circle of the (real) mu_a values, i.e. the
    midrange; c = R/0.95 real positive.  Symbol: s = 1/c, a0 = mubar - i omega/v, a2 = D.
    """
    mu = np.asarray(mu_a, dtype=np.float64)
    mubar, R = smallest_circle(np.array([mu.min(), mu.max()], dtype=np.complex128))
    if R <= 0.0:
        raise ValueError("constant absorption: splitting is degenerate")
    c = R / vnorm
    v = (mu - mubar.real) / c + 0j
    y = np.asarray(source, dtype=np.complex128) / c
    return Canonical(shape=mu.shape, spacing=tuple(spacing), s=1.0 / c,
                     a0=mubar.real - 1j * omega_over_v, a1=0.0, a2=D, v=v.astype(np.complex128),
                     y=y, c=c, bias=mubar)


def pantograph_gather(n, lam, t0, h):
    """Linear-interpolation gather  (S x)_j = x(lam t_j)  on t_j = t0 + j h.

    Entries whose argument lam t_j lies before t0 (initial condition, moved to the
    source) or beyond the last sample are zero.  Returns (index, w0, w1) with
    (S x)_j = w0_j x[idx_j] + w1_j x[idx_j + 1].
    """
    t = t0 + h * np.arange(n)
    pos = (lam * t - t0) / h
    idx = np.zeros(n, dtype=np.int64)
    w0 = np.zeros(n)
    w1 = np.zeros(n)
    for j in range(n):
        p = pos[j]
        if p < -1e-9 or p > n - 1 + 1e-9:
            continue
        i0 = int(math.floor(p + 1e-9))
        f = p - i0
        if abs(f) < 1e-9:
            f = 0.0
        if i0 >= n - 1:
            i0, f = n - 1, 0.0
        idx[j] = i0
        w0[j] = 1.0 - f
        w1[j] = f
        if i0 + 1 >= n:
            idx[j] = n - 2
            w0[j], w1[j] = 0.0, 1.0
    return idx, w0, w1


def gather_matrix(n, idx, w0, w1):
    S = np.zeros((n, n))
    for j in range(n):
        if w0[j] != 0.0:
            S[j, idx[j]] += w0[j]
        if w1[j] != 0.0:
            S[j, idx[j] + 1] += w1[j]
    return S


def canonical_pantograph(a, b, lam, t0, h, x0_at_lam_t, x0_t0, vnorm=VNORM, nyquist_zero=True):
    """Pantograph splitting (Sec. 3.3, Eq. pantograph-A).

    A x = c^-1 [(d/dt + a) x + b x(lam t)],  y = c^-1 [b x0(lam t) + x0(t0) delta(t - t0)].
    L0 = d/dt + abar, abar the smallest-circle centre of {a(t)}; the delta is sampled
    as x0(t0)/h at t0.  The paper's scale c = (sup|a - abar| + sup|b|)/0.95 bounds
    ||V|| only if the dilation gather has norm <= 1; for the discrete linear
    interpolation gather its spectral norm ||S|| exceeds 1 when lam < 1, so the
    scale used is c = (sup|a - abar| + sup|b| ||S||_2)/0.95, which restores ||V|| <= 0.95.
    Symbol: s = 1/c, a0 = abar, a1 = 1 (l(p) = (i p + abar)/c).  With nyquist_zero the
    Nyquist mode of i p is 0 (the direct form; it keeps real signals real); without it
    p = -pi/h there, which the antisymmetrised form needs: F^-1 diag(i p) F is
    skew-Hermitian for any real p, while a zero derivative at the Nyquist index
    leaves the alternating grid vector almost in the null space of A (the
    interpolation gather nearly annihilates it), which stalls the iteration.
    """
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    n = a.shape[0]
    abar, Ra = smallest_circle(a)
    idx, w0, w1 = pantograph_gather(n, lam, t0, h)
    S = gather_matrix(n, idx, w0, w1)
    snorm = float(np.linalg.norm(S, 2))
    c = (Ra + float(np.max(np.abs(b))) * snorm) / vnorm
    v = (a - abar) / c
    y = np.asarray(x0_at_lam_t, dtype=np.complex128) * b / c
    y = y.copy()
    y[0] += x0_t0 / h / c
    g0 = (b * w0) / c
    g1 = (b * w1) / c
    return Canonical(shape=(n,), spacing=(h,), s=1.0 / c, a0=abar, a1=1.0, a2=0.0, v=v, y=y, c=c,
                     bias=abar, gi=idx, g0=g0.astype(np.complex128), g1=g1.astype(np.complex128),
                     nyquist_zero=bool(nyquist_zero), extra={"gather_norm": snorm})
