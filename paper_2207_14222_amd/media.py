"""Seeded synthetic inputs: media, coefficients and sources.

This module only builds problem *inputs* (refractive-index maps, absorption
maps, ODE coefficients, sources) with the shapes and value ranges of the
paper's workloads.  It contains none of the solver's arithmetic (no bias,
scaling, splitting, symbol or iteration): both the FP64 oracle and the HIP
path receive the arrays produced here and canonicalise them independently.

Conventions
-----------
* Wavelength lambda = 1, so k0 = 2*pi; grid spacing h = lambda/4 (four points
  per wavelength) for every Helmholtz workload.
* Arrays are C-ordered, the last axis is the contiguous one ([z][y][x]).
* Absorbing layers: the imaginary part of the refractive index ramps linearly
  from 0 inside to ``kappa_max`` at the outermost pixel of every face
  (pixel j counted from the face gets kappa_max*(W-j)/W); axes combine by max.
  This is the boundary treatment the Helmholtz section describes: absorbing
  layers added to the medium to suppress the periodic wrap-around.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage

K0 = 2.0 * math.pi          # vacuum wavenumber for lambda = 1
H_WAVE = 0.25               # lambda / 4

__all__ = [
    "HelmholtzProblem", "DiffusionProblem", "PantographProblem",
    "absorbing_kappa", "helmholtz_1d", "helmholtz_spheres", "sphere_index", "beam_source", "helmholtz_disks",
    "helmholtz_homogeneous", "diffusion_blobs", "pantograph", "pantograph_constant", "batch_sizes", "FluxDiffusionProblem", "diffusion_ring",
]


@dataclass
class HelmholtzProblem:
    """Inputs of  laplacian(psi) + k^2 psi = -S  on a periodic grid."""
    k2: np.ndarray            # complex128, k0^2 (n + i kappa)^2
    source: np.ndarray        # complex128, S
    spacing: tuple            # grid spacing per axis
    index: np.ndarray = field(repr=False, default=None)  # complex refractive index n + i kappa

    @property
    def shape(self):
        return self.k2.shape


@dataclass
class DiffusionProblem:
    """Inputs of  -D laplacian(u) + mu_a u - i (omega/v) u = S  (e^{-i omega t})."""
    mu_a: np.ndarray          # float64 absorption coefficient [1/cm]
    D: float                  # diffusion constant [cm]
    omega_over_v: float       # [1/cm]
    source: np.ndarray        # complex128
    spacing: tuple

    @property
    def shape(self):
        return self.mu_a.shape


@dataclass
class PantographProblem:
    """Inputs of  -x'(t) = a(t) x(t) + b(t) x(lam t)  for t >= t0,  x = x0 before t0.

    Sampled on t_j = t0 + j h, j = 0..N-1.  ``x0_at_lam_t`` holds x0(lam t_j)
    where lam t_j < t0 (zero elsewhere) and ``x0_t0`` is x0(t0).
    """
    a: np.ndarray             # complex128 (N,)
    b: np.ndarray             # complex128 (N,)
    lam: float
    t0: float
    h: float
    x0_at_lam_t: np.ndarray   # complex128 (N,)
    x0_t0: complex

    @property
    def n(self):
        return self.a.shape[0]


def absorbing_kappa(shape, width, kappa_max=0.2):
    """Imaginary refractive index of the absorbing layers (max over axes)."""
    kappa = np.zeros(shape, dtype=np.float64)
    if width <= 0:
        return kappa
    for ax, n in enumerate(shape):
        ramp = np.zeros(n)
        j = np.arange(min(width, n))
        ramp[j] = kappa_max * (width - j) / width
        jr = np.arange(min(width, n))
        ramp[n - 1 - jr] = np.maximum(ramp[n - 1 - jr], kappa_max * (width - jr) / width)
        sh = [1] * len(shape)
        sh[ax] = n
        kappa = np.maximum(kappa, ramp.reshape(sh))
    return kappa


def _k2_from_index(nidx):
    return (K0 * nidx) ** 2


def helmholtz_1d(n=256, seed=1, width=32, kappa_max=0.2, sigma=4.0):
    """1-D random medium: n = 1 + 0.5 g, g smoothed uniform noise scaled to [0, 1].

    Unit point source at the centre, ``width``-pixel absorbing ramps at both ends.
    """
    rng = np.random.default_rng(seed)
    g = ndimage.gaussian_filter1d(rng.random(n), sigma, mode="reflect", truncate=4.0)
    g = (g - g.min()) / max(g.max() - g.min(), 1e-300)
    nre = np.clip(1.0 + 0.5 * g, 1.0, 1.5)
    nidx = nre + 1j * absorbing_kappa((n,), width, kappa_max)
    src = np.zeros(n, dtype=np.complex128)
    src[n // 2] = 1.0
    return HelmholtzProblem(k2=_k2_from_index(nidx), source=src, spacing=(H_WAVE,), index=nidx)


def _paint_balls(nre, count, rng, rmin=2.0, rmax=12.0, nmin=1.33, nmax=1.5):
    """Paint ``count`` balls (spheres in 3-D, disks in 2-D) in order; later ones overwrite."""
    shape = nre.shape
    d = len(shape)
    centres = rng.random((count, d)) * np.asarray(shape, dtype=np.float64)
    radii = rng.uniform(rmin, rmax, count)
    values = rng.uniform(nmin, nmax, count)
    for c, r, v in zip(centres, radii, values):
        lo = [max(int(math.floor(c[a] - r)), 0) for a in range(d)]
        hi = [min(int(math.ceil(c[a] + r)) + 1, shape[a]) for a in range(d)]
        if any(h <= l for l, h in zip(lo, hi)):
            continue
        grids = np.ix_(*[np.arange(lo[a], hi[a]) + 0.0 for a in range(d)])
        r2 = sum((grids[a] - c[a]) ** 2 for a in range(d))
        sl = tuple(slice(lo[a], hi[a]) for a in range(d))
        sub = nre[sl]
        sub[r2 <= r * r] = v
    return nre


def _beam_source(shape, plane, w0):
    """Gaussian beam (flat phase) on index ``plane`` of axis 0, centred in the other axes."""
    src = np.zeros(shape, dtype=np.complex128)
    rest = shape[1:]
    grids = np.ix_(*[np.arange(n) - n / 2 for n in rest])
    r2 = sum(g ** 2 for g in grids)
    src[plane] = np.exp(-r2 / (w0 * w0))
    return src


def sphere_index(shape=(256, 256, 256), seed=2, count=200, background=1.33):
    """Real refractive index of the random-sphere medium (no absorbing layers):
    background n with ``count`` spheres of radius 2-12 px and n uniform in [1.33, 1.5]."""
    rng = np.random.default_rng(seed)
    nre = np.full(shape, background, dtype=np.float64)
    return _paint_balls(nre, count, rng)


def beam_source(shape, plane=20, w0=16.0):
    """Gaussian-beam source on index ``plane`` of axis 0 (clamped to the grid)."""
    return _beam_source(shape, min(plane, shape[0] - 1), w0)


def helmholtz_spheres(shape=(256, 256, 256), seed=2, count=200, width=16,
                      kappa_max=0.2, w0=16.0, plane=20, background=1.33):
    """3-D medium: background n=1.33 with ``count`` random spheres (radius 2-12 px,
    n uniform in [1.33, 1.5]), absorbing faces, Gaussian-beam source on z = ``plane``."""
    nre = sphere_index(shape, seed, count, background)
    nidx = nre + 1j * absorbing_kappa(shape, width, kappa_max)
    return HelmholtzProblem(k2=_k2_from_index(nidx), source=beam_source(shape, plane, w0),
                            spacing=(H_WAVE,) * len(shape), index=nidx)


def helmholtz_disks(n=256, seed=4000, count=None, width=16, kappa_max=0.2, w0=16.0, row=20):
    """2-D medium of random disks; disk count keeps the 200-per-256^2 density."""
    if count is None:
        count = int(round(200 * (n / 256.0) ** 2))
    rng = np.random.default_rng(seed)
    nre = np.full((n, n), 1.33, dtype=np.float64)
    _paint_balls(nre, count, rng)
    nidx = nre + 1j * absorbing_kappa((n, n), width, kappa_max)
    return HelmholtzProblem(k2=_k2_from_index(nidx), source=_beam_source((n, n), min(row, n - 1), w0),
                            spacing=(H_WAVE, H_WAVE), index=nidx)


def helmholtz_homogeneous(shape, nidx=1.0 + 0.02j, source="point"):
    """Homogeneous (optionally absorbing) medium with a point source at the centre."""
    idx = np.full(shape, nidx, dtype=np.complex128)
    src = np.zeros(shape, dtype=np.complex128)
    src[tuple(n // 2 for n in shape)] = 1.0
    return HelmholtzProblem(k2=_k2_from_index(idx), source=src, spacing=(H_WAVE,) * len(shape), index=idx)


@dataclass
class FluxDiffusionProblem:
    """Inputs of the steady diffusion equation in flux form, div J + mu u = S,
    D^-1 J + grad u = 0, on a 2-D grid (axis 1 = x, axis 0 = y)."""
    mu: np.ndarray            # complex128 (n0, n1) absorption rate
    D: np.ndarray             # complex128 (n0, n1, 2, 2) diffusion tensor [[Dxx, Dxy], [Dyx, Dyy]]
    source: np.ndarray        # complex128 (n0, n1)
    h: float


def diffusion_ring(n=256, h=0.1, D_bg=2.0, D_t=25.0, D_r=1.0, radius=7.0, width=2.0, mu_bg=0.01,
                   mu_abs=20.0, abs_rows=16, src_row=8):
    """Anisotropic diffusion: a ring (radius and width in the units of h) where D is
    D_t along the tangent and D_r along the radius, D_bg elsewhere; absorption mu_bg
    with an absorbing layer ramping to mu_abs over the last abs_rows rows; a unit point
    source on row src_row at the centre column."""
    c = (np.arange(n) - n / 2) * h
    yy, xx = np.meshgrid(c, c, indexing="ij")
    r = np.hypot(xx, yy)
    D = np.zeros((n, n, 2, 2), dtype=np.complex128)
    D[..., 0, 0] = D_bg
    D[..., 1, 1] = D_bg
    ring = np.abs(r - radius) < width / 2
    rx, ry = xx[ring] / r[ring], yy[ring] / r[ring]          # radial unit vector; tangent (-ry, rx)
    D[ring, 0, 0] = D_t * ry * ry + D_r * rx * rx
    D[ring, 0, 1] = -D_t * ry * rx + D_r * rx * ry
    D[ring, 1, 0] = D[ring, 0, 1]
    D[ring, 1, 1] = D_t * rx * rx + D_r * ry * ry
    mu = np.full((n, n), mu_bg, dtype=np.complex128)
    for i in range(abs_rows):
        mu[n - abs_rows + i, :] = mu_bg + mu_abs * (i + 1) / abs_rows
    src = np.zeros((n, n), dtype=np.complex128)
    src[src_row, n // 2] = 1.0
    return FluxDiffusionProblem(mu=mu, D=D, source=src, h=float(h))


def diffusion_tensor_random(shape=(32, 128), seed=7, h=0.25, d_lo=0.5, d_hi=5.0, mu_lo=0.05, mu_hi=1.0,
                            smooth=3.0):
    """Random anisotropic medium on an (n0, n1) grid: per voxel D = R(theta) diag(d1, d2) R(theta)^T
    with d1, d2 log-uniform in [d_lo, d_hi] and theta uniform, all three fields smoothed
    (periodic Gaussian of `smooth` voxels) before mapping; absorption mu in [mu_lo, mu_hi] the
    same way; a complex Gaussian random source."""
    rng = np.random.default_rng(seed)
    n0, n1 = shape

    def field():
        g = rng.normal(size=shape)
        k0 = np.fft.fftfreq(n0)[:, None]
        k1 = np.fft.fftfreq(n1)[None, :]
        g = np.real(np.fft.ifft2(np.fft.fft2(g) * np.exp(-2 * (np.pi * smooth) ** 2 * (k0 ** 2 + k1 ** 2))))
        g = (g - g.mean()) / (g.std() + 1e-300)
        return 0.5 * (1.0 + np.tanh(g))          # in (0, 1)

    d1 = d_lo * (d_hi / d_lo) ** field()
    d2 = d_lo * (d_hi / d_lo) ** field()
    th = np.pi * field()
    c, s = np.cos(th), np.sin(th)
    D = np.zeros((n0, n1, 2, 2), dtype=np.complex128)
    D[..., 0, 0] = d1 * c * c + d2 * s * s
    D[..., 0, 1] = (d1 - d2) * c * s
    D[..., 1, 0] = D[..., 0, 1]
    D[..., 1, 1] = d1 * s * s + d2 * c * c
    mu = (mu_lo + (mu_hi - mu_lo) * field()).astype(np.complex128)
    src = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    return FluxDiffusionProblem(mu=mu, D=D, source=src, h=float(h))


def double_ring_well(n=512, box=6.0, depth=10.0, diameter=2.0, width=0.2, gap=0.1):
    """Potential well of two rings side by side (the eigenmode example): V = -depth on
    two annuli of the given diameter and width whose outer edges are `gap` apart along
    axis 1, 0 elsewhere, on an n x n grid covering [-box/2, box/2)^2.  Returns (V, h)."""
    h = box / n
    c = (np.arange(n) - n / 2) * h
    yy, xx = np.meshgrid(c, c, indexing="ij")
    R = 0.5 * diameter
    off = R + 0.5 * width + 0.5 * gap
    V = np.zeros((n, n))
    for sx in (-1.0, 1.0):
        r = np.hypot(xx - sx * off, yy)
        V[np.abs(r - R) < 0.5 * width] = -depth
    return V, h


def harmonic_well(n=40, h=0.45, omega=1.0, omega_y=None):
    """V = (omega^2 x^2 + omega_y^2 y^2) / 2 about the grid centre on an n x n grid
    (omega_y = omega unless given; x is axis 1).  Returns (V, h)."""
    wy = omega if omega_y is None else omega_y
    c = (np.arange(n) - n / 2) * h
    yy, xx = np.meshgrid(c, c, indexing="ij")
    return 0.5 * (omega ** 2 * xx ** 2 + wy ** 2 * yy ** 2), h


def random_start(shape, seed=0):
    """Seeded complex Gaussian start vector."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def diffusion_tensor_random3(shape=(8, 16, 32), seed=11, h=0.3, d_lo=0.5, mu_lo=0.05, mu_hi=1.0, smooth=2.0):
    """Random anisotropic 3-D medium: per voxel D = G G^T / 3 + d_lo I (symmetric
    positive definite, x, y, z order) with the nine entries of G smooth standardised
    noise (periodic Gaussian of `smooth` voxels); absorption mu in [mu_lo, mu_hi]
    from another such field mapped through tanh; a complex Gaussian random source."""
    rng = np.random.default_rng(seed)
    ks = np.meshgrid(*[np.fft.fftfreq(n) for n in shape], indexing="ij")
    filt = np.exp(-2 * (np.pi * smooth) ** 2 * sum(k ** 2 for k in ks))

    def field():
        g = np.real(np.fft.ifftn(np.fft.fftn(rng.normal(size=shape)) * filt))
        return (g - g.mean()) / (g.std() + 1e-300)

    G = np.stack([np.stack([field() for _ in range(3)], axis=-1) for _ in range(3)], axis=-2)
    D = (np.einsum("...ab,...cb->...ac", G, G) / 3.0 + d_lo * np.eye(3)).astype(np.complex128)
    mu = (mu_lo + (mu_hi - mu_lo) * 0.5 * (1.0 + np.tanh(field()))).astype(np.complex128)
    src = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    return FluxDiffusionProblem(mu=mu, D=D, source=src, h=float(h))


def batch_sizes(nprob=96, seed=4, choices=(128, 256, 512, 1024)):
    """Side lengths of the batched 2-D problems, drawn uniformly from ``choices``."""
    rng = np.random.default_rng(seed)
    return [int(c) for c in rng.choice(np.asarray(choices), size=nprob)]


def diffusion_blobs(shape=(128, 256, 256), seed=3, D=0.03, freq_hz=1e8, n_tissue=1.4,
                    h=0.05, sigma=8.0, mua_min=0.01, mua_max=0.1):
    """Frequency-domain diffusion medium: constant D, log-normal absorption blobs.

    g = white N(0,1) noise smoothed with a Gaussian (sigma voxels, periodic) and
    standardised; mu_a = clip(sqrt(min*max) * 10^(g/4), min, max).  Unit point source
    at the centre of the top face (z = 0).
    """
    rng = np.random.default_rng(seed)
    g = ndimage.gaussian_filter(rng.standard_normal(shape), sigma, mode="wrap", truncate=4.0)
    g = (g - g.mean()) / g.std()
    mua = np.clip(math.sqrt(mua_min * mua_max) * np.exp(g * math.log(10.0) / 4.0), mua_min, mua_max)
    v = 2.99792458e10 / n_tissue
    src = np.zeros(shape, dtype=np.complex128)
    src[(0,) + tuple(n // 2 for n in shape[1:])] = 1.0
    return DiffusionProblem(mu_a=mua, D=D, omega_over_v=2.0 * math.pi * freq_hz / v,
                            source=src, spacing=(h,) * len(shape))


def pantograph_constant(n=1024, lam=0.9, a_value=0.1, b_value=-5.0, h=0.01, t0=1.0):
    """Pantograph with constant coefficients (a non-accretive case for lam = 0.9,
    a = 0.1, b = -5); x0(t) = exp(-50 (t-1)^2) before t0."""
    t = t0 + h * np.arange(n)
    a = np.full(n, a_value, dtype=np.complex128)
    b = np.full(n, b_value, dtype=np.complex128)
    lt = lam * t
    x0l = np.where(lt < t0, np.exp(-50.0 * (lt - 1.0) ** 2), 0.0).astype(np.complex128)
    return PantographProblem(a=a, b=b, lam=lam, t0=t0, h=h, x0_at_lam_t=x0l,
                             x0_t0=complex(np.exp(-50.0 * (t0 - 1.0) ** 2)))


def pantograph(n=1024, lam=0.5, b_value=5.0, h=0.01, t0=1.0):
    """Pantograph workload: a = 5 on [1, 6] s and 5 - 10i after; b = b_value except
    b = 0 on [3, 5] s; x0(t) = exp(-50 (t-1)^2) before t0."""
    t = t0 + h * np.arange(n)
    a = np.where(t <= 6.0, 5.0 + 0j, 5.0 - 10.0j).astype(np.complex128)
    b = np.where((t >= 3.0) & (t <= 5.0), 0.0, b_value).astype(np.complex128)
    lt = lam * t
    x0l = np.where(lt < t0, np.exp(-50.0 * (lt - 1.0) ** 2), 0.0).astype(np.complex128)
    return PantographProblem(a=a, b=b, lam=lam, t0=t0, h=h, x0_at_lam_t=x0l,
                             x0_t0=complex(np.exp(-50.0 * (t0 - 1.0) ** 2)))
