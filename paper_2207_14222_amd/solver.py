"""Thin Python layer over the C ABI (``include/usp.h``): argument marshalling only.

PyTorch provides device memory (tensors) and the stream; every arithmetic step
of canonicalisation (host C++ in the library + a device kernel) and of the
iteration (HIP kernels) runs in ``libusp.so``.
"""
from __future__ import annotations

import ctypes as ct
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import _lib as L

__all__ = ["Operator", "FluxOperator", "canonical_flux_host", "canonical_schrodinger", "EigResult", "hermitian_eig", "SolveResult", "make_symbol", "smallest_circle", "canonical_helmholtz",
           "canonical_diffusion", "canonical_pantograph", "canonical_fields"]


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _stream_ptr(device) -> ct.c_void_p:
    return ct.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _c2(z) -> tuple:
    z = complex(z)
    return (z.real, z.imag)


def make_symbol(shape, spacing, s=1.0, a0=0.0, a1=0.0, a2=0.0, nyquist_zero=False) -> L.usp_symbol:
    """usp_symbol for l(p) = s (a0 + a2 |p|^2 + a1 i p) on a grid of ``shape``."""
    sym = L.usp_symbol()
    sym.ndim = len(shape)
    for i, n in enumerate(shape):
        sym.shape[i] = int(n)
        sym.spacing[i] = float(spacing[i])
    sym.s[:] = _c2(s)
    sym.a0[:] = _c2(a0)
    sym.a1[:] = _c2(a1)
    sym.a2[:] = _c2(a2)
    sym.nyquist_zero = int(bool(nyquist_zero))
    return sym


def symbol_coeffs(sym: L.usp_symbol) -> dict:
    return {k: complex(getattr(sym, k)[0], getattr(sym, k)[1]) for k in ("s", "a0", "a1", "a2")}


def smallest_circle(points, kind: str = "complex"):
    """usp_smallest_circle on host points; returns (centre, radius)."""
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.complex128).ravel()).view(np.float64)
    centre = np.zeros(2)
    radius = np.zeros(1)
    k = L.USP_BIAS_COMPLEX if kind == "complex" else L.USP_BIAS_REAL
    L.check(L.lib().usp_smallest_circle(_dp(pts), pts.size // 2, k, _dp(centre), _dp(radius)))
    return complex(centre[0], centre[1]), float(radius[0])


def canonical_fields(q: torch.Tensor, S: torch.Tensor, bias, c, src_scale: float, dtype) -> tuple:
    """B = 1 - (q - bias)/c and y = src_scale S / c on the device (usp_canonical_fields)."""
    dev = q.device
    n = q.numel()
    B = torch.empty(q.shape, dtype=dtype, device=dev)
    y = torch.empty(q.shape, dtype=dtype, device=dev)
    dt = L.USP_C64 if dtype == torch.complex64 else L.USP_C128
    b = np.array(_c2(bias))
    cc = np.array(_c2(c))
    L.check(L.lib().usp_canonical_fields(_ptr(q), _ptr(S), n, _dp(b), _dp(cc), float(src_scale), dt, _ptr(B),
                                         _ptr(y), _stream_ptr(dev)))
    return B, y


@dataclass
class Canonical:
    symbol: L.usp_symbol
    B: torch.Tensor
    y: torch.Tensor
    c: complex
    bias: complex


def canonical_helmholtz(k2, source, spacing, bias: str = "complex", given=None, vnorm: float = 0.95,
                        dtype=torch.complex64, device="cuda") -> Canonical:
    """Helmholtz canonical form (usp_canonical_helmholtz + usp_canonical_fields)."""
    k2n = np.ascontiguousarray(np.asarray(k2, dtype=np.complex128))
    shape = k2n.shape
    grid = make_symbol(shape, spacing)
    out = L.usp_symbol()
    c = np.zeros(2)
    b = np.zeros(2)
    g = None if given is None else np.array(_c2(given[0]) + _c2(given[1]))
    kind = L.USP_BIAS_COMPLEX if bias == "complex" else L.USP_BIAS_REAL
    flat = k2n.ravel().view(np.float64)
    L.check(L.lib().usp_canonical_helmholtz(_dp(flat), k2n.size, kind, None if g is None else _dp(g), vnorm,
                                            ct.byref(grid), ct.byref(out), _dp(c), _dp(b)))
    q = torch.from_numpy(k2n).to(device)
    S = torch.from_numpy(np.ascontiguousarray(np.asarray(source, dtype=np.complex128))).to(device)
    Bt, yt = canonical_fields(q, S, complex(b[0], b[1]), complex(c[0], c[1]), -1.0, dtype)
    return Canonical(out, Bt, yt, complex(c[0], c[1]), complex(b[0], b[1]))


def helmholtz_symbol(shape, spacing, bias, c) -> L.usp_symbol:
    """Symbol l(p) = (kbar^2 - |p|^2)/c of the Helmholtz canonical form for a given
    bias kbar^2 and scale c (usp_canonical_helmholtz with both given)."""
    grid = make_symbol(shape, spacing)
    out = L.usp_symbol()
    cc, b = np.zeros(2), np.zeros(2)
    g = np.array(_c2(bias) + _c2(c))
    L.check(L.lib().usp_canonical_helmholtz(None, 0, L.USP_BIAS_COMPLEX, _dp(g), 0.95, ct.byref(grid), ct.byref(out),
                                            _dp(cc), _dp(b)))
    return out


def canonical_diffusion(mu_a, D, omega_over_v, source, spacing, vnorm: float = 0.95, dtype=torch.complex64,
                        device="cuda") -> Canonical:
    """Constant-D diffusion canonical form (usp_canonical_diffusion + usp_canonical_fields)."""
    mu = np.ascontiguousarray(np.asarray(mu_a, dtype=np.float64))
    grid = make_symbol(mu.shape, spacing)
    out = L.usp_symbol()
    c = np.zeros(2)
    b = np.zeros(2)
    L.check(L.lib().usp_canonical_diffusion(_dp(mu.ravel()), mu.size, float(D), float(omega_over_v), vnorm,
                                            ct.byref(grid), ct.byref(out), _dp(c), _dp(b)))
    q = torch.from_numpy(mu.astype(np.complex128)).to(device)
    S = torch.from_numpy(np.ascontiguousarray(np.asarray(source, dtype=np.complex128))).to(device)
    Bt, yt = canonical_fields(q, S, complex(b[0], b[1]), complex(c[0], c[1]), 1.0, dtype)
    return Canonical(out, Bt, yt, complex(c[0], c[1]), complex(b[0], b[1]))


def canonical_schrodinger(V, spacing, shift, vnorm: float = 0.95, dtype=torch.complex128,
                          device="cuda") -> Canonical:
    """H + shift = -1/2 laplacian + V + shift as the constant-D operator with D = 1/2,
    mu = V + shift, omega = 0 (Sec. 4, Eq. schrodinger; usp_canonical_schrodinger +
    usp_canonical_fields on V); energies E = c lam - shift."""
    Vn = np.ascontiguousarray(np.asarray(V, dtype=np.float64))
    grid = make_symbol(Vn.shape, spacing)
    out = L.usp_symbol()
    c = np.zeros(2)
    b = np.zeros(2)
    L.check(L.lib().usp_canonical_schrodinger(_dp(Vn.ravel()), Vn.size, float(shift), vnorm, ct.byref(grid),
                                              ct.byref(out), _dp(c), _dp(b)))
    q = torch.from_numpy(Vn.astype(np.complex128)).to(device)
    S = torch.zeros(Vn.shape, dtype=torch.complex128, device=device)
    Bt, yt = canonical_fields(q, S, complex(b[0], b[1]), complex(c[0], c[1]), 1.0, dtype)
    return Canonical(out, Bt, yt, complex(c[0], c[1]), complex(b[0], b[1]))


@dataclass
class EigResult:
    evals: np.ndarray          # ascending eigenvalues of the canonical A
    evecs: torch.Tensor        # (nev,) + field shape, unit norm
    resid: np.ndarray          # ||A u - lam u|| / ||lam u||
    restarts: int
    inner_iterations: int      # CG iterations over all inner solves
    status: int

    @property
    def converged(self):
        return self.status == L.USP_OK


@dataclass
class CanonicalPantograph(Canonical):
    gather: tuple = None   # (idx int32, g0, g1) device tensors


def canonical_pantograph(a, b, lam, t0, h, x0_at_lam_t, x0_t0, vnorm: float = 0.95, dtype=torch.complex128,
                         device="cuda", nyquist_zero: bool = True) -> CanonicalPantograph:
    """Pantograph canonical form (usp_canonical_pantograph, host) uploaded to the device.
    nyquist_zero=False keeps the Nyquist mode of the derivative symbol (the choice the
    antisymmetrised form needs; the library returns it set)."""
    def c128(z):
        return np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    a, b, x0l = c128(a), c128(b), c128(x0_at_lam_t)
    n = a.shape[0]
    x0t = np.array(_c2(x0_t0))
    sym = L.usp_symbol()
    Bh = np.zeros(n, np.complex128)
    idx = np.zeros(n, np.int32)
    g0 = np.zeros(n, np.complex128)
    g1 = np.zeros(n, np.complex128)
    yh = np.zeros(n, np.complex128)
    c = np.zeros(2)
    bias = np.zeros(2)
    f = lambda z: _dp(z.view(np.float64))
    L.check(L.lib().usp_canonical_pantograph(f(a), f(b), n, float(lam), float(t0), float(h), f(x0l), _dp(x0t),
                                             float(vnorm), ct.byref(sym), f(Bh),
                                             idx.ctypes.data_as(ct.POINTER(ct.c_int32)), f(g0), f(g1), f(yh),
                                             _dp(c), _dp(bias)))
    sym.nyquist_zero = int(bool(nyquist_zero))
    T = lambda z: torch.from_numpy(z).to(device=device, dtype=dtype)
    return CanonicalPantograph(symbol=sym, B=T(Bh), y=T(yh), c=complex(c[0], c[1]), bias=complex(bias[0], bias[1]),
                               gather=(torch.from_numpy(idx).to(device), T(g0), T(g1)))


@dataclass
class SolveResult:
    x: torch.Tensor
    iterations: int
    status: int
    hist_pre: np.ndarray = field(repr=False, default=None)     # ||Delta_i||^2
    hist_true: np.ndarray = field(repr=False, default=None)    # (iteration, rho) rows

    @property
    def converged(self):
        return self.status == L.USP_OK

    @property
    def status_name(self):
        return L.STATUS_NAMES.get(self.status, str(self.status))


class Operator:
    """A prepared operator handle (usp_prepare_operator) with its workspace tensor."""

    def __init__(self, symbol: L.usp_symbol, B: torch.Tensor, refine: bool = False, gather=None,
                 antisym: bool = False):
        """antisym: solve the antisymmetrised system (1-D): fields are (2, N), [x~; x~']."""
        if not B.is_cuda:
            raise ValueError("B must be a device tensor")
        self.B = B
        self.device = B.device
        self.dtype = B.dtype
        self.dt = L.USP_C64 if B.dtype == torch.complex64 else L.USP_C128
        self.flags = (L.USP_FLAG_REFINE if refine else 0) | (L.USP_FLAG_ANTISYM if antisym else 0)
        self.field_shape = (2,) + tuple(B.shape) if antisym else tuple(B.shape)
        self.symbol = symbol
        self.gather = gather   # keep device arrays alive
        nbytes = ct.c_size_t()
        L.check(L.lib().usp_workspace_bytes(ct.byref(symbol), self.dt, self.flags, ct.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        g = None
        if gather is not None:
            idx, g0, g1 = gather
            g = L.usp_gather(idx.data_ptr(), g0.data_ptr(), g1.data_ptr())
        h = ct.c_void_p()
        L.check(L.lib().usp_prepare_operator(ct.byref(symbol), self.dt, self.flags, _ptr(B),
                                             None if g is None else ct.byref(g), _ptr(self.workspace),
                                             nbytes.value, _stream_ptr(self.device), ct.byref(h)))
        self.handle = h

    @property
    def shape(self):
        return self.field_shape

    def close(self):
        if getattr(self, "handle", None):
            L.lib().usp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _field(self, t):
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() or tuple(t.shape) != self.shape:
            raise ValueError(f"expected a contiguous {self.dtype} tensor of shape {self.shape} on {self.device}")
        return t

    def solve(self, y, x=None, alpha=0.8, tol=1e-6, maxit=10000, check_every=20, hist_cap=None,
              judge_guess=False) -> SolveResult:
        """usp_solve; with judge_guess the guess x is kept only if its residual is below ||y||
        (hist_true[0] is then the guess's relative residual)."""
        y = self._field(y)
        guess = x is not None
        x = self._field(x) if guess else torch.empty_like(y)
        hc = maxit if hist_cap is None else hist_cap
        hp = np.zeros(max(hc, 1))
        ntc = maxit // check_every + 2
        ht = np.zeros(2 * ntc)
        it = ct.c_int()
        nt = ct.c_int()
        rc = L.check(L.lib().usp_solve(self.handle, _ptr(y), _ptr(x), (2 if judge_guess else 1) if guess else 0,
                                       float(alpha), float(tol),
                                       int(maxit), int(check_every), ct.byref(it), _dp(hp), hc, _dp(ht), ntc,
                                       ct.byref(nt)))
        n = min(it.value, hc)
        m = min(nt.value, ntc)
        return SolveResult(x=x, iterations=it.value, status=rc, hist_pre=hp[:n].copy(),
                           hist_true=ht[:2 * m].reshape(m, 2).copy())

    def iterate(self, y, x=None, alpha=0.8, K=1):
        """Exactly K iterations (test hook); returns (x, ||Delta_i||^2 array)."""
        y = self._field(y)
        guess = x is not None
        x = self._field(x) if guess else torch.empty_like(y)
        hp = np.zeros(max(K, 1))
        L.check(L.lib().usp_iterate(self.handle, _ptr(y), _ptr(x), int(guess), float(alpha), int(K), _dp(hp), K))
        return x, hp[:K].copy()

    def profile(self, y, x, alpha=0.8, K=20):
        """Per-pass average launch time (ms) and per-iteration time (ms) via usp_profile."""
        pm = np.zeros(L.USP_NPASS)
        it = np.zeros(1)
        L.check(L.lib().usp_profile(self.handle, _ptr(self._field(y)), _ptr(self._field(x)), float(alpha), int(K),
                                    _dp(pm), _dp(it)))
        return dict(zip(L.PASS_NAMES, pm.tolist())), float(it[0])

    def get_plan(self) -> dict:
        p = L.usp_plan()
        L.check(L.lib().usp_get_plan(self.handle, ct.byref(p)))
        return {"x_prefetch": p.x_prefetch, "w_mid": p.w_mid, "w_sym": p.w_sym, "x_stream": p.x_stream,
                "r_load": p.r_load}

    def set_plan(self, x_prefetch=0, w_mid=0, w_sym=0, x_stream=0, r_load=0):
        p = L.usp_plan(int(x_prefetch), int(w_mid), int(w_sym), int(x_stream), int(r_load))
        L.check(L.lib().usp_set_plan(self.handle, ct.byref(p)))

    def autotune(self, y, x, alpha=0.8, reps=5) -> dict:
        """usp_autotune: pick the fastest launch plan (results are identical for all)."""
        p = L.usp_plan()
        L.check(L.lib().usp_autotune(self.handle, _ptr(self._field(y)), _ptr(self._field(x)), float(alpha),
                                     int(reps), ct.byref(p)))
        return {"x_prefetch": p.x_prefetch, "w_mid": p.w_mid, "w_sym": p.w_sym, "x_stream": p.x_stream,
                "r_load": p.r_load}

    def krylov(self, y, x=None, method="bicgstab", restart=20, tol=1e-6, maxit=10000, check_every=20,
               hist_cap=None) -> SolveResult:
        """usp_solve_krylov: BiCGSTAB or GMRES(restart) on the preconditioned system
        (workspace allocated here as a torch tensor).  hist_pre holds the method's
        squared residual estimates (see usp.h)."""
        y = self._field(y)
        guess = x is not None
        x = self._field(x) if guess else torch.empty_like(y)
        meth = {"bicgstab": L.USP_KRYLOV_BICGSTAB, "gmres": L.USP_KRYLOV_GMRES, "cg": L.USP_KRYLOV_CG}[method]
        nb = ct.c_size_t()
        L.check(L.lib().usp_krylov_workspace_bytes(self.handle, meth, int(restart), ct.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        hc = maxit if hist_cap is None else hist_cap
        hp = np.zeros(max(hc, 1))
        ntc = maxit + 2
        ht = np.zeros(2 * ntc)
        it, nt = ct.c_int(), ct.c_int()
        rc = L.check(L.lib().usp_solve_krylov(self.handle, meth, int(restart), _ptr(y), _ptr(x), int(guess),
                                              float(tol), int(maxit), int(check_every), _ptr(ws), nb.value,
                                              ct.byref(it), _dp(hp), hc, _dp(ht), ntc, ct.byref(nt)))
        m = min(nt.value, ntc)
        return SolveResult(x=x, iterations=it.value, status=rc, hist_pre=hp[:min(it.value, hc)].copy(),
                           hist_true=ht[:2 * m].reshape(m, 2).copy())

    def eigs(self, nev=5, ncv=32, v0=None, tol=1e-8, max_restarts=50, inner_tol=1e-11, inner_maxit=2000,
             seed=0) -> EigResult:
        """usp_eigs: the nev smallest eigenvalues of a Hermitian canonical A and their
        eigenvectors (shift-invert Lanczos, CG inner solves, thick restart)."""
        if v0 is None:
            g = torch.Generator(device="cpu").manual_seed(seed)
            v0 = torch.randn(self.shape, generator=g, dtype=torch.float64).to(self.dtype).to(self.device)
        v0 = self._field(v0)
        nb = ct.c_size_t()
        L.check(L.lib().usp_eigs_workspace_bytes(self.handle, int(nev), int(ncv), ct.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        evecs = torch.empty((nev,) + tuple(self.shape), dtype=self.dtype, device=self.device)
        ev = np.zeros(nev)
        rs = np.zeros(nev)
        nr, ni = ct.c_int(), ct.c_int()
        rc = L.check(L.lib().usp_eigs(self.handle, int(nev), int(ncv), _ptr(v0), float(tol), int(max_restarts),
                                      float(inner_tol), int(inner_maxit), _ptr(evecs), _dp(ev), _dp(rs), _ptr(ws),
                                      nb.value, ct.byref(nr), ct.byref(ni)))
        return EigResult(evals=ev, evecs=evecs, resid=rs, restarts=nr.value, inner_iterations=ni.value, status=rc)

    def apply_precond(self, v, rhs=False):
        """usp_apply_precond: P v, or b = B (L + I)^-1 v with rhs."""
        v = self._field(v)
        w = torch.empty_like(v)
        nb = ct.c_size_t()
        L.check(L.lib().usp_krylov_workspace_bytes(self.handle, L.USP_KRYLOV_BICGSTAB, 0, ct.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        L.check(L.lib().usp_apply_precond(self.handle, _ptr(v), _ptr(w), int(rhs), _ptr(ws), nb.value))
        return w

    def residual(self, y, x):
        """(||y - A x||/||y||, ||y - A x||, ||y||) in FP64."""
        rel, rn, yn = np.zeros(1), np.zeros(1), np.zeros(1)
        L.check(L.lib().usp_residual(self.handle, _ptr(self._field(y)), _ptr(self._field(x)), _dp(rel), _dp(rn),
                                     _dp(yn)))
        return float(rel[0]), float(rn[0]), float(yn[0])


def stream_copy(src: torch.Tensor, dst: torch.Tensor):
    """usp_stream_copy: dst <- src (same byte size, contiguous device tensors) with
    non-temporal loads and stores on the current stream (measurement hook)."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("contiguous device tensors expected")
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("src and dst must have the same size in bytes")
    L.check(L.lib().usp_stream_copy(_ptr(src), _ptr(dst), nb, _stream_ptr(src.device)))


def hermitian_eig(a):
    """usp_hermitian_eig (host): ascending eigenvalues and eigenvector columns of the
    Hermitian part of a square complex matrix."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    n = a.shape[0]
    w = np.zeros(n)
    z = np.zeros((n, n), np.complex128)
    L.check(L.lib().usp_hermitian_eig(n, _dp(a.view(np.float64)), _dp(w), _dp(z.view(np.float64))))
    return w, z


def canonical_flux_host(mu, D, source, h, vnorm: float = 0.95):
    """usp_canonical_flux (host) on a 2-D or 3-D grid: returns (usp_flux_symbol, bu (grid),
    b2 (grid + (d, d)), y ((1 + d,) + grid)); D in the (x, y[, z]) order of the flux
    components, x the contiguous axis."""
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.complex128))
    Dm = np.ascontiguousarray(np.asarray(D, dtype=np.complex128))
    src = np.ascontiguousarray(np.asarray(source, dtype=np.complex128))
    d = mu.ndim
    if d not in (2, 3) or Dm.shape != mu.shape + (d, d) or src.shape != mu.shape:
        raise ValueError("mu (grid), D (grid + (d, d)), source (grid) on a 2-D or 3-D grid")
    sym = L.usp_flux_symbol()
    bu = np.zeros(mu.shape, np.complex128)
    b2 = np.zeros(mu.shape + (d, d), np.complex128)
    y = np.zeros((1 + d,) + mu.shape, np.complex128)
    shape = (ct.c_int * 3)(*(list(mu.shape) + [1] * (3 - d)))
    f = lambda z: _dp(z.view(np.float64))
    L.check(L.lib().usp_canonical_flux(f(mu), f(Dm), f(src), d, shape, float(h), float(vnorm), ct.byref(sym),
                                       f(bu), f(b2), f(y)))
    return sym, bu, b2, y


class FluxOperator:
    """Steady diffusion in flux form with a tensor coefficient (usp_canonical_flux
    on the host, then usp_flux_solve / usp_flux_residual on the device), 2-D or
    3-D.  Fields are (1 + d,) + grid tensors: [u; Jx; Jy (; Jz)] of the
    canonical system."""

    def __init__(self, mu, D, source, h, vnorm: float = 0.95, dtype=torch.complex128, device="cuda",
                 refine: bool = False):
        if refine and dtype != torch.complex128:
            raise ValueError("refine=True needs complex128 fields")
        self.sym, bu, b2, y = canonical_flux_host(mu, D, source, h, vnorm)
        self.device = torch.device(device)
        self.dtype = dtype
        self.refine = refine
        self.dt = L.USP_C64 if dtype == torch.complex64 else L.USP_C128
        T = lambda z: torch.from_numpy(z).to(device=self.device, dtype=dtype)
        self.bu, self.b2, self.y = T(bu), T(b2), T(y)
        self.device = self.y.device          # "cuda" resolved to "cuda:<index>"
        self.shape = tuple(y.shape)
        nb = ct.c_size_t()
        if refine:
            L.check(L.lib().usp_flux_refined_workspace_bytes(ct.byref(self.sym), ct.byref(nb)))
        else:
            L.check(L.lib().usp_flux_workspace_bytes(ct.byref(self.sym), self.dt, ct.byref(nb)))
        self.ws_bytes = nb.value
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)

    @property
    def s(self):
        return np.array(self.sym.s[:self.sym.ndim + 1])

    @property
    def c(self):
        return float(self.sym.c)

    def _field(self, t):
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() or tuple(t.shape) != self.shape:
            raise ValueError(f"expected a contiguous {self.dtype} tensor of shape {self.shape} on {self.device}")
        return t

    def solve(self, y=None, x=None, alpha=1.0, tol=1e-6, maxit=10000, check_every=20, judge_guess=False) -> SolveResult:
        """Algorithm 1; with refine=True, check_every is the refinement interval
        (complex64 inner iterations, FP64 residual and update every cycle) and
        judge_guess discards a guess whose residual is not below ||y||."""
        y = self.y if y is None else self._field(y)
        guess = x is not None
        x = self._field(x) if guess else torch.empty_like(y)
        hp = np.zeros(max(maxit, 1))
        ntc = maxit + 2 if self.refine else maxit // check_every + 2
        ht = np.zeros(2 * ntc)
        it, nt = ct.c_int(), ct.c_int()
        g = (2 if judge_guess else 1) if guess else 0
        if self.refine:
            rc = L.check(L.lib().usp_flux_solve_refined(
                ct.byref(self.sym), _ptr(self.bu), _ptr(self.b2), _ptr(y), _ptr(x), g, float(alpha), float(tol),
                int(maxit), int(check_every), _ptr(self.workspace), self.ws_bytes, _stream_ptr(self.device),
                ct.byref(it), _dp(hp), maxit, _dp(ht), ntc, ct.byref(nt)))
        else:
            rc = L.check(L.lib().usp_flux_solve(ct.byref(self.sym), self.dt, _ptr(self.bu), _ptr(self.b2), _ptr(y),
                                                _ptr(x), g, float(alpha), float(tol), int(maxit),
                                                int(check_every), _ptr(self.workspace), self.ws_bytes,
                                                _stream_ptr(self.device), ct.byref(it), _dp(hp), maxit, _dp(ht), ntc,
                                                ct.byref(nt)))
        m = min(nt.value, ntc)
        return SolveResult(x=x, iterations=it.value, status=rc, hist_pre=hp[:min(it.value, maxit)].copy(),
                           hist_true=ht[:2 * m].reshape(m, 2).copy())

    def iterate(self, y=None, x=None, alpha=1.0, K=1):
        """Exactly K iterations (no early stop); returns (x, ||Delta_i||^2 array)."""
        r = self.solve(y, x, alpha=alpha, tol=-1.0, maxit=K, check_every=max(K, 1))
        return r.x, r.hist_pre

    def residual(self, x, y=None) -> float:
        """FP64 ||y - A x|| / ||y||."""
        y = self.y if y is None else self._field(y)
        rel = np.zeros(1)
        L.check(L.lib().usp_flux_residual(ct.byref(self.sym), self.dt, _ptr(self.bu), _ptr(self.b2), _ptr(y),
                                          _ptr(self._field(x)), _ptr(self.workspace), self.ws_bytes,
                                          _stream_ptr(self.device), _dp(rel)))
        return float(rel[0])

    def physical(self, x):
        """[u; Jx; Jy] = S x / sqrt(c)."""
        s = torch.tensor(self.s, dtype=torch.float64, device=x.device).to(x.real.dtype)
        return x * (s.reshape((-1,) + (1,) * (x.dim() - 1)) / np.sqrt(self.c))


@dataclass
class BatchResult:
    iterations: list
    status: list
    rho: list
    t_done_ms: list
    elapsed_ms: float
    worst: int


class Batch:
    """Many independent square 2-D refined problems solved together (usp_solve_batched).
    ops: refined Operators; ys / xs: complex128 tensors.  variant: bits 0-1 fused-pass
    plan, bit 2 persistent one-launch schedule (else grouped launches), bit 3 narrow
    column tiles of the grouped schedule."""

    def __init__(self, ops, ys, xs, alpha=0.8, tol=1e-6, maxit=20000):
        if not (len(ops) == len(ys) == len(xs)) or not ops:
            raise ValueError("ops, ys, xs must have the same non-zero length")
        for op, y, x in zip(ops, ys, xs):
            if not op.flags & L.USP_FLAG_REFINE or op.dtype != torch.complex128:
                raise ValueError("batched problems need refined complex128 operators")
            op._field(y)
            op._field(x)
        self.ops, self.ys, self.xs = ops, ys, xs
        self.n = len(ops)
        arr = (L.usp_batch_item * self.n)()
        for i, (op, y, x) in enumerate(zip(ops, ys, xs)):
            arr[i] = L.usp_batch_item(op.handle.value, y.data_ptr(), x.data_ptr(), 0, float(alpha), float(tol),
                                      int(maxit))
        self.items = arr
        nb = ct.c_size_t()
        L.check(L.lib().usp_batch_workspace_bytes(self.items, self.n, ct.byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=ops[0].device)
        self.ws_bytes = nb.value
        self.variant = 0

    def autotune(self, refine_every=20) -> int:
        v = ct.c_int()
        L.check(L.lib().usp_autotune_batched(self.items, self.n, int(refine_every), _ptr(self.ws), self.ws_bytes,
                                             _stream_ptr(self.ws.device), ct.byref(v)))
        self.variant = v.value
        return v.value

    def solve(self, refine_every=20, use_graph=True, variant=None) -> BatchResult:
        res = (L.usp_batch_result * self.n)()
        ms = np.zeros(1)
        v = self.variant if variant is None else int(variant)
        rc = L.check(L.lib().usp_solve_batched(self.items, self.n, int(refine_every), v, _ptr(self.ws),
                                               self.ws_bytes, _stream_ptr(self.ws.device), int(bool(use_graph)),
                                               res, _dp(ms)))
        return BatchResult(iterations=[r.iterations for r in res], status=[r.status for r in res],
                           rho=[r.rho for r in res], t_done_ms=[r.t_done_ms for r in res],
                           elapsed_ms=float(ms[0]), worst=rc)
