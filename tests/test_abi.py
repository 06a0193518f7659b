"""The C ABI library loads and exports every symbol include/usp.h declares (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "usp.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(usp_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("usp_prepare_operator", "usp_solve", "usp_workspace_bytes", "usp_destroy", "usp_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2207_14222_amd import _lib
    L = _lib.lib()
    for name in declared():
        assert hasattr(L, name), name
    assert set(_lib.EXPORTS) == set(declared())


def test_workspace_bytes_and_shape_validation():
    from paper_2207_14222_amd import _lib, solver
    L = _lib.lib()
    sym = solver.make_symbol((64, 32, 16), (0.25,) * 3, s=1j, a0=2.0, a2=-1.0)
    n = ctypes.c_size_t()
    assert L.usp_workspace_bytes(ctypes.byref(sym), _lib.USP_C64, 0, ctypes.byref(n)) == 0
    N = 64 * 32 * 16
    assert n.value >= N * (8 + 16)
    nr = ctypes.c_size_t()
    assert L.usp_workspace_bytes(ctypes.byref(sym), _lib.USP_C128, _lib.USP_FLAG_REFINE, ctypes.byref(nr)) == 0
    assert nr.value >= N * (8 + 16 + 3 * 8)
    # refined mode requires complex128 buffers
    assert L.usp_workspace_bytes(ctypes.byref(sym), _lib.USP_C64, _lib.USP_FLAG_REFINE, ctypes.byref(n)) == -1
    bad = solver.make_symbol((64, 30, 16), (0.25,) * 3)
    assert L.usp_workspace_bytes(ctypes.byref(bad), _lib.USP_C64, 0, ctypes.byref(n)) == _lib.USP_ERR_UNSUPPORTED_SHAPE
    assert "power of two" in _lib.last_error()
    big = solver.make_symbol((2048,), (0.25,))
    assert L.usp_workspace_bytes(ctypes.byref(big), _lib.USP_C64, 0, ctypes.byref(n)) == _lib.USP_ERR_UNSUPPORTED_SHAPE
    # the first-derivative term is 1-D only: a 2-D / 3-D symbol carrying it is rejected
    for shape in ((32, 16), (8, 16, 32)):
        for kw in (dict(a1=1.0), dict(nyquist_zero=True)):
            s2 = solver.make_symbol(shape, (0.25,) * len(shape), s=1j, a0=2.0, a2=-1.0, **kw)
            assert L.usp_workspace_bytes(ctypes.byref(s2), _lib.USP_C64, 0, ctypes.byref(n)) == _lib.USP_ERR_INVALID
            assert "a1" in _lib.last_error()
    s1 = solver.make_symbol((64,), (0.25,), s=1.0, a0=2.0, a1=1.0, nyquist_zero=True)
    assert L.usp_workspace_bytes(ctypes.byref(s1), _lib.USP_C128, 0, ctypes.byref(n)) == 0


def test_host_smallest_circle_matches_oracle():
    """Host Welzl (library) against the oracle's exhaustive hull search."""
    from oracle import canon
    from paper_2207_14222_amd import solver
    rng = np.random.default_rng(5)
    for trial in range(5):
        pts = rng.normal(size=300) * 5 + 1j * rng.normal(size=300) * (1 + trial)
        z, r = solver.smallest_circle(pts)
        zo, ro = canon.smallest_circle(pts)
        assert abs(z - zo) < 1e-10 * (1 + abs(zo)) and abs(r - ro) < 1e-10 * ro
        zr, rr = solver.smallest_circle(pts, "real")
        zor, ror = canon.smallest_real_centre(pts)
        assert abs(zr - zor) < 1e-7 * (1 + abs(zor)) and abs(rr - ror) < 1e-12 * ror


def test_host_canonical_helmholtz_matches_oracle():
    from oracle import canon
    from paper_2207_14222_amd import _lib, media, solver
    p = media.helmholtz_spheres(shape=(16, 16, 16), count=5, width=3, w0=3.0, plane=2)
    k2 = np.ascontiguousarray(p.k2)
    grid = solver.make_symbol(k2.shape, p.spacing)
    out = _lib.usp_symbol()
    c = np.zeros(2)
    b = np.zeros(2)
    flat = k2.ravel().view(np.float64)
    rc = _lib.lib().usp_canonical_helmholtz(flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), k2.size, 0, None,
                                            0.95, ctypes.byref(grid), ctypes.byref(out),
                                            c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0
    cp = canon.canonical_helmholtz(p.k2, p.source, p.spacing)
    assert abs(complex(*c) - cp.c) < 1e-12 * abs(cp.c)
    assert abs(complex(*b) - cp.bias) < 1e-12 * abs(cp.bias)
    co = solver.symbol_coeffs(out)
    assert abs(co["s"] - cp.s) < 1e-14 and co["a0"] == complex(*b) and co["a2"] == -1


def test_host_canonical_schrodinger_matches_oracle():
    """usp_canonical_schrodinger (shift applied in the library) against the oracle's
    canonical form of H + shift: c, the symbol, and B built from the returned field
    bias on V itself."""
    from oracle import eigen
    from paper_2207_14222_amd import _lib, media, solver
    V, h = media.double_ring_well(n=32, box=6.0)
    shift = 5.0
    grid = solver.make_symbol(V.shape, (h, h))
    out = _lib.usp_symbol()
    c = np.zeros(2)
    b = np.zeros(2)
    DPT = ctypes.POINTER(ctypes.c_double)
    Vc = np.ascontiguousarray(V, dtype=np.float64)
    rc = _lib.lib().usp_canonical_schrodinger(Vc.ctypes.data_as(DPT), Vc.size, shift, 0.95, ctypes.byref(grid),
                                              ctypes.byref(out), c.ctypes.data_as(DPT), b.ctypes.data_as(DPT))
    assert rc == 0
    cp = eigen.canonical_schrodinger(V, (h, h), shift)
    assert abs(complex(*c) - cp.c) < 1e-12 * abs(cp.c)
    co = solver.symbol_coeffs(out)
    assert abs(co["s"] - cp.s) < 1e-14 * abs(cp.s)
    assert abs(co["a0"] - cp.a0) < 1e-13 and co["a2"] == cp.a2 == 0.5
    B = 1.0 - (V - complex(*b)) / complex(*c)
    assert np.max(np.abs(B - cp.B)) < 1e-14
    # a constant potential has no smallest circle of positive radius
    flat = np.full(16, -3.0)
    assert _lib.lib().usp_canonical_schrodinger(flat.ctypes.data_as(DPT), 16, 1.0, 0.95, ctypes.byref(grid),
                                                ctypes.byref(out), c.ctypes.data_as(DPT),
                                                b.ctypes.data_as(DPT)) == _lib.USP_ERR_INVALID


def test_host_canonical_pantograph_matches_oracle():
    """Library pantograph canonical form (power-iteration gather norm) vs the oracle (dense SVD)."""
    from oracle import canon
    from paper_2207_14222_amd import _lib, media, solver
    for bval in (5.0, -5.0):
        pp = media.pantograph(n=1024, b_value=bval)
        cp = canon.canonical_pantograph(pp.a, pp.b, pp.lam, pp.t0, pp.h, pp.x0_at_lam_t, pp.x0_t0)
        n = pp.n
        f = lambda z: np.ascontiguousarray(z, dtype=np.complex128)
        a, b, x0l = f(pp.a), f(pp.b), f(pp.x0_at_lam_t)
        dp = lambda z: z.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        sym = _lib.usp_symbol()
        Bh, g0, g1, yh = (np.zeros(n, np.complex128) for _ in range(4))
        idx = np.zeros(n, np.int32)
        c, bias, x0t = np.zeros(2), np.zeros(2), np.array([pp.x0_t0.real, pp.x0_t0.imag])
        rc = _lib.lib().usp_canonical_pantograph(dp(a), dp(b), n, pp.lam, pp.t0, pp.h, dp(x0l),
                                                 x0t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0.95,
                                                 ctypes.byref(sym), dp(Bh), idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                                 dp(g0), dp(g1), dp(yh),
                                                 c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 bias.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        assert rc == 0
        assert abs(complex(*c) - cp.c) < 1e-10 * abs(cp.c)
        assert abs(complex(*bias) - cp.bias) < 1e-12 * abs(cp.bias)
        assert np.allclose(Bh, cp.B, atol=1e-10) and np.allclose(yh, cp.y, atol=1e-10)
        # same gather as a matrix (index conventions may differ where weights vanish)
        So = np.zeros((n, n), complex)
        Sl = np.zeros((n, n), complex)
        for j in range(n):
            So[j, cp.gi[j]] += cp.g0[j]
            So[j, min(cp.gi[j] + 1, n - 1)] += cp.g1[j]
            Sl[j, idx[j]] += g0[j]
            Sl[j, min(idx[j] + 1, n - 1)] += g1[j]
        assert np.allclose(So, Sl, atol=1e-10)
        co = solver.symbol_coeffs(sym)
        assert co["a1"] == 1 and sym.nyquist_zero == 1 and abs(co["s"] - cp.s) < 1e-12


def test_host_canonical_flux_matches_oracle():
    """Library flux-form canonicalisation (closed-form 2 x 2 and trigonometric
    3 x 3 spectral norms, exact where they set c) vs the oracle (numpy SVD
    norms), on the anisotropic ring, an isotropic case and a random 3-D
    tensor medium."""
    from oracle import flux as F
    from paper_2207_14222_amd import _lib, media, solver
    p = media.diffusion_ring(n=64, h=0.4, radius=8.0, width=3.0, abs_rows=6, src_row=3)
    cases = [(p.mu, p.D, p.source, p.h)]
    n = 16
    Di = np.zeros((n, n, 2, 2), complex)
    Di[..., 0, 0] = Di[..., 1, 1] = 1.7
    mu = np.full((n, n), 0.3, complex)
    mu[0, 0] = 2.0
    cases.append((mu, Di, np.ones((n, n)), 0.5))
    q = media.diffusion_tensor_random3(shape=(8, 16, 32), seed=3)
    cases.append((q.mu, q.D, q.source, q.h))
    for mu, D, src, h in cases:
        d = mu.ndim
        cp = F.canonical_flux(mu, D, src, h)
        sym, bu, b2, y = solver.canonical_flux_host(mu, D, src, h)
        assert sym.ndim == d and list(sym.n[:d]) == list(mu.shape)
        assert abs(sym.c - cp.c) < 1e-12 * cp.c
        assert np.allclose(np.array(sym.s[:d + 1]), cp.s, rtol=1e-12)
        assert abs(complex(*sym.mubar) - cp.mubar) < 1e-12 * (1 + abs(cp.mubar))
        dib = np.array([complex(*sym.dibar[e]) for e in range(d * d)]).reshape(d, d)
        assert np.allclose(dib, cp.Dibar, rtol=1e-12, atol=1e-14)
        assert np.allclose(bu, cp.Buu, atol=1e-12) and np.allclose(b2, cp.B2, atol=1e-12)
        assert np.allclose(y, cp.y, rtol=1e-12, atol=1e-14)
    # a singular tensor is rejected
    Ds = np.array(p.D, dtype=complex)
    Ds[3, 3] = 0.0
    with pytest.raises(_lib.UspError):
        solver.canonical_flux_host(p.mu, Ds, p.source, p.h)


def test_host_hermitian_eig_matches_numpy():
    """The Jacobi eigensolver of the Rayleigh-Ritz step against numpy.linalg.eigh,
    including repeated eigenvalues (eigenvectors checked through A Z = Z diag(w))."""
    from paper_2207_14222_amd import solver
    rng = np.random.default_rng(9)
    cases = []
    for n in (1, 2, 5, 40, 64):
        m = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        cases.append(m + m.conj().T)
    q, _ = np.linalg.qr(rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12)))
    d = np.array([1.0, 1.0, 1.0, 2.0, 2.0, -3.0, 5.0, 5.0, 5.0, 5.0, 0.5, 7.0])
    cases.append(q @ np.diag(d) @ q.conj().T)
    cases.append(np.diag(rng.standard_normal(9)).astype(complex))   # already diagonal
    for a in cases:
        w, z = solver.hermitian_eig(a)
        scale = max(1.0, float(np.abs(a).max()))
        assert np.allclose(w, np.linalg.eigvalsh(a), atol=1e-12 * scale)
        assert np.allclose(z.conj().T @ z, np.eye(len(w)), atol=1e-12)
        assert np.allclose(a @ z, z * w[None, :], atol=1e-11 * scale)
