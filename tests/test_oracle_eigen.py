"""Pins for the eigenmode oracle and the CG driver (CPU):
* the 2-D isotropic harmonic oscillator: the lowest energies of the shifted,
  canonicalised operator are omega (n + 1) with degeneracy n + 1
  (1, 2, 2, 3, 3, 3) to 1e-8 (spectral derivatives resolve the Gaussians);
* shifting by Abar moves every energy by Abar and leaves the modes alone
  (two shifts give the same energies and the same eigenspaces);
* P is Hermitian with its spectrum in (0, 2) for the Hermitian canonical
  operator, and its condition number stays put under grid refinement while
  that of A grows like h^-2;
* CG on a constant-V grid terminates after exactly as many iterations as P
  has distinct eigenvalues on the right-hand side, and not one earlier;
* CG minimises the P-norm error: never above the fixed-point iterate with the
  same number of operator applications; CG reaches the dense LU solution."""
import numpy as np
import pytest

from oracle import canon, eigen, krylov, operators, richardson
from paper_2207_14222_amd import media


def _op(V, h, shift):
    cp = eigen.canonical_schrodinger(V, (h, h), shift)
    return cp, operators.Operator(cp)


def test_harmonic_oscillator_energies():
    V, h = media.harmonic_well(n=40, h=0.45, omega=1.0)
    shift = 10.0
    cp, op = _op(V, h, shift)
    lam, U = eigen.lowest_modes(op, 6)
    E = eigen.energies(cp, lam, shift)
    assert np.allclose(E, [1.0, 2.0, 2.0, 3.0, 3.0, 3.0], atol=1e-8)
    for i in range(6):
        assert eigen.eigen_residual(op, lam[i], U[:, i]) < 1e-10


def test_shift_moves_energies_and_keeps_modes():
    V, h = media.double_ring_well(n=32, box=6.0)
    cp1, op1 = _op(V, h, 5.0)
    cp2, op2 = _op(V, h, 12.0)
    l1, U1 = eigen.lowest_modes(op1, 4)
    l2, U2 = eigen.lowest_modes(op2, 4)
    assert np.allclose(eigen.energies(cp1, l1, 5.0), eigen.energies(cp2, l2, 12.0), atol=1e-9)
    assert eigen.subspace_distance(U1, U2) < 1e-7
    assert eigen.energies(cp1, l1, 5.0)[0] < 0.0          # a bound state of the well


def test_precond_hermitian_positive_definite_and_grid_independent():
    """P is Hermitian with its spectrum in (0, 2) (the iteration with alpha = 1
    contracts, Theorem 1); refining the grid multiplies kappa(A) (~ h^-2) while
    kappa(P) stays put."""
    ks = []
    for n in (32, 48):
        V, h = media.double_ring_well(n=n, box=6.0)
        cp, op = _op(V, h, 5.0)
        P = op._dense(lambda v: krylov.precond_apply(op, v))
        assert np.allclose(P, P.conj().T, atol=1e-12)
        kA, kP, ea, ep = eigen.condition_numbers(op)
        assert ea[0] > 0 and 0.0 < ep[0] and ep[-1] < 2.0
        ks.append((kA, kP))
    assert ks[1][0] / ks[0][0] > 2.0
    assert ks[1][1] / ks[0][1] < 1.2


def _constant(shape=(8, 8)):
    """The canonical operator with V = 0 (the potential equal to its bias):
    P = F^-1 diag(l / (l + 1)) F."""
    V = np.full(shape, 0.7)
    V[0, 0] = -0.3              # a non-constant potential for the canonical form ...
    cp = eigen.canonical_schrodinger(V, (0.5, 0.5), 2.0)
    cp.v[...] = 0.0             # ... whose V is then replaced by 0
    return cp, operators.Operator(cp)


def test_cg_terminates_at_the_number_of_distinct_eigenvalues():
    cp, op = _constant()
    b0 = 1.0 - op.v.flat[0]
    lam = b0 * (1.0 - b0 / (op.l + 1.0))
    modes = [(0, 0), (1, 0), (1, 1), (2, 0)]       # |k|^2 = 0, 1, 2, 4
    assert len({round(float(abs(lam[m])), 12) for m in modes}) == len(modes)
    rng = np.random.default_rng(3)
    yhat = np.zeros(op.shape, dtype=complex)
    for m in modes:
        yhat[m] = rng.standard_normal() + 1j * rng.standard_normal()
    y = np.fft.ifft2(yhat)
    q = len(modes)
    r_short = krylov.cg(op, y, 1e-30, q - 1)
    r_full = krylov.cg(op, y, 1e-30, q)
    assert r_short.hist_true[-1][1] > 1e-6
    assert r_full.hist_true[-1][1] < 1e-12


def test_cg_minimises_p_norm_error_and_reaches_lu():
    V, h = media.double_ring_well(n=16, box=6.0)
    cp, op = _op(V, h, 5.0)
    rng = np.random.default_rng(2)
    y = rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape)
    xs = richardson.solve_direct(op, y)
    P = op._dense(lambda v: krylov.precond_apply(op, v))

    def pnorm(e):
        e = e.ravel()
        return float(np.real(np.vdot(e, P @ e)))

    xf = np.zeros(op.shape, dtype=complex)
    for j in range(1, 13):
        xf, _ = richardson.step(op, xf, y, 1.0)
        xc = krylov.cg(op, y, 1e-30, j).x
        assert pnorm(xc - xs) <= pnorm(xf - xs) * (1 + 1e-10)
    r = krylov.cg(op, y, 1e-11, 2000, check_every=5)
    assert r.converged
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < 1e-9
