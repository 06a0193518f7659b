"""Lowest-energy eigenmodes with the split preconditioner (Sec. 4, the
eigenmode example, Eq. schrodinger).

TEST INFRASTRUCTURE (FP64 oracle) -- see ``oracle/__init__.py``.

H = -1/2 laplacian + V_s (unit mass, hbar = 1) on a periodic grid.  Adding a
constant Abar to both sides shifts every eigenvalue by Abar and keeps the
eigenvectors, so for Abar large enough H + Abar is positive definite.
H + Abar = -1/2 laplacian + (V_s + Abar) is the constant-D diffusion
operator with D = 1/2, mu = V_s + Abar and omega = 0, so its canonical form
(``canon.canonical_diffusion``) is A = (H + Abar) / c with c real: A, L and V
are Hermitian and the preconditioned operator P of ``krylov`` is Hermitian
positive definite (conjugate gradients apply).  An eigenpair A u = lam u
gives the energy E = c lam - Abar.

The result the method approaches is the k smallest eigenvalues of A and
their eigenvectors; the definition used here is the dense Hermitian
eigendecomposition (numpy.linalg.eigh), for small grids.
"""
from __future__ import annotations

import numpy as np

from .canon import VNORM, Canonical, canonical_diffusion
from .krylov import precond_apply
from .operators import Operator


def canonical_schrodinger(V, spacing, shift, vnorm=VNORM) -> Canonical:
    """Canonical form of H + shift = -1/2 laplacian + V + shift (V real)."""
    V = np.asarray(V, dtype=np.float64)
    return canonical_diffusion(V + shift, 0.5, 0.0, np.zeros(V.shape), spacing, vnorm)


def dense_hermitian_A(op: Operator):
    A = op.dense_A()
    return 0.5 * (A + A.conj().T)


def lowest_modes(op: Operator, k: int):
    """The k smallest eigenvalues of A (ascending) and orthonormal eigenvectors
    (columns, flattened grids)."""
    lam, U = np.linalg.eigh(dense_hermitian_A(op))
    return lam[:k], U[:, :k]


def energies(cp: Canonical, lam, shift):
    """E = c lam - shift."""
    return np.real(cp.c) * np.asarray(lam) - shift


def eigen_residual(op: Operator, lam, u):
    """||A u - lam u|| / ||lam u||."""
    u = np.asarray(u, dtype=np.complex128).reshape(op.shape)
    return float(np.linalg.norm(op.apply_A(u) - lam * u) / np.linalg.norm(lam * u))


def condition_numbers(op: Operator):
    """(kappa(A), kappa(P)) from dense eigenvalues (both Hermitian positive definite)."""
    ea = np.linalg.eigvalsh(dense_hermitian_A(op))
    P = op._dense(lambda v: precond_apply(op, v))
    ep = np.linalg.eigvalsh(0.5 * (P + P.conj().T))
    return float(ea[-1] / ea[0]), float(ep[-1] / ep[0]), ea, ep


def subspace_distance(U, W):
    """Largest principal-angle sine between the column spaces of U and W (same
    dimension; columns orthonormalised here)."""
    qu, _ = np.linalg.qr(np.asarray(U))
    qw, _ = np.linalg.qr(np.asarray(W))
    s = np.linalg.svd(qu.conj().T @ qw, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - float(np.min(s)) ** 2)))
