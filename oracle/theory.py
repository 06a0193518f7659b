"""Dense-matrix quantities from the paper's appendix, used as invariants on tiny
problems.

TEST INFRASTRUCTURE (FP64 oracle) -- see ``oracle/__init__.py``.

Definitions (appendix):
* Re[X] = inf over unit x of Re <x, X x>, i.e. the smallest eigenvalue of the
  Hermitian part (X + X^H)/2 (accretivity condition, Sec. 2).
* Gamma^-1 = alpha B (A + B)^-1 with B = I - V and A + B = L + I (Theorem 2).
* M = I - Gamma^-1 A (iteration matrix; Theorem 1, Theorem 2).
"""
from __future__ import annotations

import numpy as np


def re_part(X):
    """Re[X]: smallest eigenvalue of the Hermitian part of X."""
    H = 0.5 * (X + X.conj().T)
    return float(np.linalg.eigvalsh(H)[0])


def precond_inv(A, B, alpha):
    """Gamma^-1 = alpha B (A + B)^-1  (Theorem 2 notation)."""
    return alpha * B @ np.linalg.inv(A + B)


def iteration_matrix(A, B, alpha):
    """M = I - Gamma^-1 A."""
    n = A.shape[0]
    return np.eye(n) - precond_inv(A, B, alpha) @ A


def eliminated(A, B, alpha):
    """Gamma^-1 A in the eliminated form  alpha B [I - (L + I)^-1 B]  (Sec. 2.1),
    with L + I = A + B."""
    n = A.shape[0]
    return alpha * B @ (np.eye(n) - np.linalg.solve(A + B, B))


def alpha_max(A, B):
    """2 Re[A^-1 + B^-1]: the sharp step-size threshold of Theorem 2."""
    return 2.0 * re_part(np.linalg.inv(A) + np.linalg.inv(B))


def opnorm(X):
    return float(np.linalg.norm(X, 2))


def condition_bound(A, B):
    """Condition-number bound  (||A^-1|| + ||B^-1||) / Re[B^-1]  (appendix, condition number)."""
    Ai, Bi = np.linalg.inv(A), np.linalg.inv(B)
    return (opnorm(Ai) + opnorm(Bi)) / re_part(Bi)


def rate_bound(A, B):
    """Rate bound at alpha = Re[B^-1]:  ||M||^2 <= 1 - (Re[B^-1] / (||A^-1|| + ||B^-1||))^2
    (Theorem 3, intermediate inequality).  Returns (alpha, bound on ||M||)."""
    Ai, Bi = np.linalg.inv(A), np.linalg.inv(B)
    a = re_part(Bi)
    return a, float(np.sqrt(1.0 - (a / (opnorm(Ai) + opnorm(Bi))) ** 2))


def rate_bound_S(S):
    """Closed-form worst-case rate sqrt(1 - (1 + sqrt(2S))^-4) with S = ||A^-1|| ||V|| (Theorem 3)."""
    return float(np.sqrt(1.0 - (1.0 + np.sqrt(2.0 * S)) ** -4))


def kappa_bound_S(S):
    """(1 + sqrt(2S))^2: minimum over ||V|| of the condition bound (appendix)."""
    return float((1.0 + np.sqrt(2.0 * S)) ** 2)
