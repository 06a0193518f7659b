"""Krylov drivers on the preconditioned system with the forward problem
eliminated (Sec. 2.1; the solver comparison of Sec. 4, Table 1b): BiCGSTAB
(van der Vorst, 1992), restarted GMRES(m) (Saad and Schultz, 1986) and, for
Hermitian positive definite A (the eigenmode example of Sec. 4, whose linear
solves use conjugate gradients), CG (Hestenes and Stiefel, 1952): with A, L
and V Hermitian, P = B - B (L + I)^-1 B is Hermitian, and P = B [B^-1 -
(L + I)^-1] B is positive definite when A = L + I - B is (B is, as ||V|| < 1).

TEST INFRASTRUCTURE (FP64 oracle) -- see ``oracle/__init__.py``.

With Gamma^-1 = B (L + I)^-1 (step size 1) the preconditioned system is
Gamma^-1 A x = Gamma^-1 y, and since A = L + I - B (Sec. 2.1)

    P v = B [v - (L + I)^-1 (B v)],        b = B (L + I)^-1 y,

so one step of Algorithm 1 is x <- x + alpha (b - P x).  The Krylov methods
solve P x = b with the textbook recurrences (unpreconditioned form applied to
the already preconditioned operator).  Stopping: the true residual
||y - A x||/||y|| of the original system, every ``check_every`` iterations
for BiCGSTAB and at the end of every GMRES cycle.  A GMRES cycle also ends
early when its residual estimate, scaled by the ratio of true to
preconditioned residual seen at the last check, falls below the tolerance.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .operators import Operator


def precond_apply(op: Operator, v):
    """P v = B [v - (L + I)^-1 B v]."""
    return op.apply_B(v - op.apply_LI_inv(op.apply_B(v)))


def precond_rhs(op: Operator, y):
    """b = B (L + I)^-1 y."""
    return op.apply_B(op.apply_LI_inv(y))


def _rel_true(op, x, y):
    return float(np.linalg.norm(op.residual(x, y)) / np.linalg.norm(y))


@dataclass
class KrylovResult:
    x: np.ndarray
    iterations: int
    converged: bool = False
    breakdown: bool = False
    hist_true: list = field(default_factory=list)   # (iteration, ||y - A x||/||y||)
    hist_est: list = field(default_factory=list)    # GMRES: (iteration, ||b - P x||) estimates


def bicgstab(op: Operator, y, tol, maxit, check_every=1, x0=None) -> KrylovResult:
    """BiCGSTAB on P x = b, shadow vector r^ = r_0."""
    x = np.zeros(op.shape, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    b = precond_rhs(op, y)
    r = b - precond_apply(op, x)
    rhat = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(r)
    p = np.zeros_like(r)
    res = KrylovResult(x=x, iterations=0)
    for i in range(maxit):
        rho_new = np.vdot(rhat, r)
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = precond_apply(op, p)
        den = np.vdot(rhat, v)
        if den == 0:
            res.breakdown = True
            break
        alpha = rho_new / den
        s = r - alpha * v
        t = precond_apply(op, s)
        tt = np.vdot(t, t)
        if tt == 0:                     # s = 0: x + alpha p is exact
            x = x + alpha * p
            r = s
            res.iterations = i + 1
            rho_t = _rel_true(op, x, y)
            res.hist_true.append((i + 1, rho_t))
            res.converged = rho_t < tol
            break
        omega = np.vdot(t, s) / tt
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        res.iterations = i + 1
        if (i + 1) % check_every == 0 or i + 1 == maxit:
            rho_t = _rel_true(op, x, y)
            res.hist_true.append((i + 1, rho_t))
            if rho_t < tol:
                res.converged = True
                break
    res.x = x
    return res


def cg(op: Operator, y, tol, maxit, check_every=1, x0=None) -> KrylovResult:
    """Conjugate gradients on P x = b (P Hermitian positive definite)."""
    x = np.zeros(op.shape, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    b = precond_rhs(op, y)
    r = b - precond_apply(op, x)
    p = r.copy()
    rr = float(np.vdot(r, r).real)
    res = KrylovResult(x=x, iterations=0)
    for i in range(maxit):
        q = precond_apply(op, p)
        pq = np.vdot(p, q)
        if pq == 0:
            res.breakdown = True
            break
        alpha = rr / pq
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(np.vdot(r, r).real)
        p = r + (rr_new / rr) * p
        rr = rr_new
        res.iterations = i + 1
        res.hist_est.append((i + 1, float(np.sqrt(rr))))
        if (i + 1) % check_every == 0 or i + 1 == maxit:
            rho_t = _rel_true(op, x, y)
            res.hist_true.append((i + 1, rho_t))
            if rho_t < tol:
                res.converged = True
                break
    res.x = x
    return res


def gmres(op: Operator, y, m, tol, maxit, x0=None) -> KrylovResult:
    """Restarted GMRES(m) on P x = b: Arnoldi with modified Gram-Schmidt, Givens
    rotations on the Hessenberg matrix, x updated at the end of each cycle."""
    x = np.zeros(op.shape, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    b = precond_rhs(op, y)
    bn = float(np.linalg.norm(b))
    res = KrylovResult(x=x, iterations=0)
    ratio = 1.0   # true / preconditioned relative residual at the last check (1 at x = 0)
    total = 0
    while total < maxit:
        r = b - precond_apply(op, x)
        beta = float(np.linalg.norm(r))
        if total > 0 and res.hist_true:
            ratio = res.hist_true[-1][1] / max(beta / bn, 1e-300)
        V = [r / beta]
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        k = 0
        for j in range(m):
            w = precond_apply(op, V[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            # rotations of the earlier columns, then a new one zeroing H[j+1, j]
            for i in range(j):
                hi, hi1 = H[i, j], H[i + 1, j]
                H[i, j] = np.conj(cs[i]) * hi + np.conj(sn[i]) * hi1
                H[i + 1, j] = -sn[i] * hi + cs[i] * hi1
            den = np.sqrt(abs(H[j, j]) ** 2 + abs(H[j + 1, j]) ** 2)
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            k = j + 1
            total += 1
            res.hist_est.append((total, float(abs(g[j + 1]))))
            happy = hn == 0.0          # the Krylov space is invariant: the cycle's solution is exact
            if not happy:
                V.append(w / hn)
            if happy or total >= maxit or abs(g[j + 1]) / bn * ratio < tol:
                break
        # back substitution for the cycle's coefficients
        z = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            z[i] = (g[i] - np.dot(H[i, i + 1:k], z[i + 1:k])) / H[i, i]
        for i in range(k):
            x = x + z[i] * V[i]
        rho_t = _rel_true(op, x, y)
        res.hist_true.append((total, rho_t))
        if rho_t < tol:
            res.converged = True
            break
    res.x = x
    res.iterations = total
    return res
