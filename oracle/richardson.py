"""Algorithm 1 of the paper (preconditioned fixed-point iteration with the forward
problem eliminated, Sec. 2.1) and its FP64 outer-refinement form.

TEST INFRASTRUCTURE (FP64 oracle) -- see ``oracle/__init__.py``.

One step, in the paper's order:
    Delta <- B [ (L + I)^-1 (B x + y) - x ]        (residual of the preconditioned system)
    x     <- x + alpha Delta                       (update)
which is x <- x + Gamma^-1 (y - A x) with Gamma^-1 = alpha B (L + I)^-1, because
A = L + I - B (Sec. 2.1).

Reading of the stopping rule: Algorithm 1 stops on ||Delta|| relative to the
preconditioned source; the paper's tables stop on ||A x - y|| / ||y||.  This
oracle records both: ``hist_pre[i] = ||Delta_i||`` every iteration and the true
relative residual ||y - A x|| / ||y|| every ``check_every`` iterations, and stops
on the latter.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .operators import Operator


@dataclass
class SolveResult:
    x: np.ndarray
    iterations: int
    hist_pre: list = field(default_factory=list)     # ||Delta_i||, i = 0..iterations-1
    hist_true: list = field(default_factory=list)    # (iteration, ||y - A x||/||y||)
    converged: bool = False


def step(op: Operator, x, y, alpha):
    """One iteration of Algorithm 1; returns (x_new, Delta)."""
    t = op.apply_B(x) + y
    u = op.apply_LI_inv(t)
    delta = op.apply_B(u - x)
    return x + alpha * delta, delta


def iterate(op: Operator, y, alpha, K, x0=None):
    """Exactly K iterations of Algorithm 1 from x0 (default 0)."""
    x = np.zeros(op.shape, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    hist = []
    for _ in range(K):
        x, d = step(op, x, y, alpha)
        hist.append(float(np.linalg.norm(d)))
    return x, hist


def relative_residual(op: Operator, x, y):
    return float(np.linalg.norm(op.residual(x, y)) / np.linalg.norm(y))


def solve(op: Operator, y, alpha, tol, maxit, check_every=1, x0=None) -> SolveResult:
    """Algorithm 1 until ||y - A x||/||y|| < tol (checked every ``check_every`` iterations)."""
    x = np.zeros(op.shape, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    res = SolveResult(x=x, iterations=0)
    for i in range(maxit):
        x, d = step(op, x, y, alpha)
        res.hist_pre.append(float(np.linalg.norm(d)))
        if (i + 1) % check_every == 0 or i + 1 == maxit:
            rho = relative_residual(op, x, y)
            res.hist_true.append((i + 1, rho))
            if rho < tol:
                res.converged = True
                res.iterations = i + 1
                res.x = x
                return res
    res.iterations = maxit
    res.x = x
    return res


def solve_refined(op: Operator, y, alpha, tol, maxit, inner=20, x0=None) -> SolveResult:
    """Outer iterative refinement, all in FP64 (reference semantics for the
    mixed-precision solver): r = y - A x; stop if ||r||/||y|| < tol; run ``inner``
    iterations of Algorithm 1 on A d = r from d = 0; x <- x + d.

    Since the fixed-point iteration keeps no state besides x (Sec. 2.1: a single
    vector), this produces the same iterates as ``solve`` up to rounding.
    """
    x = np.zeros(op.shape, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    ynorm = np.linalg.norm(y)
    res = SolveResult(x=x, iterations=0)
    it = 0
    while True:
        r = op.residual(x, y)
        rho = float(np.linalg.norm(r) / ynorm)
        res.hist_true.append((it, rho))
        if rho < tol:
            res.converged = True
            break
        if it >= maxit:
            break
        d = np.zeros_like(x)
        for _ in range(min(inner, maxit - it)):
            d, delta = step(op, d, r, alpha)
            res.hist_pre.append(float(np.linalg.norm(delta)))
            it += 1
        x = x + d
    res.x = x
    res.iterations = it
    return res


def solve_direct(op: Operator, y):
    """x* = A^-1 y by dense LU (numpy.linalg.solve); tiny grids only."""
    A = op.dense_A()
    return np.linalg.solve(A, np.asarray(y, dtype=np.complex128).ravel()).reshape(op.shape)
