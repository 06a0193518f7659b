"""Pins for the antisymmetrised canonical form (oracle, CPU), on the pantograph
with lam = 0.9, a = 0.1, b = -5 (non-accretive):
* the original system is not accretive and Algorithm 1 on it diverges;
* the antisymmetrised A is skew-Hermitian (c real), ||V|| = ||V~|| <= 0.95;
* (L + I)^-1 per Fourier mode equals the dense inverse of L + I;
* its solution is [x~; 0] with x~ the LU solution of the original system;
* Algorithm 1 on it decreases ||Delta|| monotonically (appendix, convergence).
The paper's printed count (below 1e-8 in 125 iterations) depends on a time
window and boundary treatment it does not give: parity unpinned."""
import numpy as np
import pytest

from oracle import antisym as AS
from oracle import canon, operators
from oracle import richardson as R
from paper_2207_14222_amd import media


@pytest.fixture(scope="module")
def system():
    p = media.pantograph_constant(n=96)
    cp = canon.canonical_pantograph(p.a, p.b, p.lam, p.t0, p.h, p.x0_at_lam_t, p.x0_t0)
    op = operators.Operator(cp)
    return cp, op, AS.AntisymOperator(op)


def test_original_is_not_accretive_and_diverges(system):
    cp, op, _ = system
    A = op.dense_A()
    assert np.linalg.eigvalsh(0.5 * (A + A.conj().T)).min() < -0.1
    res = R.solve(op, cp.y, 0.8, 1e-8, 60, 1)
    assert not res.converged
    assert res.hist_pre[-1] > 1e3 * res.hist_pre[0]


def test_antisymmetrised_structure(system):
    cp, op, aop = system
    assert abs(np.imag(cp.c)) == 0.0
    A = aop.dense(aop.apply_A)
    assert np.abs(A + A.conj().T).max() < 1e-12 * np.abs(A).max()
    V = aop.dense(aop.apply_V)
    Vt = op.dense_V()
    assert abs(np.linalg.norm(V, 2) - np.linalg.norm(Vt, 2)) < 1e-12
    assert np.linalg.norm(V, 2) <= 0.95 + 1e-12
    # V block structure: [[0, -V~^H], [V~, 0]]
    n = op.shape[0]
    assert np.allclose(V[:n, n:], -Vt.conj().T, atol=1e-14) and np.allclose(V[n:, :n], Vt, atol=1e-14)
    L = aop.dense(aop.apply_L)
    LIinv = aop.dense(aop.apply_LI_inv)
    assert np.allclose(LIinv, np.linalg.inv(L + np.eye(2 * n)), atol=1e-12)


def test_solution_is_original_solution(system):
    cp, op, aop = system
    A = aop.dense(aop.apply_A)
    y = AS.rhs(cp.y)
    x = np.linalg.solve(A, y.ravel()).reshape(aop.shape)
    xs = np.linalg.solve(op.dense_A(), cp.y)
    assert np.linalg.norm(x[0] - xs) / np.linalg.norm(xs) < 1e-10
    assert np.linalg.norm(x[1]) < 1e-10 * np.linalg.norm(xs)


def test_fixed_point_on_antisymmetrised_is_monotone(system):
    cp, op, aop = system
    y = AS.rhs(cp.y)
    for alpha in (1.0, 0.8):
        res = R.solve(aop, y, alpha, 1e-14, 400, 400)
        d = np.array(res.hist_pre)
        assert np.all(np.diff(d) <= 1e-13 * d[0])
        assert d[-1] < 0.5 * d[0]
