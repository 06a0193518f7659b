"""Appendix theorems as invariants on tiny dense problems (Lemma 2, Theorem 2,
Corollary 1, condition-number bound, Theorem 3 rate bounds, shift splitting)."""
import numpy as np
import pytest

from oracle import canon, operators, theory
from paper_2207_14222_amd import media


def random_accretive(n, rng, vnorm=0.95):
    """A = L + V with L accretive (random skew part + positive semidefinite part)
    and V a random matrix scaled to ||V|| = vnorm, A shifted to be accretive."""
    G = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    S = (G - G.conj().T) / 2 * 3.0            # skew-Hermitian
    P = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    H = P @ P.conj().T / n * 0.2               # Hermitian PSD
    V = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    V *= vnorm / np.linalg.norm(V, 2)
    A = S + H + V
    shift = max(0.0, -theory.re_part(A)) + 1e-3
    A = A + shift * np.eye(n)
    return A, V


@pytest.mark.parametrize("seed", range(5))
def test_theorem2_sharp_threshold(seed):
    """||I - alpha B (A + B)^-1 A|| < 1  iff  alpha < 2 Re[A^-1 + B^-1]."""
    rng = np.random.default_rng(seed)
    A, V = random_accretive(6, rng)
    B = np.eye(6) - V
    amax = theory.alpha_max(A, B)
    assert amax > 1.0  # Corollary 1
    assert theory.opnorm(theory.iteration_matrix(A, B, 0.99 * amax)) < 1.0
    assert theory.opnorm(theory.iteration_matrix(A, B, 1.01 * amax)) >= 1.0


@pytest.mark.parametrize("seed", range(5))
def test_lemma2_equivalence(seed):
    """||I - G|| < 1  iff  Re[G^-1] > 1/2, checked on both sides of the boundary."""
    rng = np.random.default_rng(100 + seed)
    G0 = rng.normal(size=(5, 5)) + 1j * rng.normal(size=(5, 5))
    for s in (0.05, 0.2, 0.5, 1.0, 2.0):
        G = s * (np.eye(5) + 0.3 * G0)
        lhs = theory.opnorm(np.eye(5) - G) < 1.0
        rhs = theory.re_part(np.linalg.inv(G)) > 0.5
        assert lhs == rhs


def test_corollary1_contraction_for_canonical_operators():
    """For the canonical Helmholtz / diffusion / pantograph operators, ||M|| < 1 for alpha in (0, 1]."""
    probs = []
    p = media.helmholtz_1d(n=64, width=8)
    probs.append(canon.canonical_helmholtz(p.k2, p.source, p.spacing))
    q = media.helmholtz_spheres(shape=(6, 6, 6), count=2, width=1, w0=1.0, plane=1)
    probs.append(canon.canonical_helmholtz(q.k2, q.source, q.spacing))
    d = media.diffusion_blobs(shape=(4, 4, 8), sigma=1.0)
    probs.append(canon.canonical_diffusion(d.mu_a, d.D, d.omega_over_v, d.source, d.spacing))
    for cp in probs:
        op = operators.Operator(cp)
        A, B = op.dense_A(), op.dense_B()
        for alpha in (0.3, 0.8, 1.0):
            assert theory.opnorm(theory.iteration_matrix(A, B, alpha)) < 1.0


@pytest.mark.parametrize("seed", range(4))
def test_condition_and_rate_bounds(seed):
    rng = np.random.default_rng(200 + seed)
    A, V = random_accretive(6, rng, vnorm=0.5 + 0.1 * seed)
    B = np.eye(6) - V
    n = A.shape[0]
    P = theory.precond_inv(A, B, 1.0) @ A
    kappa = np.linalg.cond(P)
    assert kappa <= theory.condition_bound(A, B) * (1 + 1e-12)
    a, bound = theory.rate_bound(A, B)
    assert theory.opnorm(theory.iteration_matrix(A, B, a)) <= bound * (1 + 1e-12)
    # closed-form S-bounds: kappa <= (1 + sqrt(2S))^2 at the optimal ||V||,
    # in general the bound with the actual ||V|| is (S/||V|| + 1/(1-||V||)) (1 + ||V||)
    vn = theory.opnorm(V)
    S = theory.opnorm(np.linalg.inv(A)) * vn
    assert kappa <= (S / vn + 1 / (1 - vn)) * (1 + vn) * (1 + 1e-12)
    assert theory.kappa_bound_S(S) <= (S / vn + 1 / (1 - vn)) * (1 + vn) * (1 + 1e-12)


def test_hermitian_rate_equality():
    """A, B Hermitian: ||M|| = max |1 - alpha lambda| over the spectrum of (A^-1 + B^-1)^-1,
    and alpha = 2/(lmin + lmax) gives (lmax - lmin)/(lmax + lmin)."""
    rng = np.random.default_rng(9)
    n = 7
    Q = np.linalg.qr(rng.normal(size=(n, n)))[0]
    A = Q @ np.diag(rng.uniform(0.1, 3.0, n)) @ Q.T
    W = np.linalg.qr(rng.normal(size=(n, n)))[0]
    V = W @ np.diag(rng.uniform(-0.9, 0.9, n)) @ W.T
    B = np.eye(n) - V
    lam = np.linalg.eigvalsh(np.linalg.inv(np.linalg.inv(A) + np.linalg.inv(B)))
    for alpha in (0.5, 1.0, 1.3):
        M = theory.iteration_matrix(A, B, alpha)
        assert abs(theory.opnorm(M) - np.max(np.abs(1 - alpha * lam))) < 1e-12
    a = 2 / (lam[0] + lam[-1])
    assert abs(theory.opnorm(theory.iteration_matrix(A, B, a)) - (lam[-1] - lam[0]) / (lam[-1] + lam[0])) < 1e-12


def test_shift_splitting_special_case():
    """V = 0, L = A0/gamma, alpha = 2:  Gamma^-1 A = (1/2 (A0 + gamma I))^-1 A0 (Sec. 4.2)."""
    rng = np.random.default_rng(11)
    n = 6
    A0, _ = random_accretive(n, rng)
    gamma = 1.7
    A = A0 / gamma
    B = np.eye(n)
    lhs = theory.precond_inv(A, B, 2.0) @ A
    rhs = np.linalg.solve(0.5 * (A0 + gamma * np.eye(n)), A0)
    assert np.allclose(lhs, rhs, atol=1e-12)
