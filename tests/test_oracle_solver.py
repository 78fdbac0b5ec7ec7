"""Pins for the oracle's solver pieces (CPU only): soft-thresholding, FISTA
(Alg. 1/Alg. 2), power iteration, duality gap, KKT and the SPAI lemma."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fista, lasso, lipschitz, precond


def test_soft_threshold_is_the_l1_prox():
    """S_t(z0) minimises 1/2 (z - z0)^2 + t |z| (checked on a fine grid)."""
    grid = np.linspace(-5, 5, 200001)
    for z0, t in [(2.0, 0.5), (-1.3, 0.4), (0.2, 0.7), (-0.7, 0.7), (0.0, 1.0)]:
        best = grid[np.argmin(0.5 * (grid - z0) ** 2 + t * np.abs(grid))]
        assert abs(fista.soft_threshold(np.array([z0]), t)[0] - best) < 1e-4
    assert fista.soft_threshold(np.array([0.7]), 0.7)[0] == 0.0


def test_momentum_weights():
    assert [fista.momentum(k) for k in (1, 2, 3, 4)] == [0.0, 0.25, 0.4, 0.5]


def test_first_iterates_worked_example():
    """Alg. 1 by hand, in exact rationals, on A = [[2, 1], [0, 1]], x0 = (3, 1),
    lam = 1/2, tau = 1/8 (any tau <= 1/L works for the worked example):
      k=1: y = 0,        g = A^T(Ay - x0) = (-6, -4),  z = (3/4, 1/2),
           x1 = S_{1/16}(z) = (11/16, 7/16),  y = x1 (weight 0)
      k=2: Ay - x0 = (29/16 - 3, 7/16 - 1) = (-19/16, -9/16),
           g = (-38/16, -28/16), z = y - g/8 = (11/16 + 19/64, 7/16 + 14/64)
             = (63/64, 42/64), x2 = (59/64, 38/64),
           y = x2 + 1/4 (x2 - x1) = (59/64 + 15/256, 38/64 + 10/256)
    """
    A = np.array([[2.0, 1.0], [0.0, 1.0]])
    x0 = np.array([3.0, 1.0])
    x1, _, y1 = fista.fista(A, x0, 0.5, 0.125, 1)
    assert np.allclose(x1, [11 / 16, 7 / 16], rtol=0, atol=1e-15)
    x2, xp, y2 = fista.fista(A, x0, 0.5, 0.125, 2)
    assert np.allclose(xp, [11 / 16, 7 / 16], rtol=0, atol=1e-15)
    assert np.allclose(x2, [59 / 64, 38 / 64], rtol=0, atol=1e-15)
    F = Fraction
    assert np.allclose(y2, [float(F(59, 64) + F(15, 256)), float(F(38, 64) + F(10, 256))],
                       rtol=0, atol=1e-15)


def _tiny_problem(seed, m=10, N=7):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, N)) / np.sqrt(m)
    b = rng.standard_normal(m)
    lam = 0.15 * np.max(np.abs(A.T @ b))
    return A, b, lam


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_fista_reaches_bruteforce_lasso(seed):
    A, b, lam = _tiny_problem(seed)
    xs, Es = lasso.lasso_bruteforce(A, b, lam)
    L = np.linalg.eigvalsh(A.T @ A).max()
    x, _, _ = fista.fista(A, b, lam, 1.0 / L, 3000)
    assert abs(fista.objective(A, b, lam, x) - Es) < 1e-10 * max(1.0, Es)
    assert np.max(np.abs(x - xs)) < 1e-6
    # O(1/k^2) bound, E(x_k) - E* <= 2 L ||x_init - x*||^2 / (k + 1)^2
    for k in [1, 5, 20, 100]:
        xk, _, _ = fista.fista(A, b, lam, 1.0 / L, k)
        assert fista.objective(A, b, lam, xk) - Es <= 2 * L * float(xs @ xs) / (k + 1) ** 2 + 1e-12


@pytest.mark.parametrize("seed", [4, 5])
def test_preconditioned_fista_reaches_same_optimum(seed):
    A, b, lam = _tiny_problem(seed)
    _, Es = lasso.lasso_bruteforce(A, b, lam)
    p = precond.spai(sp.csr_matrix(A))
    Lp, _ = lipschitz.lipschitz_precond(sp.csr_matrix(A), p, np.ones(A.shape[1]))
    x, _, _ = fista.fista(A, b, lam, 1.0 / Lp, 4000, p=p)
    assert abs(fista.objective(A, b, lam, x) - Es) < 1e-9 * max(1.0, Es)


def test_gap_and_kkt():
    A, b, lam = _tiny_problem(9, m=30, N=20)
    L = np.linalg.eigvalsh(A.T @ A).max()
    for k in [1, 10, 100]:
        x, _, _ = fista.fista(A, b, lam, 1.0 / L, k)
        E, D, gap, rel = fista.duality_gap(A, b, lam, x)
        assert gap >= -1e-14
        assert abs(E - fista.objective(A, b, lam, x)) < 1e-14
    x, _, _ = fista.fista(A, b, lam, 1.0 / L, 20000)
    E, D, gap, rel = fista.duality_gap(A, b, lam, x)
    assert rel < 1e-12
    bound, eq = fista.kkt(A, b, lam, x)
    assert bound < 1e-8 and eq < 1e-8
    # a non-optimal point violates the conditions
    assert max(fista.kkt(A, b, lam, 1.1 * x)) > 1e-3


def test_power_iteration_matches_eigensolver():
    rng = np.random.default_rng(11)
    A = sp.random(300, 300, density=0.05, random_state=rng, format="csr")
    L, its = lipschitz.lipschitz(A, rng.standard_normal(300))
    ev = np.linalg.eigvalsh((A.T @ A).toarray()).max()
    assert abs(L - ev) < 1e-9 * ev
    assert its > 2


def test_spai_lemma_minimises_frobenius_objective():
    rng = np.random.default_rng(2)
    A = sp.csr_matrix(rng.standard_normal((12, 9)))
    M = (A.T @ A).toarray()
    p = precond.spai(A)
    f0 = precond.spai_objective(M, p)
    for i in range(9):
        for d in (1e-4, -1e-4, 0.05):
            q = p.copy()
            q[i] *= 1 + d
            assert precond.spai_objective(M, q) >= f0
    # grouped form minimises the objective among group-constant diagonals
    groups = np.array([0, 0, 0, 1, 1, 2, 2, 2, 2])
    pg = precond.spai_grouped(A, groups)
    fg = precond.spai_objective(M, pg)
    for gid in range(3):
        for d in (1e-3, -1e-3):
            q = pg.copy()
            q[groups == gid] *= 1 + d
            assert precond.spai_objective(M, q) >= fg
    # singleton groups reduce to the lemma
    assert np.allclose(precond.spai_grouped(A, np.arange(9)), p, rtol=1e-14, atol=0)


def test_planted_momentum_mistake_is_caught(monkeypatch):
    monkeypatch.setattr(fista, "momentum", lambda k: k / (k + 3.0))
    A = np.array([[2.0, 1.0], [0.0, 1.0]])
    x2, _, _ = fista.fista(A, np.array([3.0, 1.0]), 0.5, 0.125, 3)
    monkeypatch.undo()
    x2_ok, _, _ = fista.fista(A, np.array([3.0, 1.0]), 0.5, 0.125, 3)
    assert np.max(np.abs(x2 - x2_ok)) > 1e-3


def test_planted_gradient_transpose_mistake_is_caught():
    """Using A instead of A^T in the gradient misses the brute-force optimum."""
    A, b, lam = _tiny_problem(1)

    class Wrong:
        """Square matrix whose 'transpose' is itself."""
        def __init__(self, M):
            self.M = M
            self.T = self
            self.shape = M.shape

        def __matmul__(self, v):
            return self.M @ v

    Asq = A[: A.shape[1], :]          # square, not symmetric
    bsq = b[: A.shape[1]]
    _, Esq = lasso.lasso_bruteforce(Asq, bsq, lam)
    L = np.linalg.eigvalsh(Asq.T @ Asq).max()
    with np.errstate(all="ignore"):
        x, _, _ = fista.fista(Wrong(Asq), bsq, lam, 1.0 / L, 3000)
    E = fista.objective(Asq, bsq, lam, x) if np.all(np.isfinite(x)) else np.inf
    assert not abs(E - Esq) < 1e-8


@pytest.mark.parametrize("seed", [3, 4])
def test_ista_descends_and_reaches_the_bruteforce_optimum(seed):
    """ISTA with tau = 1/L is a descent method (the objective never increases)
    and converges to the exact Lasso minimiser."""
    from oracle import lasso
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((9, 7))
    b = rng.standard_normal(9)
    lam = 0.25
    L = np.linalg.norm(A, 2) ** 2
    x = np.zeros(7)
    E_prev = fista.objective(A, b, lam, x)
    for _ in range(300):
        x = fista.ista(A, b, lam, 1.0 / L, 1, x_init=x)
        E = fista.objective(A, b, lam, x)
        assert E <= E_prev + 1e-12
        E_prev = E
    x_star, _ = lasso.lasso_bruteforce(A, b, lam)
    x = fista.ista(A, b, lam, 1.0 / L, 50000, x_init=x)
    assert np.max(np.abs(x - x_star)) <= 1e-7
    # its first step is FISTA's first step (the extrapolation weight of k = 1 is 0)
    assert np.array_equal(fista.ista(A, b, lam, 1.0 / L, 1), fista.fista(A, b, lam, 1.0 / L, 1)[0])
