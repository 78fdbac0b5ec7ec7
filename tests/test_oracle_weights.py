"""Pins of the weighted forms (the paper's tuning, Sec. 1.3 weights w[i] and
Sec. 3.7 weighted thresholding) in the oracle."""
import itertools

import numpy as np
import pytest

from oracle import dwt, fista, lasso, theta


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_weighted_fista_reaches_the_rescaled_bruteforce_optimum(seed):
    """With z = w x the weighted problem is the textbook Lasso in z for A
    diag(1/w), whose optimum is found by enumeration."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((8, 7))
    b = rng.standard_normal(8)
    w = rng.uniform(1.0, 3.0, 7)
    lam = 0.3
    z, _ = lasso.lasso_bruteforce(A / w[None, :], b, lam)
    x_star = z / w
    L = np.linalg.norm(A, 2) ** 2
    x, _, _ = fista.fista(A, b, lam, 1.0 / L, 20000, w=w)
    assert np.max(np.abs(x - x_star)) <= 1e-8 * max(1.0, np.max(np.abs(x_star)))
    E, D, gap, rel = fista.duality_gap(A, b, lam, x_star, w)
    assert abs(rel) <= 1e-10
    bound, eq = fista.kkt(A, b, lam, x_star, w)
    assert bound <= 1e-9 and eq <= 1e-9


def test_weighted_gap_is_nonnegative_away_from_the_optimum():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((12, 9))
    b = rng.standard_normal(12)
    w = rng.uniform(0.5, 4.0, 9)
    for _ in range(20):
        x = rng.standard_normal(9)
        _, _, gap, _ = fista.duality_gap(A, b, 0.2, x, w)
        assert gap >= -1e-12


def test_planted_dual_scaling_mistake_is_caught():
    """Scaling the dual by max |g_i| w_i (instead of / w_i) leaves a gap at the optimum."""
    rng = np.random.default_rng(7)
    A = rng.standard_normal((8, 6))
    b = rng.standard_normal(8)
    w = rng.uniform(1.5, 3.0, 6)
    lam = 0.4
    z, _ = lasso.lasso_bruteforce(A / w[None, :], b, lam)
    x = z / w
    r = A @ x - b
    s_bad = min(1.0, lam / float(np.max(np.abs(A.T @ r) * w)))
    E = fista.objective(A, b, lam, x, w)
    D_bad = -0.5 * s_bad ** 2 * float(r @ r) - s_bad * float(r @ b)
    assert (E - D_bad) / E > 1e-3
    assert abs(fista.duality_gap(A, b, lam, x, w)[3]) <= 1e-10


def test_weighted_threshold_solves_the_minimax_problem():
    """Keeping the K largest |sigma_b T[a, b]| minimises
    sup_{sum_b |x_b| / sigma_b <= 1} ||(T - T_K) x||_inf = max over dropped |T[a, b]| sigma_b
    over all K-subsets (enumerated)."""
    rng = np.random.default_rng(11)
    T = rng.standard_normal((4, 4))
    sigma = np.array([1.0, 0.5, 0.25, 0.125])
    K = 5
    r, c, v = theta.top_k_weighted(T, K, sigma)
    kept = set(zip(r.tolist(), c.tolist()))
    def err(sub):
        return max((abs(T[a, b]) * sigma[b] for a in range(4) for b in range(4) if (a, b) not in sub), default=0.0)
    best = min(err(set(s)) for s in itertools.combinations([(a, b) for a in range(4) for b in range(4)], K))
    assert err(kept) == pytest.approx(best, abs=0)
    assert np.allclose(v, T[r, c])
    # uniform weights reduce to the naive rule
    r1, c1, _ = theta.top_k_weighted(T, K, np.ones(4))
    r0, c0, _ = theta.top_k(T, K)
    assert np.array_equal(r1, r0) and np.array_equal(c1, c0)


def test_scale_index_counts():
    n, J = 64, 3
    j = dwt.scale_index(n, J)
    # approximation and level-J details share scale log2(n) - J; a detail scale j has 3 * 4^j coefficients
    assert np.sum(j == 3) == 4 ** 3 + 3 * 4 ** 3
    assert np.sum(j == 4) == 3 * 4 ** 4 and np.sum(j == 5) == 3 * 4 ** 5
    sig = theta.column_scale_weights(n, J)
    assert sig[0] == 2.0 ** -3 and sig[-1] == 2.0 ** -5
