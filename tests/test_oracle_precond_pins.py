"""Pins for the oracle's Jacobi diagonal (Sec. 4.2), its per-scale grouping of
the SPAI objective and the Lipschitz constant of Alg. 2 (CPU only).

Each pin checks a property the paper or the mathematics fixes, computed by a
route other than the oracle's own formula, and a planted mistake in the oracle
fails it.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dwt, filters, lipschitz, precond


def _operator_with_weak_columns(seed=5, m=40, N=24):
    """A dense operator whose first columns are scaled far down, so that
    diag(A^T A) falls below eps = 1e-3 on them and stays above it elsewhere."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, N)) / np.sqrt(m)
    A[:, :4] *= np.array([0.0, 1e-3, 5e-3, 0.2])[None, :]
    return A


def test_jacobi_makes_the_hessian_unit_diagonal_and_takes_eps_below_it():
    """Sec. 4.2: P = max(diag(Theta_K^T Theta_K), eps).  Away from eps the
    preconditioned Hessian P^-1/2 M P^-1/2 (dense product) has unit diagonal;
    where diag(M) < eps, P equals eps exactly."""
    A = _operator_with_weak_columns()
    eps = 1e-3
    p = precond.jacobi(sp.csr_matrix(A), eps)
    M = A.T @ A
    S = np.diag(1.0 / np.sqrt(p))
    H = S @ M @ S
    col_sq = np.array([float(A[:, i] @ A[:, i]) for i in range(A.shape[1])])
    low = col_sq < eps
    assert low.sum() == 3 and (~low).sum() == A.shape[1] - 3   # eps active on 3 coordinates
    assert np.allclose(np.diag(H)[~low], 1.0, rtol=0, atol=1e-12)
    assert np.all(p[low] == eps)
    # where eps is active the diagonal stays below one (M_ii / eps < 1)
    assert np.all(np.diag(H)[low] < 1.0)


@pytest.mark.parametrize("mistake", ["min", "sum", "no_eps"])
def test_planted_jacobi_mistakes_are_caught(monkeypatch, mistake):
    A = _operator_with_weak_columns()
    eps = 1e-3
    m1 = precond.hessian_diagonals(sp.csr_matrix(A))[0]
    wrong = {"min": lambda a, e: np.minimum(m1, e), "sum": lambda a, e: m1 + e,
             "no_eps": lambda a, e: m1.copy()}[mistake]
    monkeypatch.setattr(precond, "jacobi", wrong)
    p = precond.jacobi(sp.csr_matrix(A), eps)
    M = A.T @ A
    col_sq = np.diag(M)
    low = col_sq < eps
    with np.errstate(divide="ignore", invalid="ignore"):
        H = np.diag(M) / p
    ok = (np.allclose(H[~low], 1.0, rtol=0, atol=1e-12) and np.all(p[low] == eps))
    assert not ok


def _level_from_atom(n, J, h, i):
    """Level and kind of coefficient i read off its synthesised Haar atom:
    the atom of level l covers a 2^l x 2^l square; approximation atoms have
    non-zero mean, detail atoms zero mean."""
    e = np.zeros(n * n)
    e[i] = 1.0
    atom = dwt.idwt2(e, h, J, n)
    area = int(np.count_nonzero(np.abs(atom) > 1e-12))
    level = int(round(np.log2(area) / 2))
    approx = abs(atom.sum()) > 1e-9
    return level, approx


@pytest.mark.parametrize("n,J", [(16, 3), (32, 2)])
def test_scale_groups_follow_the_atoms(n, J):
    """Per-scale groups: A_J alone (group 0, 4^(log n - J) coefficients), then
    one group per detail level l holding its three subbands,
    3 * 4^(log n - l) coefficients, numbered 1 + (J - l).  The expected group
    of every coefficient is read off its Haar atom, not from the layout."""
    h = filters.haar()
    g = precond.scale_groups(n, J)
    lg = int(np.log2(n))
    expect = np.empty(n * n, dtype=np.int64)
    for i in range(n * n):
        level, approx = _level_from_atom(n, J, h, i)
        assert 1 <= level <= J
        expect[i] = 0 if approx else 1 + (J - level)
        if approx:
            assert level == J
    assert np.array_equal(g, expect)
    sizes = np.bincount(g)
    assert sizes[0] == 4 ** (lg - J)
    for lev in range(1, J + 1):
        assert sizes[1 + J - lev] == 3 * 4 ** (lg - lev)


def test_planted_scale_group_merge_is_caught(monkeypatch):
    """Merging A_J into the group of level J must fail the atom-based pin."""
    n, J = 16, 3
    orig = precond.scale_groups
    monkeypatch.setattr(precond, "scale_groups", lambda n_, J_: np.maximum(orig(n_, J_), 1))
    h = filters.haar()
    g = precond.scale_groups(n, J)
    mismatch = 0
    for i in range(n * n):
        level, approx = _level_from_atom(n, J, h, i)
        mismatch += int(g[i] != (0 if approx else 1 + (J - level)))
    assert mismatch == 4 ** (int(np.log2(n)) - J)


def _spread_operator(seed=8, m=60, N=30):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, N)) * np.exp(rng.uniform(-2, 1, N))[None, :]
    p = np.exp(rng.uniform(-3, 2, N))
    return A, p


def test_lipschitz_precond_is_the_top_eigenvalue_of_the_scaled_hessian():
    """Alg. 2's constant: lambda_max(P^-1/2 A^T A P^-1/2) from a dense
    symmetric eigensolver, against the oracle's power iteration to 1e-9."""
    A, p = _spread_operator()
    S = np.diag(p ** -0.5)
    ev = np.linalg.eigvalsh(S @ (A.T @ A) @ S)
    assert ev[-1] > 1.05 * ev[-2]     # a spectral gap the power iteration resolves
    L, its = lipschitz.lipschitz_precond(sp.csr_matrix(A), p, np.ones(A.shape[1]))
    assert abs(L - ev[-1]) <= 1e-9 * ev[-1]
    assert its < 20000


def test_planted_lipschitz_precond_power_mistake_is_caught(monkeypatch):
    """P^-1 on both sides (the wrong power of P) gives a different constant."""
    A, p = _spread_operator()
    S = np.diag(p ** -0.5)
    ev = np.linalg.eigvalsh(S @ (A.T @ A) @ S)[-1]
    orig = lipschitz.lipschitz_precond
    monkeypatch.setattr(lipschitz, "lipschitz_precond",
                        lambda A_, p_, s_, **kw: orig(A_, np.asarray(p_) ** 2, s_, **kw))
    L, _ = lipschitz.lipschitz_precond(sp.csr_matrix(A), p, np.ones(A.shape[1]))
    assert abs(L - ev) > 1e-3 * ev
