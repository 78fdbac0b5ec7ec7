"""Diagonal preconditioners for Alg. 2 (test oracle).

With M = A^T A (A = Theta_K):
* Jacobi (Sec. 4.2): P = max(diag(M), eps).
* SPAI (Sec. 4.3, lemma): the diagonal minimiser of ||Id - P^{-1} M||_F^2 is
  P[i,i] = M^2[i,i] / M[i,i] where M[i,i] != 0 (any positive value elsewhere;
  1 is used).  M[i,i] = ||A e_i||^2 and M^2[i,i] = ||M e_i||^2.
* Per-group SPAI: the same Frobenius objective with P constrained to be
  constant on groups of coordinates (a scale or a subband).  Setting the
  derivative in p_s to zero gives p_s = sum_{i in s} M^2[i,i] / sum_{i in s} M[i,i],
  which is the lemma when every group is a single coordinate.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def hessian_diagonals(A):
    """(diag(M), diag(M^2)) for M = A^T A."""
    A = sp.csr_matrix(A)
    m1 = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    M = (A.T @ A).tocsc()
    m2 = np.asarray(M.multiply(M).sum(axis=0)).ravel()
    return m1, m2


def spai(A) -> np.ndarray:
    m1, m2 = hessian_diagonals(A)
    p = np.ones_like(m1)
    nz = m1 != 0
    p[nz] = m2[nz] / m1[nz]
    return p


def spai_grouped(A, groups: np.ndarray) -> np.ndarray:
    """Per-group SPAI; ``groups`` gives each coordinate's group id."""
    m1, m2 = hessian_diagonals(A)
    ng = int(groups.max()) + 1
    s1 = np.bincount(groups, weights=m1, minlength=ng)
    s2 = np.bincount(groups, weights=m2, minlength=ng)
    pg = np.ones(ng)
    nz = s1 != 0
    pg[nz] = s2[nz] / s1[nz]
    return pg[groups]


def scale_groups(n: int, levels: int) -> np.ndarray:
    """Group ids for the per-scale reading: the coarsest approximation A_J is
    group 0 and the three detail subbands of level l form group 1 + (J - l)."""
    from .dwt import subbands
    g = np.empty(n * n, dtype=np.int64)
    for lev, e, off, s in subbands(n, levels):
        g[off:off + s * s] = 0 if e == (0, 0) else 1 + (levels - lev)
    return g


def jacobi(A, eps: float) -> np.ndarray:
    m1, _ = hessian_diagonals(A)
    return np.maximum(m1, eps)


def spai_objective(M: np.ndarray, p: np.ndarray) -> float:
    """||Id - P^{-1} M||_F^2 for a dense symmetric M."""
    R = np.eye(M.shape[0]) - M / p[:, None]
    return float(np.sum(R * R))
