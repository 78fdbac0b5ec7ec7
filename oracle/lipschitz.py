"""Largest eigenvalue of A^T A by power iteration (test oracle).

Alg. 1 takes the step tau = 1 / ||A||_2^2 without saying how the norm is
obtained.  Here: v_0 = start / ||start||, and for k = 1, 2, ...

    w = A v_{k-1},  rho_k = ||w||^2,  v_k = A^T w / ||A^T w||,

stopping at the first k >= 2 with |rho_k - rho_{k-1}| <= tol * rho_k (or at
``max_iters``) and returning rho_k (a Rayleigh quotient of A^T A, since
||v_{k-1}|| = 1).  ``apply``/``apply_t`` may be any linear maps, so the
preconditioned constant of Alg. 2 uses the same routine with
v -> P^{-1/2} A^T A P^{-1/2} v.
"""
from __future__ import annotations

import numpy as np


def power_iteration(apply, apply_t, start: np.ndarray, tol: float = 1e-12,
                    max_iters: int = 20000):
    v = np.asarray(start, dtype=np.float64)
    v = v / np.linalg.norm(v)
    rho_prev = None
    for k in range(1, max_iters + 1):
        w = apply(v)
        rho = float(w @ w)
        u = apply_t(w)
        nu = np.linalg.norm(u)
        if nu == 0.0:
            return 0.0, k
        v = u / nu
        if rho_prev is not None and abs(rho - rho_prev) <= tol * rho:
            return rho, k
        rho_prev = rho
    return rho, max_iters


def lipschitz(A, start: np.ndarray, tol: float = 1e-12, max_iters: int = 20000):
    """(L, iterations) with L = lambda_max(A^T A) for a sparse or dense A."""
    At = A.T
    return power_iteration(lambda v: A @ v, lambda w: At @ w, start, tol, max_iters)


def lipschitz_precond(A, p: np.ndarray, start: np.ndarray, tol: float = 1e-12,
                      max_iters: int = 20000):
    """lambda_max(P^{-1/2} A^T A P^{-1/2}) for a positive diagonal P."""
    s = 1.0 / np.sqrt(np.asarray(p, dtype=np.float64))
    At = A.T
    return power_iteration(lambda v: A @ (s * v), lambda w: s * (At @ w), start, tol, max_iters)
