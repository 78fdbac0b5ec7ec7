"""Exact Lasso minimum for tiny problems by enumeration (a pin for the oracle's FISTA).

For min_x 1/2 ||A x - b||^2 + lam ||x||_1 every minimiser satisfies, for a
support S and signs s on S: A_S^T A_S x_S = A_S^T b - lam s with
sign(x_S) = s, and |A_i^T (b - A x)| <= lam off S.  Enumerating every
(S, s) and keeping the feasible candidate of least objective gives the exact
optimum (3^N candidates, so only for N <= ~9).
"""
from __future__ import annotations

import itertools

import numpy as np


def lasso_bruteforce(A: np.ndarray, b: np.ndarray, lam: float):
    A = np.asarray(A, dtype=np.float64)
    N = A.shape[1]
    best_x, best_E = np.zeros(N), 0.5 * float(b @ b)
    for signs in itertools.product((-1, 0, 1), repeat=N):
        s = np.array(signs, dtype=np.float64)
        S = s != 0
        if not S.any():
            continue
        AS = A[:, S]
        G = AS.T @ AS
        try:
            xs = np.linalg.solve(G, AS.T @ b - lam * s[S])
        except np.linalg.LinAlgError:
            continue
        if np.any(np.sign(xs) != s[S]):
            continue
        x = np.zeros(N)
        x[S] = xs
        r = b - A @ x
        if np.any(np.abs(A[:, ~S].T @ r) > lam * (1 + 1e-12)):
            continue
        E = 0.5 * float((A @ x - b) @ (A @ x - b)) + lam * float(np.abs(x).sum())
        if E < best_E:
            best_x, best_E = x, E
    return best_x, best_E
