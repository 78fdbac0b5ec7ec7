"""Accelerated proximal gradient for the approximate problem (test oracle).

Problem (Sec. 1.3, approximate problem): minimise
    E(x) = 1/2 ||A x - x0||^2 + lam * sum_i w_i |x_i|
with A = Theta_K and x0 = Psi^* u0.

* ``fista``: Alg. 1 (and Alg. 2 when a diagonal P is given).  For k = 1..Nit
      g = A^T (A y - x0)                      (gradient of Sec. 1.3; the
                                               printed formula drops the y)
      z = y - tau * g / P
      x_k = S_{tau lam w / P}(z)              (prox of the weighted l1 norm in
                                               the P-metric: coordinate-wise
                                               soft-thresholding, Sec. 4 text
                                               after Alg. 2)
      y = x_k + (k - 1)/(k + 2) (x_k - x_{k-1})
  with x^(0) = y^(1) = x_init (zero by default).  Alg. 2 prints u0 where x0
  is meant in the gradient; x0 is used.
* ``ista``: the same step without extrapolation (y = x).
* ``soft_threshold``: S_t(z) = sign(z) max(|z| - t, 0).
* ``objective``, ``duality_gap``: E and the textbook Lasso dual bound (the
  paper stops on E(x) - E* instead, Sec. 5.5; the gap is a computable
  substitute that needs no E*).
* ``kkt``: the l1 optimality conditions |(A^T(Ax - x0))_i| <= lam w_i, with
  equality and opposite sign on the support.
"""
from __future__ import annotations

import numpy as np


def soft_threshold(z: np.ndarray, t) -> np.ndarray:
    return np.sign(z) * np.maximum(np.abs(z) - t, 0.0)


def momentum(k: int) -> float:
    """Extrapolation weight (k - 1)/(k + 2) of Alg. 1."""
    return (k - 1.0) / (k + 2.0)


def fista(A, x0: np.ndarray, lam: float, tau: float, iters: int, x_init=None,
          p=None, w=None, k0: int = 1, callback=None):
    """Run ``iters`` iterations of Alg. 1 (Alg. 2 if ``p`` is given).

    Returns (x, x_prev, y) after the last iteration so a run can be resumed
    with ``k0`` = next iteration index.
    """
    x0 = np.asarray(x0, dtype=np.float64)
    N = A.shape[1]
    x = np.zeros(N) if x_init is None else np.asarray(x_init, dtype=np.float64).copy()
    y = x.copy()
    At = A.T
    pinv = np.ones(N) if p is None else 1.0 / np.asarray(p, dtype=np.float64)
    wt = np.ones(N) if w is None else np.asarray(w, dtype=np.float64)
    x_prev = x
    for k in range(k0, k0 + iters):
        g = At @ (A @ y - x0)
        z = y - tau * pinv * g
        x_new = soft_threshold(z, tau * lam * wt * pinv)
        y = x_new + momentum(k) * (x_new - x)
        x_prev, x = x, x_new
        if callback is not None:
            callback(k, x)
    return x, x_prev, y


def ista(A, x0: np.ndarray, lam: float, tau: float, iters: int, x_init=None, p=None, w=None):
    """Proximal gradient without extrapolation (ISTA; the un-accelerated
    baseline of the preconditioner comparison, Sec. 5): x_k = S(x_{k-1} -
    tau g(x_{k-1}) / P) with threshold tau lam w / P."""
    x0 = np.asarray(x0, dtype=np.float64)
    N = A.shape[1]
    x = np.zeros(N) if x_init is None else np.asarray(x_init, dtype=np.float64).copy()
    At = A.T
    pinv = np.ones(N) if p is None else 1.0 / np.asarray(p, dtype=np.float64)
    wt = np.ones(N) if w is None else np.asarray(w, dtype=np.float64)
    for _ in range(iters):
        g = At @ (A @ x - x0)
        x = soft_threshold(x - tau * pinv * g, tau * lam * wt * pinv)
    return x


def objective(A, x0: np.ndarray, lam: float, x: np.ndarray, w=None) -> float:
    r = A @ x - x0
    wt = 1.0 if w is None else w
    return 0.5 * float(r @ r) + lam * float(np.sum(wt * np.abs(x)))


def duality_gap(A, x0: np.ndarray, lam: float, x: np.ndarray, w=None):
    """(E, D, gap, rel_gap).

    r = A x - x0.  The dual of the weighted problem is max -1/2 ||nu||^2 - <nu, x0>
    over |(A^T nu)_i| <= lam w_i; nu = s r with the largest s <= 1 that is
    feasible, s = min(1, lam / max_i(|(A^T r)_i| / w_i)), gives
    D(nu) = -1/2 s^2 ||r||^2 - s <r, x0> and gap = E - D >= 0 (weak duality).
    Uniform weights when w is None.
    """
    r = A @ x - x0
    wt = np.ones(A.shape[1]) if w is None else np.asarray(w, dtype=np.float64)
    E = 0.5 * float(r @ r) + lam * float(np.sum(wt * np.abs(x)))
    gmax = float(np.max(np.abs(A.T @ r) / wt)) if r.size else 0.0
    s = 1.0 if gmax <= lam else lam / gmax
    D = -0.5 * s * s * float(r @ r) - s * float(r @ x0)
    gap = E - D
    return E, D, gap, (gap / E if E > 0 else 0.0)


def kkt(A, x0: np.ndarray, lam: float, x: np.ndarray, w=None):
    """Violations of the l1 optimality conditions.

    Returns (max over i of |g_i| - lam w_i, clipped at 0, relative to lam;
    max over the support of |g_i + lam w_i sign(x_i)| relative to lam).
    """
    g = A.T @ (A @ x - x0)
    wt = np.ones_like(g) if w is None else w
    bound = np.maximum(np.abs(g) - lam * wt, 0.0).max(initial=0.0) / lam
    supp = x != 0
    eq = np.abs(g[supp] + lam * wt[supp] * np.sign(x[supp])).max(initial=0.0) / lam
    return bound, eq
