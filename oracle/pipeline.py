"""End-to-end oracle runs on a named synthetic workload (test infrastructure).

Chains the oracle pieces in the order of the method: observation
u0 = H u + b (Sec. 1.1), x0 = Psi^* u0 and Theta_K (Sec. 1.3, Sec. 3.4,
Sec. 3.7), tau = 1/L (Alg. 1), then Alg. 1 iterations.
"""
from __future__ import annotations

import numpy as np

from . import blur, dwt, filters, fista, lipschitz, theta


def build_problem(wl, K=None, dense=True):
    """Everything the oracle needs for workload ``wl`` (a ``synth.Workload``).

    The observation is rounded to float32 (the GPU library consumes float32
    images), and every later oracle step works in float64 from that rounded
    image, so both sides solve the same problem.
    """
    n = wl.n
    h = filters.by_name(wl.wavelet)
    field = wl.psf()
    H = blur.blur_matrix(field)
    u = wl.image()
    u0 = blur.observe(field, u, wl.noise(), H).astype(np.float32)
    x0 = dwt.dwt2(u0.astype(np.float64), h, wl.levels)
    out = {"n": n, "h": h, "field": field, "H": H, "u": u, "u0": u0, "x0": x0}
    if dense:
        T = theta.theta_dense(field, h, wl.levels, H)
        rows, cols, vals = theta.top_k(T, wl.nnz if K is None else K)
        A = theta.to_csr(rows, cols, vals, n * n)
        out.update(T=T, A=A, thr=float(np.min(np.abs(vals))))
    return out


def solve(A, x0, lam, iters, start, x_init=None):
    """(x, L): Alg. 1 for ``iters`` iterations with tau = 1/L."""
    L, _ = lipschitz.lipschitz(A, start)
    x, _, _ = fista.fista(A, x0, lam, 1.0 / L, iters, x_init=x_init)
    return x, L
