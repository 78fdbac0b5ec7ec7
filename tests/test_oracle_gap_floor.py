"""Why a float32 iterate cannot certify small duality gaps (CPU, oracle only).

The stopping test scores an iterate by the Lasso duality gap (the textbook
dual point s r with s = min(1, lambda / ||Theta_K^T r||_inf); not in the
paper, which stops on E - E*, Sec. 5.5).  Rounding a coefficient of size |x_i|
to float32 moves it by up to |x_i| 2^-24, and Theta_K^T Theta_K passes that
to the gradient, so |(Theta_K^T r)_i| exceeds lambda by about
max|x| 2^-24 / lambda in relative terms; the dual scaling s then shrinks by
as much and the gap grows by about that factor times lambda ||x||_1.  The
approximation coefficients reach 2^J times the image mean, so with the
workloads' lambda this floor sits far above 1e-6.  Here the converged float64
solution of a small problem certifies a tiny gap while its float32 rounding
certifies one hundreds of times larger: the reason the library carries an
anchored iterate (float64 anchor, float32 displacement).
"""
import numpy as np
import scipy.sparse as sp

import synth
from oracle import blur, dwt, filters, fista, lipschitz, theta


def test_float32_rounding_of_a_converged_iterate_raises_the_gap():
    n, J, lam = 32, 2, 1e-3
    h = filters.db4()
    field = synth.psf_rotating(n, 2.0, 1.0)
    T = theta.theta_dense(field, h, J)
    r, c, v = theta.top_k(T, 20 * n * n)
    A = sp.csr_matrix((v, (r, c)), shape=(n * n, n * n))
    u0 = blur.observe(field, synth.piecewise_image(n, 1), synth.noise(n, 0.01, 2))
    x0 = dwt.dwt2(u0, h, J)
    L, _ = lipschitz.lipschitz(A, synth.power_start(n * n, 3))
    x, _, _ = fista.fista(A, x0, lam, 1.0 / L, 20000)
    E, D, gap, rel = fista.duality_gap(A, x0, lam, x)
    assert 0.0 <= rel <= 1e-7                         # float64 iterate: converged
    x32 = x.astype(np.float32).astype(np.float64)
    rel32 = fista.duality_gap(A, x0, lam, x32)[3]
    assert rel32 >= 100.0 * max(rel, 1e-8)            # its float32 rounding: far above
    # the size of the effect: the rounding moves the gradient by ~max|x| 2^-24,
    # a relative excess over lambda of that order
    g32 = A.T @ (A @ x32 - x0)
    excess = np.max(np.abs(g32)) / lam - 1.0
    scale = np.max(np.abs(x)) * 2.0 ** -24 / lam
    assert 0.1 * scale <= excess <= 10.0 * scale
    # the objective itself barely moves: the floor is in the certificate
    assert abs(fista.objective(A, x0, lam, x32) - E) <= 1e-9 * E
