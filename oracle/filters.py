"""Orthogonal wavelet filters (test oracle; see the package header).

The paper works with compactly supported orthogonal wavelets with M vanishing
moments (Sec. 2, definition of vanishing moments) and names Daubechies
wavelets (Sec. 3.5).  The Daubechies low-pass filter with p vanishing moments
is obtained here by spectral factorisation, in float64, with no typed-in
coefficient values:

    |m0(w)|^2 = cos(w/2)^(2p) * P(sin(w/2)^2),   P(y) = sum_{k<p} C(p-1+k, k) y^k,

and with y = (2 - z - 1/z)/4 each root of P gives a reciprocal pair of roots
in z; keeping the ones inside the unit circle (minimum phase) together with
the p-fold root at z = -1 and normalising sum(h) = sqrt(2) yields h.
"""
from __future__ import annotations

import math

import numpy as np


def haar() -> np.ndarray:
    """Haar low-pass filter h = [1, 1] / sqrt(2)."""
    return np.array([1.0, 1.0]) / math.sqrt(2.0)


def daubechies(p: int) -> np.ndarray:
    """Minimum-phase Daubechies low-pass filter with p vanishing moments (2p taps)."""
    if p == 1:
        return haar()
    # P(y) in ascending powers, then numpy.roots wants descending order.
    poly_y = np.array([math.comb(p - 1 + k, k) for k in range(p)], dtype=np.float64)
    y_roots = np.roots(poly_y[::-1])
    z_inside = []
    for y in y_roots:
        # (2 - z - 1/z)/4 = y  <=>  z^2 - (2 - 4y) z + 1 = 0
        pair = np.roots([1.0, -(2.0 - 4.0 * y), 1.0])
        z_inside.append(pair[np.argmin(np.abs(pair))])
    # H as a polynomial in w = z^{-1}: (1 + w)^p * prod (1 - z_i w)
    coeffs = np.array([1.0 + 0.0j])
    for _ in range(p):
        coeffs = np.convolve(coeffs, [1.0, 1.0])
    for zi in z_inside:
        coeffs = np.convolve(coeffs, [1.0, -zi])
    h = coeffs.real
    return h * (math.sqrt(2.0) / h.sum())


def db4() -> np.ndarray:
    """Daubechies filter with 4 vanishing moments (8 taps)."""
    return daubechies(4)


def by_name(name: str) -> np.ndarray:
    if name == "haar":
        return haar()
    if name == "db4":
        return db4()
    raise ValueError(f"unknown wavelet {name!r}")


def highpass(h: np.ndarray) -> np.ndarray:
    """Quadrature mirror high-pass g[m] = (-1)^m h[L-1-m]."""
    L = len(h)
    return np.array([(-1.0) ** m * h[L - 1 - m] for m in range(L)])
