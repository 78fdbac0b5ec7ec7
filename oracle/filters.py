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


def _zero_choices(p: int):
    """Roots of P(y) sorted by (real, imag) and, per root y, the reciprocal
    pair {z, 1/z} solving (2 - z - 1/z)/4 = y, inside-the-circle root first."""
    poly_y = np.array([math.comb(p - 1 + k, k) for k in range(p)], dtype=np.float64)
    y_roots = sorted(np.roots(poly_y[::-1]), key=lambda y: (round(y.real, 12), round(y.imag, 12)))
    pairs = []
    for y in y_roots:
        pr = np.roots([1.0, -(2.0 - 4.0 * y), 1.0])
        pr = sorted(pr, key=abs)
        pairs.append((y, pr[0], pr[1]))
    return pairs


def _filter_from_zeros(p: int, zs) -> np.ndarray:
    coeffs = np.array([1.0 + 0.0j])
    for _ in range(p):
        coeffs = np.convolve(coeffs, [1.0, 1.0])
    for zi in zs:
        coeffs = np.convolve(coeffs, [1.0, -zi])
    h = coeffs.real
    return h * (math.sqrt(2.0) / h.sum())


def phase_deviation(p: int, zs, grid: int = 2048) -> float:
    """Largest distance, over w in [0, pi], between the unwrapped phase of
    Q(w) = prod_i (1 - z_i e^{-iw}) and its chord from w = 0 to w = pi.  The
    factor (1 + e^{-iw})^p of m0 has exactly linear phase, so this measures how
    far the phase of m0 is from linear."""
    w = np.linspace(0.0, math.pi, grid + 1)
    e = np.exp(-1j * w)
    Q = np.ones_like(e)
    for zi in zs:
        Q = Q * (1.0 - zi * e)
    ph = np.unwrap(np.angle(Q))
    chord = ph[0] + (ph[-1] - ph[0]) * w / math.pi
    return float(np.max(np.abs(ph - chord)))


def symlet(p: int) -> np.ndarray:
    """Least-asymmetric ("Symmlet") filter with p vanishing moments (2p taps):
    the spectral factor of the same |m0|^2 as the Daubechies filter whose phase
    is closest to linear (Daubechies 1992, Sec. 8.1).  Each root y of P
    contributes z or 1/z (a complex-conjugate pair of roots the same choice for
    both, so h is real); among these choices the smallest phase_deviation wins,
    and of a choice and its mirror image (all zeros inverted: the time-reversed
    filter, same deviation) the one taking the inner zero for the first root in
    (real, imag) order."""
    if p == 1:
        return haar()
    pairs = _zero_choices(p)
    # group complex-conjugate y roots so that they share one choice
    groups, used = [], set()
    for i, (y, _, _) in enumerate(pairs):
        if i in used:
            continue
        grp = [i]
        if abs(y.imag) > 1e-12:
            for j in range(i + 1, len(pairs)):
                if j not in used and abs(pairs[j][0] - np.conj(y)) < 1e-9:
                    grp.append(j)
                    used.add(j)
                    break
        used.add(i)
        groups.append(grp)
    best, best_dev = None, None
    for mask in range(1 << len(groups)):
        if mask & 1:      # mirror images: keep the inner zero for the first group
            continue
        zs = []
        for gi, grp in enumerate(groups):
            for i in grp:
                zs.append(pairs[i][2] if (mask >> gi) & 1 else pairs[i][1])
        dev = phase_deviation(p, zs)
        if best_dev is None or dev < best_dev - 1e-12:
            best, best_dev = zs, dev
    return _filter_from_zeros(p, best)


def sym6() -> np.ndarray:
    """Symmlet with 6 vanishing moments (12 taps), the wavelet of Sec. 5."""
    return symlet(6)


def db4() -> np.ndarray:
    """Daubechies filter with 4 vanishing moments (8 taps)."""
    return daubechies(4)


def by_name(name: str) -> np.ndarray:
    if name == "haar":
        return haar()
    if name == "db4":
        return db4()
    if name == "sym6":
        return sym6()
    raise ValueError(f"unknown wavelet {name!r}")


def highpass(h: np.ndarray) -> np.ndarray:
    """Quadrature mirror high-pass g[m] = (-1)^m h[L-1-m]."""
    L = len(h)
    return np.array([(-1.0) ** m * h[L - 1 - m] for m in range(L)])
