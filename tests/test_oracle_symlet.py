"""Pins of the Symmlet-6 oracle (the wavelet of the experiments of Sec. 5).
No published table is available here, so the filter is pinned by what
defines it: an orthonormal 12-tap filter with 6 vanishing moments whose
|m0|^2 is Daubechies' (it is a spectral factor of the same polynomial), and
whose phase is the closest to linear among all such factors, enumerated
independently below from the roots of |m0|^2 as a polynomial in z."""
import itertools
import math

import numpy as np

from oracle import dwt, filters


def test_sym6_is_orthonormal_with_six_vanishing_moments():
    h = filters.sym6()
    L = len(h)
    assert L == 12
    assert abs(h.sum() - math.sqrt(2.0)) <= 1e-14
    for k in range(L // 2):
        assert abs(np.dot(h[:L - 2 * k], h[2 * k:]) - (1.0 if k == 0 else 0.0)) <= 1e-14
    n = np.arange(L)
    for m in range(6):   # high-pass moments vanish <=> sum (-1)^n n^m h[n] = 0
        assert abs(np.sum((-1.0) ** n * n ** m * h)) <= 1e-9 * (L ** m)


def test_sym6_has_daubechies_magnitude_response():
    h, d = filters.sym6(), filters.daubechies(6)
    w = np.linspace(0, math.pi, 513)
    E = np.exp(-1j * np.outer(w, np.arange(12)))
    assert np.max(np.abs(np.abs(E @ h) - np.abs(E @ d))) <= 1e-12
    assert np.max(np.abs(h - d)) > 0.1    # but not the minimum-phase filter


def _phase_dev_of(h):
    """Deviation of the phase of m0 from linear, computed from the taps: divide
    the filter polynomial by (1 + z)^6 (exactly linear phase) and measure the
    unwrapped phase of the quotient against its chord over [0, pi]."""
    ones = np.array([1.0])
    for _ in range(6):
        ones = np.convolve(ones, [1.0, 1.0])
    q, rem = np.polydiv(np.asarray(h)[::-1], ones)   # polynomial in w = e^{-iw}, highest power first
    assert np.max(np.abs(rem)) <= 1e-10
    w = np.linspace(0, math.pi, 2049)
    Q = np.polyval(q, np.exp(-1j * w))
    ph = np.unwrap(np.angle(Q))
    chord = ph[0] + (ph[-1] - ph[0]) * w / math.pi
    return float(np.max(np.abs(ph - chord)))


def test_sym6_minimises_phase_nonlinearity_over_all_real_factors():
    """Enumerate the real spectral factors from the 20 zeros (other than z = -1)
    of the autocorrelation polynomial z^11 |m0|^2, one from each reciprocal pair."""
    d = filters.daubechies(6)
    auto = np.convolve(d, d[::-1])              # z^11 |m0(z)|^2 coefficients
    ones = np.array([1.0])
    for _ in range(12):
        ones = np.convolve(ones, [1.0, 1.0])
    quot, rem = np.polydiv(auto, ones)          # divide out the 12-fold zero at z = -1
    assert np.max(np.abs(rem)) <= 1e-10
    roots = np.roots(quot)
    inner = roots[np.abs(roots) < 1]            # 5 zeros inside the circle
    assert inner.size == 5
    # group conjugates
    groups, used = [], set()
    for i, z in enumerate(inner):
        if i in used:
            continue
        g = [i]
        for j in range(i + 1, inner.size):
            if j not in used and abs(inner[j] - np.conj(z)) < 1e-8 and abs(z.imag) > 1e-10:
                g.append(j)
                used.add(j)
                break
        used.add(i)
        groups.append(g)
    devs = []
    for choice in itertools.product((0, 1), repeat=len(groups)):
        zs = []
        for c, g in zip(choice, groups):
            zs += [inner[i] if c == 0 else 1 / inner[i] for i in g]
        poly = np.array([1.0 + 0j])
        for _ in range(6):
            poly = np.convolve(poly, [1.0, 1.0])
        for z in zs:
            poly = np.convolve(poly, [1.0, -z])
        h = poly.real * math.sqrt(2.0) / poly.real.sum()
        devs.append(_phase_dev_of(h))
    assert _phase_dev_of(filters.sym6()) <= min(devs) + 1e-6   # next best is above 0.6 rad
    assert _phase_dev_of(filters.daubechies(6)) > min(devs) + 1e-3


def test_sym6_transform_is_orthogonal_and_reconstructs():
    n, J = 64, 2
    h = filters.sym6()
    W = dwt.analysis_matrix(n, h, J)
    assert np.max(np.abs(W @ W.T - np.eye(n * n))) <= 1e-12
    u = np.random.default_rng(3).standard_normal((n, n))
    assert np.max(np.abs(dwt.idwt2(dwt.dwt2(u, h, J), h, J, n) - u)) <= 1e-12
