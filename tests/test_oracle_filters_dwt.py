"""Pins for the oracle's filters and wavelet transform (CPU only).

Each check comes from the mathematics of orthogonal wavelets (Sec. 2: an
orthogonal basis on the torus, wavelets with M vanishing moments) or from a
published table, never from re-running the oracle's own formula.
"""
import math
import os

import numpy as np
import pytest

from oracle import dwt, filters

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_db4():
    vals = [float(l) for l in open(os.path.join(GOLDEN, "db4_daubechies_table.txt"))
            if l.strip() and not l.startswith("#")]
    return np.array(vals)


def test_haar_closed_form():
    assert np.allclose(filters.haar(), [1 / math.sqrt(2), 1 / math.sqrt(2)], atol=0, rtol=1e-15)


def test_db4_matches_published_table():
    assert np.max(np.abs(filters.db4() - _golden_db4())) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_daubechies_identities(p):
    h = filters.daubechies(p)
    L = len(h)
    assert L == 2 * p
    assert abs(h.sum() - math.sqrt(2)) < 1e-13
    # orthonormality of the even shifts: sum_m h[m] h[m + 2k] = delta_k
    for k in range(-(L // 2) + 1, L // 2):
        s = sum(h[m] * h[m + 2 * k] for m in range(L) if 0 <= m + 2 * k < L)
        assert abs(s - (1.0 if k == 0 else 0.0)) < 1e-13
    # p vanishing moments of the high-pass filter
    g = filters.highpass(h)
    for q in range(p):
        assert abs(sum(g[m] * m ** q for m in range(L))) < 1e-10 * max(1, L ** q)
    # minimum phase: every zero of H other than -1 lies inside the unit circle
    zeros = np.roots(h)
    others = zeros[np.abs(zeros + 1) > 1e-3]
    assert np.all(np.abs(others) < 1)


def _analysis_1d_matrix(M, f):
    """Periodic filter-and-downsample as an explicit (M/2) x M matrix."""
    D = np.zeros((M // 2, M))
    for i in range(M // 2):
        for m, fm in enumerate(f):
            D[i, (2 * i + m) % M] += fm
    return D


def _kron_analysis_matrix(n, h, J):
    """W assembled from Kronecker products of 1D level matrices and the layout."""
    g = filters.highpass(h)
    N = n * n
    W = np.zeros((N, N))
    # Running approximation operator (side m x m) as a matrix acting on images.
    A = np.eye(N)
    m = n
    blocks = {}
    for lev in range(1, J + 1):
        Lo, Hi = _analysis_1d_matrix(m, h), _analysis_1d_matrix(m, g)
        # image X (m x m): rows filtered by the left factor, columns by the right
        blocks[(lev, (0, 1))] = np.kron(Lo, Hi) @ A
        blocks[(lev, (1, 0))] = np.kron(Hi, Lo) @ A
        blocks[(lev, (1, 1))] = np.kron(Hi, Hi) @ A
        A = np.kron(Lo, Lo) @ A
        m //= 2
    off = 0
    W[off:off + A.shape[0]] = A
    off += A.shape[0]
    for lev in range(J, 0, -1):
        for e in ((0, 1), (1, 0), (1, 1)):
            B = blocks[(lev, e)]
            W[off:off + B.shape[0]] = B
            off += B.shape[0]
    return W


@pytest.mark.parametrize("name,n,J", [("haar", 8, 3), ("haar", 16, 2), ("db4", 16, 2), ("db4", 32, 3)])
def test_dwt_matches_kronecker_construction(name, n, J):
    h = filters.by_name(name)
    W = dwt.analysis_matrix(n, h, J)
    assert np.max(np.abs(W - _kron_analysis_matrix(n, h, J))) < 1e-13


@pytest.mark.parametrize("name,n,J", [("haar", 64, 3), ("db4", 32, 2), ("db4", 16, 1)])
def test_transform_is_orthogonal(name, n, J):
    h = filters.by_name(name)
    W = dwt.analysis_matrix(n, h, J)
    assert np.max(np.abs(W.T @ W - np.eye(n * n))) < 1e-12


@pytest.mark.parametrize("name,n,J", [("haar", 64, 3), ("db4", 64, 3), ("db4", 128, 4)])
def test_perfect_reconstruction_and_parseval(name, n, J):
    h = filters.by_name(name)
    u = np.random.default_rng(7).standard_normal((n, n))
    x = dwt.dwt2(u, h, J)
    assert abs(np.dot(x, x) - np.sum(u * u)) < 1e-10 * np.sum(u * u)
    assert np.max(np.abs(dwt.idwt2(x, h, J, n) - u)) < 1e-12


def test_haar_two_by_two_closed_form():
    a, b, c, d = 1.0, 2.0, 5.0, 11.0
    x = dwt.dwt2(np.array([[a, b], [c, d]]), filters.haar(), 1)
    expect = [(a + b + c + d) / 2, ((a - b) + (c - d)) / 2,    # A, e=(0,1)
              ((a + b) - (c + d)) / 2, ((a - b) - (c - d)) / 2]  # e=(1,0), e=(1,1)
    assert np.allclose(x, expect, rtol=0, atol=1e-14)


def test_vanishing_moments_kill_interior_polynomials():
    """Detail coefficients of a cubic vanish where the filter support does
    not straddle the periodic seam; the approximation of a constant is
    constant * 2^J."""
    n, J = 64, 2
    h = filters.db4()
    u = np.full((n, n), 3.0)
    x = dwt.dwt2(u, h, J)
    side = n >> J
    assert np.allclose(x[:side * side], 3.0 * 2 ** J, atol=1e-12)
    assert np.max(np.abs(x[side * side:])) < 1e-12
    t = np.arange(n, dtype=np.float64) / n
    poly = (0.3 + t - 2 * t ** 2 + 1.5 * t ** 3)[None, :].repeat(n, axis=0)
    x = dwt.dwt2(poly, h, 1)
    s = n // 2
    for _lev, e, off, sd in dwt.subbands(n, 1):
        if e == (0, 1):          # high-pass along columns: sensitive to the cubic
            band = x[off:off + sd * sd].reshape(sd, sd)
            interior = band[:, :s - 4]   # windows 2i..2i+7 that stay inside [0, n)
            assert np.max(np.abs(interior)) < 1e-12
            assert np.max(np.abs(band[:, s - 4:])) > 1e-3   # the seam is seen
        if e in ((1, 0), (1, 1)):
            assert np.max(np.abs(x[off:off + sd * sd])) < 1e-12


def test_planted_layout_mistake_is_caught(monkeypatch):
    """Swapping two detail subbands in the oracle breaks the Kronecker pin."""
    monkeypatch.setattr(dwt, "DETAIL_ORDER", ((1, 0), (0, 1), (1, 1)))
    h = filters.haar()
    W = dwt.analysis_matrix(8, h, 2)
    monkeypatch.undo()
    assert np.max(np.abs(W - _kron_analysis_matrix(8, h, 2))) > 0.1


def test_planted_highpass_sign_mistake_is_caught(monkeypatch):
    bad = lambda h: np.array([h[len(h) - 1 - m] for m in range(len(h))])  # sign dropped
    monkeypatch.setattr(dwt, "highpass", bad)
    h = filters.db4()
    W = dwt.analysis_matrix(16, h, 1)
    monkeypatch.undo()
    assert np.max(np.abs(W.T @ W - np.eye(256))) > 0.1
