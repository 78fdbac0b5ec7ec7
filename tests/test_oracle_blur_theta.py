"""Pins for the oracle's blur operator, Theta and thresholding (CPU only)."""
import math

import numpy as np
import pytest

import synth
from oracle import blur, dwt, filters, theta


def _const_field(n, sM, sm, ang, trunc=3.0):
    return synth.PsfField(n, np.full((n, n), sM), np.full((n, n), sm), np.full((n, n), ang), trunc)


@pytest.mark.parametrize("field", [synth.psf_isotropic(32), synth.psf_rotating(32, 4.0, 1.0)])
def test_blur_preserves_mass(field):
    H = blur.blur_matrix(field)
    assert np.max(np.abs(np.asarray(H.sum(axis=0)).ravel() - 1.0)) < 1e-14


@pytest.mark.parametrize("ang", [0.0, math.pi / 4, 2.0])
def test_psf_covariance_matches_rotated_axes(ang):
    """With a generous cut-off the discrete kernel's covariance is
    R(ang) diag(sM^2, sm^2) R(ang)^T, angle measured from x toward y."""
    sM, sm = 3.0, 2.0
    dy, dx, w = blur.psf_offsets(sM, sm, ang, trunc=9.0)
    cxx = np.sum(w * dx * dx)
    cyy = np.sum(w * dy * dy)
    cxy = np.sum(w * dx * dy)
    c, s = math.cos(ang), math.sin(ang)
    exx = sM ** 2 * c * c + sm ** 2 * s * s
    eyy = sM ** 2 * s * s + sm ** 2 * c * c
    exy = (sM ** 2 - sm ** 2) * c * s
    assert abs(cxx - exx) < 1e-8 and abs(cyy - eyy) < 1e-8 and abs(cxy - exy) < 1e-8
    assert abs(np.sum(w * dx)) < 1e-12 and abs(np.sum(w * dy)) < 1e-12


def test_constant_field_is_circular_convolution():
    n = 32
    f = _const_field(n, 2.5, 1.2, 0.7)
    H = blur.blur_matrix(f)
    dy, dx, w = blur.psf_offsets(2.5, 1.2, 0.7, 3.0)
    ker = np.zeros((n, n))
    np.add.at(ker, (dy % n, dx % n), w)
    u = np.random.default_rng(3).standard_normal((n, n))
    conv = np.real(np.fft.ifft2(np.fft.fft2(ker) * np.fft.fft2(u)))
    assert np.max(np.abs(blur.blur(f, u, H) - conv)) < 1e-12


def test_columns_carry_the_source_psf():
    """Column convention: column s of H is the PSF of source s."""
    n = 32
    f = synth.psf_isotropic(n, 1.0, 3.0)
    H = blur.blur_matrix(f).tocsc()
    for (r, c) in [(5, 2), (17, 29)]:
        s = r * n + c
        col = H[:, s].toarray().ravel().reshape(n, n)
        dy = ((np.arange(n) - r + n // 2) % n - n // 2)[:, None]
        dx = ((np.arange(n) - c + n // 2) % n - n // 2)[None, :]
        var_x = float(np.sum(col * dx * dx))
        _, ddx, w = blur.psf_offsets(f.sig_major[r, c], f.sig_minor[r, c], 0.0, 3.0)
        assert abs(var_x - np.sum(w * ddx * ddx)) < 1e-12
        # the row-convention operator would give the target's PSF instead
        row = H[s, :].toarray().ravel().reshape(n, n)
        assert abs(float(np.sum(row * dx * dx)) - var_x) > 1e-3


@pytest.fixture(scope="module")
def tiny_varying():
    n, J = 16, 2
    h = filters.db4()
    f = synth.psf_rotating(n, 2.0, 1.0)
    H = blur.blur_matrix(f)
    W = dwt.analysis_matrix(n, h, J)
    return n, J, h, f, H, W, theta.theta_dense(f, h, J, H, W)


def test_theta_is_similar_to_H(tiny_varying):
    n, J, h, f, H, W, T = tiny_varying
    Hd = H.toarray()
    assert abs(np.linalg.norm(T) - np.linalg.norm(Hd)) < 1e-12
    ev_t = np.sort_complex(np.linalg.eigvals(T))
    ev_h = np.sort_complex(np.linalg.eigvals(Hd))
    assert np.max(np.abs(ev_t - ev_h)) < 1e-9
    assert abs(np.linalg.norm(T, 2) - np.linalg.norm(Hd, 2)) < 1e-12


def test_theta_entries_are_atom_inner_products(tiny_varying):
    n, J, h, f, H, W, T = tiny_varying
    rng = np.random.default_rng(0)
    for a, b in rng.integers(0, n * n, size=(12, 2)):
        assert abs(T[a, b] - theta.theta_entry(f, h, J, int(a), int(b), H)) < 1e-14
    col = theta.theta_column(f, h, J, 37, H)
    assert np.max(np.abs(col - T[:, 37])) < 1e-14
    # a varying blur is not symmetric, so the index order matters
    assert np.max(np.abs(T - T.T)) > 1e-3


def test_identity_blur_gives_identity():
    n = 16
    f = _const_field(n, 0.2, 0.2, 0.0)
    T = theta.theta_dense(f, filters.db4(), 2)
    assert np.max(np.abs(T - np.eye(n * n))) < 1e-13


@pytest.mark.parametrize("name,J", [("haar", 3), ("db4", 2)])
def test_convolution_subbands_are_circulant(name, J):
    """Theorem of Sec. 3.6: every subband block of Theta is circulant when H
    is a convolution; a varying field breaks it."""
    n = 32
    h = filters.by_name(name)
    bands = dwt.subbands(n, J)

    def max_defect(T):
        worst = 0.0
        for (_la, _ea, oa, sa) in bands:
            for (_lb, _eb, ob, sb) in bands:
                B = T[oa:oa + sa * sa, ob:ob + sb * sb]
                if sb >= sa:
                    r = sb // sa
                    base = B[0].reshape(sb, sb)
                    for p in range(sa):
                        for q in range(sa):
                            shifted = np.roll(base, (r * p, r * q), axis=(0, 1))
                            worst = max(worst, np.max(np.abs(B[p * sa + q].reshape(sb, sb) - shifted)))
                else:
                    r = sa // sb
                    base = B[:, 0].reshape(sa, sa)
                    for p in range(sb):
                        for q in range(sb):
                            shifted = np.roll(base, (r * p, r * q), axis=(0, 1))
                            worst = max(worst, np.max(np.abs(B[:, p * sb + q].reshape(sa, sa) - shifted)))
        return worst

    T = theta.theta_dense(_const_field(n, 2.0, 1.0, 0.5), h, J)
    assert max_defect(T) < 1e-13
    Tv = theta.theta_dense(synth.psf_isotropic(n, 1.0, 3.0), h, J)
    assert max_defect(Tv) > 1e-4


def test_symmetric_psf_gives_symmetric_theta():
    T = theta.theta_dense(_const_field(16, 1.5, 1.5, 0.0), filters.db4(), 2)
    assert np.max(np.abs(T - T.T)) < 1e-14


def test_top_k_against_brute_force():
    rng = np.random.default_rng(5)
    T = rng.standard_normal((20, 20))
    T[rng.random((20, 20)) < 0.3] = 0.0
    T[3, 4], T[7, 1], T[2, 9] = 0.5, -0.5, 0.5          # an exact tie
    for K in [1, 17, 100, 280, 400]:
        rows, cols, vals = theta.top_k(T, K)
        items = sorted(((-abs(T[a, b]), a * 20 + b) for a in range(20) for b in range(20) if T[a, b] != 0))
        keep = sorted(idx for _, idx in items[:K])
        assert list(rows * 20 + cols) == keep
        assert np.all(vals == T[rows, cols])
    rows, cols, _ = theta.top_k(T, 10_000)
    assert rows.size == np.count_nonzero(T)


def test_top_k_tie_break_prefers_smaller_linear_index():
    T = np.zeros((4, 4))
    T[0, 3] = T[1, 0] = T[2, 2] = T[3, 1] = 1.0
    rows, cols, _ = theta.top_k(T, 2)
    assert list(zip(rows, cols)) == [(0, 3), (1, 0)]


def test_thresholded_theta_properties(tiny_varying):
    n, J, h, f, H, W, T = tiny_varying
    K = 10 * n * n
    rows, cols, vals = theta.top_k(T, K)
    assert rows.size == K
    kept = np.zeros_like(T, dtype=bool)
    kept[rows, cols] = True
    assert np.min(np.abs(T[kept])) >= np.max(np.abs(T[~kept]))
    assert np.sum(vals ** 2) <= np.linalg.norm(H.toarray()) ** 2 + 1e-12
