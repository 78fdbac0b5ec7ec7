"""Spatially varying blur H (test oracle).

Sec. 3.1 models blur as an integral operator whose kernel K(., y) is the PSF
at location y: column s of H is the (discrete) PSF of source pixel s,

    H[i, s] = k_s(i - s),   offsets taken modulo n on each axis (torus, Sec. 2).

k_s is a Gaussian with covariance R(angle) diag(sig_major^2, sig_minor^2)
R(angle)^T, with the angle turning the major axis from the column (x) axis
toward the row (y) axis, cut off where the Mahalanobis distance exceeds
``trunc`` and normalised to unit sum (so H preserves mass).  For an offset
d = (dy, dx) (rows, columns):

    t1 = dx cos(angle) + dy sin(angle),  t2 = -dx sin(angle) + dy cos(angle),
    q  = t1^2 / sig_major^2 + t2^2 / sig_minor^2,   weight ~ exp(-q / 2) if q <= trunc^2.

Offsets are searched in the box |dy|, |dx| <= floor(trunc * max(sig)), which
contains every offset with q <= trunc^2.  The field must not wrap a PSF onto
itself: 2 * radius + 1 <= n.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def psf_offsets(sig_major: float, sig_minor: float, angle: float, trunc: float):
    """Integer offsets (dy, dx) and normalised weights of one truncated PSF."""
    R = int(math.floor(trunc * max(sig_major, sig_minor)))
    dy, dx = np.meshgrid(np.arange(-R, R + 1, dtype=np.float64),
                         np.arange(-R, R + 1, dtype=np.float64), indexing="ij")
    c, s = math.cos(angle), math.sin(angle)
    t1 = dx * c + dy * s
    t2 = -dx * s + dy * c
    q = t1 * t1 / (sig_major * sig_major) + t2 * t2 / (sig_minor * sig_minor)
    keep = q <= trunc * trunc
    w = np.exp(-0.5 * q[keep])
    return dy[keep].astype(np.int64), dx[keep].astype(np.int64), w / w.sum()


def field_radius(field) -> int:
    return int(math.floor(field.trunc * float(max(np.max(field.sig_major), np.max(field.sig_minor)))))


def blur_matrix(field) -> sp.csc_matrix:
    """H as a sparse n^2 x n^2 matrix (pixel index = row * n + col)."""
    n = field.n
    if 2 * field_radius(field) + 1 > n:
        raise ValueError("PSF support wraps around the torus")
    rows, cols, vals = [], [], []
    cache = {}
    for r in range(n):
        for c in range(n):
            key = (float(field.sig_major[r, c]), float(field.sig_minor[r, c]), float(field.angle[r, c]))
            if key not in cache:          # many sources share one PSF
                cache[key] = psf_offsets(*key, field.trunc)
            dy, dx, w = cache[key]
            rows.append(((r + dy) % n) * n + (c + dx) % n)
            cols.append(np.full(w.size, r * n + c, dtype=np.int64))
            vals.append(w)
    N = n * n
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def blur(field, u: np.ndarray, H=None) -> np.ndarray:
    """Hu for an n x n image (returns n x n)."""
    if H is None:
        H = blur_matrix(field)
    return (H @ np.asarray(u, dtype=np.float64).ravel()).reshape(u.shape)


def observe(field, u: np.ndarray, b: np.ndarray, H=None) -> np.ndarray:
    """Observation u0 = H u + b (Sec. 1.1)."""
    return blur(field, u, H) + b
