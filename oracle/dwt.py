"""Periodic separable 2D orthogonal wavelet transform (test oracle).

Follows the paper's basis (Sec. 2): tensor products of 1D scaling functions
and wavelets at the same scale on the torus (circular boundary conditions),
so the discrete transform is an orthogonal N x N matrix.

Conventions written out here (the paper fixes none of them):

* One analysis step along an axis of length M with filter f:
  out[i] = sum_m f[m] * x[(2 i + m) mod M],  i < M/2.
* A 2D level filters along columns (axis 1) then rows (axis 0).  Subband
  e = (e_row, e_col) uses the high-pass filter along the axes where e is 1.
* Coefficient vector layout ("canonical"): the coarsest approximation A_J,
  then for level l = J, J-1, ..., 1 the subbands e = (0,1), (1,0), (1,1),
  each row-major.  Level l subbands are (n / 2^l)^2; the paper's scale index
  is j = log2(n) - l (Sec. 2 numbers scales from coarse j = 0).
"""
from __future__ import annotations

import numpy as np

from .filters import highpass

DETAIL_ORDER = ((0, 1), (1, 0), (1, 1))


def check_sizes(n: int, flen: int, levels: int) -> None:
    if n < 2 or n & (n - 1):
        raise ValueError("image side must be a power of two")
    if levels < 1 or (n >> (levels - 1)) < max(flen, 2) or (n >> levels) < 1:
        raise ValueError("too many levels for this image side and filter length")


def subbands(n: int, levels: int):
    """List of (level, e, offset, side) in canonical order."""
    side = n >> levels
    out = [(levels, (0, 0), 0, side)]
    off = side * side
    for lev in range(levels, 0, -1):
        s = n >> lev
        for e in DETAIL_ORDER:
            out.append((lev, e, off, s))
            off += s * s
    return out


def analysis_step(x: np.ndarray, f: np.ndarray, axis: int) -> np.ndarray:
    M = x.shape[axis]
    i = np.arange(M // 2)
    out = None
    for m, fm in enumerate(f):
        term = fm * np.take(x, (2 * i + m) % M, axis=axis)
        out = term if out is None else out + term
    return out


def synthesis_step(c: np.ndarray, f: np.ndarray, axis: int) -> np.ndarray:
    """Transpose of :func:`analysis_step` (output length 2 * len along axis)."""
    half = c.shape[axis]
    M = 2 * half
    shape = list(c.shape)
    shape[axis] = M
    out = np.zeros(shape)
    i = np.arange(half)
    for m, fm in enumerate(f):
        idx = (2 * i + m) % M
        if axis == 0:
            np.add.at(out, (idx, slice(None)), fm * c)
        else:
            np.add.at(out, (slice(None), idx), fm * c)
    return out


def dwt2(u: np.ndarray, h: np.ndarray, levels: int) -> np.ndarray:
    """Forward transform x = Psi^* u of an n x n image; returns the canonical vector."""
    n = u.shape[0]
    check_sizes(n, len(h), levels)
    g = highpass(h)
    A = np.asarray(u, dtype=np.float64)
    details = {}
    for lev in range(1, levels + 1):
        lo = analysis_step(A, h, axis=1)
        hi = analysis_step(A, g, axis=1)
        details[(lev, (0, 1))] = analysis_step(hi, h, axis=0)
        details[(lev, (1, 0))] = analysis_step(lo, g, axis=0)
        details[(lev, (1, 1))] = analysis_step(hi, g, axis=0)
        A = analysis_step(lo, h, axis=0)
    parts = [A.ravel()]
    for lev in range(levels, 0, -1):
        for e in DETAIL_ORDER:
            parts.append(details[(lev, e)].ravel())
    return np.concatenate(parts)


def idwt2(x: np.ndarray, h: np.ndarray, levels: int, n: int) -> np.ndarray:
    """Inverse transform u = Psi x; ``x`` in canonical layout."""
    check_sizes(n, len(h), levels)
    g = highpass(h)
    bands = {}
    for lev, e, off, s in subbands(n, levels):
        bands[(lev, e)] = np.asarray(x[off:off + s * s], dtype=np.float64).reshape(s, s)
    A = bands[(levels, (0, 0))]
    for lev in range(levels, 0, -1):
        lo = synthesis_step(A, h, axis=0) + synthesis_step(bands[(lev, (1, 0))], g, axis=0)
        hi = synthesis_step(bands[(lev, (0, 1))], h, axis=0) + synthesis_step(bands[(lev, (1, 1))], g, axis=0)
        A = synthesis_step(lo, h, axis=1) + synthesis_step(hi, g, axis=1)
    return A


def analysis_matrix(n: int, h: np.ndarray, levels: int) -> np.ndarray:
    """Dense W (n^2 x n^2) with W @ u.ravel() == dwt2(u); column p = dwt2(e_p)."""
    N = n * n
    W = np.empty((N, N))
    e = np.zeros((n, n))
    for p in range(N):
        e.flat[p] = 1.0
        W[:, p] = dwt2(e, h, levels)
        e.flat[p] = 0.0
    return W


def basis_image(n: int, h: np.ndarray, levels: int, b: int) -> np.ndarray:
    """The synthesis atom psi_b = Psi e_b as an n x n image."""
    x = np.zeros(n * n)
    x[b] = 1.0
    return idwt2(x, h, levels, n)


def level_of(n: int, levels: int):
    """Per-coefficient level l (approximation gets ``levels``) in canonical order."""
    out = np.empty(n * n, dtype=np.int64)
    for lev, _e, off, s in subbands(n, levels):
        out[off:off + s * s] = lev
    return out


def scale_index(n: int, levels: int):
    """Per-coefficient scale j(i) = log2(n) - level in the paper's convention
    (a subband of scale j has 2^j x 2^j coefficients; the approximation has the
    scale of level J)."""
    return int(np.log2(n)) - level_of(n, levels)


def subband_of(n: int, levels: int):
    """Per-coefficient subband index (canonical order: 0 = A_J, then details)."""
    out = np.empty(n * n, dtype=np.int64)
    for k, (_lev, _e, off, s) in enumerate(subbands(n, levels)):
        out[off:off + s * s] = k
    return out
