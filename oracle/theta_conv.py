"""Theta of a convolution from one atom per subband, Alg. 3 (test oracle).

When H is a convolution (a stationary PSF field), the theorem of Sec. 3.6
makes every subband block of Theta a rectangular circulant matrix, so Theta
follows from the blurred atoms H psi and H^* psi of the atom at position 0 of
each subband: one forward wavelet transform each (Alg. 3).  In the orientation
of the matrix product (row a = analysis atom, column b = synthesised atom,
entry <psi_a, H psi_b>), for a row subband R of side s_R and a column subband
C of side s_C:

* s_C >= s_R (C at least as fine): translating psi_{R,0} by m positions of R
  translates the image by a multiple of C's spacing, so
      Theta[(R, m), (C, q)] = <H^* psi_{R,0}, psi_{C, q - r m}>,  r = s_C / s_R,
  the row of psi_{R,0} shifted by r m;
* s_C < s_R (C coarser):
      Theta[(R, m), (C, q)] = <psi_{R, m - r q}, H psi_{C,0}>,  r = s_R / s_C,
  the column of psi_{C,0} shifted by r q.

Shifts act on both axes of the subband and are periodic.  Everything is float64
and dense (small images only).
"""
from __future__ import annotations

import numpy as np

from . import blur as _blur
from . import dwt as _dwt


def is_stationary(field) -> bool:
    """True when every pixel carries the same PSF (H is a convolution)."""
    return all(float(np.ptp(a)) == 0.0 for a in (field.sig_major, field.sig_minor, field.angle))


def representatives(field, h: np.ndarray, levels: int, H=None):
    """For each subband k: (Psi^* H^* psi_k0, Psi^* H psi_k0), psi_k0 its atom at position 0."""
    n = field.n
    if H is None:
        H = _blur.blur_matrix(field)
    rows, cols = [], []
    for _lev, _e, off, _s in _dwt.subbands(n, levels):
        psi = _dwt.basis_image(n, h, levels, off)
        cols.append(_dwt.dwt2(_blur.blur(field, psi, H), h, levels))
        rows.append(_dwt.dwt2((H.T @ psi.ravel()).reshape(n, n), h, levels))
    return rows, cols


def theta_convolution(field, h: np.ndarray, levels: int, H=None) -> np.ndarray:
    """Dense Theta of a stationary field, assembled from the circulant blocks."""
    if not is_stationary(field):
        raise ValueError("Alg. 3 needs a convolution (the same PSF at every pixel)")
    n = field.n
    N = n * n
    bands = _dwt.subbands(n, levels)
    rows, cols = representatives(field, h, levels, H)
    T = np.zeros((N, N))
    for kr, (_lr, _er, offr, sr) in enumerate(bands):
        for kc, (_lc, _ec, offc, sc) in enumerate(bands):
            if sc >= sr:
                r = sc // sr
                rep = rows[kr][offc:offc + sc * sc].reshape(sc, sc)
                for m1 in range(sr):
                    for m2 in range(sr):
                        T[offr + m1 * sr + m2, offc:offc + sc * sc] = np.roll(rep, (r * m1, r * m2), (0, 1)).ravel()
            else:
                r = sr // sc
                rep = cols[kc][offr:offr + sr * sr].reshape(sr, sr)
                for q1 in range(sc):
                    for q2 in range(sc):
                        T[offr:offr + sr * sr, offc + q1 * sc + q2] = np.roll(rep, (r * q1, r * q2), (0, 1)).ravel()
    return T
