"""Wavelet representation Theta of the blur and its K-sparse thresholding (test oracle).

* Sec. 3.4 defines the discrete operator as Theta = Psi^* H Psi.  With the
  analysis matrix W (so Psi^* = W, Psi = W^T) this is W H W^T, and entry
  (a, b) is <psi_a, H psi_b>: row a indexes the analysis (output) atom and
  column b the synthesised (input) atom.  (The entry-wise definition in
  Sec. 3.2 writes the two atoms the other way round; the matrix product is
  what enters the approximate problem of Sec. 1.3, so it is the one used.)
* Sec. 3.7, naive rule: keep the K entries of largest magnitude.  The paper
  does not say how equal magnitudes at the cut are ordered; here the smaller
  linear index a * N + b wins.  If Theta has fewer than K non-zeros all of
  them are kept.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import dwt as _dwt
from . import blur as _blur


def theta_dense(field, h: np.ndarray, levels: int, H=None, W=None) -> np.ndarray:
    """Full Theta = W H W^T for small images (n^2 <= 4096)."""
    n = field.n
    if W is None:
        W = _dwt.analysis_matrix(n, h, levels)
    if H is None:
        H = _blur.blur_matrix(field)
    return W @ np.asarray(H @ W.T)


def theta_column(field, h: np.ndarray, levels: int, b: int, H=None) -> np.ndarray:
    """Column b of Theta computed as Psi^* (H psi_b) with explicit atoms."""
    n = field.n
    psi_b = _dwt.basis_image(n, h, levels, b)
    return _dwt.dwt2(_blur.blur(field, psi_b, H), h, levels)


def theta_entry(field, h: np.ndarray, levels: int, a: int, b: int, H=None) -> float:
    """Single entry <psi_a, H psi_b> from explicit atom images."""
    n = field.n
    psi_a = _dwt.basis_image(n, h, levels, a)
    psi_b = _dwt.basis_image(n, h, levels, b)
    return float(np.sum(psi_a * _blur.blur(field, psi_b, H)))


def top_k_weighted(T: np.ndarray, K: int, sigma: np.ndarray):
    """Weighted thresholding of Sec. 3.7: keep the K entries whose
    |sigma_b Theta[a, b]| are largest (sigma on the column, i.e. the input
    coefficient the operator acts on; ties: smaller linear index first);
    the kept values are Theta's own.  Returns (rows, cols, vals) by (row, col)."""
    S = np.abs(T) * np.asarray(sigma, dtype=np.float64)[None, :]
    flat = S.ravel()
    nz = int(np.count_nonzero(flat))
    K = min(int(K), nz)
    order = np.argsort(-flat, kind="stable")[:K]
    order.sort()
    N = T.shape[1]
    rows = order // N
    cols = order % N
    return rows, cols, T.ravel()[order]


def column_scale_weights(n: int, levels: int) -> np.ndarray:
    """sigma_b = 2^-k for a column b of paper scale k (Sec. 3.7)."""
    return 2.0 ** (-_dwt.scale_index(n, levels).astype(np.float64))


def top_k(T: np.ndarray, K: int):
    """Keep the K largest |T| (ties: smaller linear index first).

    Returns (rows, cols, vals) of the kept entries sorted by (row, col).
    """
    flat = np.abs(T).ravel()
    nz = int(np.count_nonzero(flat))
    K = min(int(K), nz)
    order = np.argsort(-flat, kind="stable")[:K]
    order.sort()
    N = T.shape[1]
    rows = order // N
    cols = order % N
    return rows.astype(np.int64), cols.astype(np.int64), T.ravel()[order]


def threshold_value(T: np.ndarray, K: int) -> float:
    """Magnitude of the K-th kept entry."""
    flat = np.sort(np.abs(T).ravel())[::-1]
    return float(flat[min(K, flat.size) - 1])


def to_csr(rows, cols, vals, N: int) -> sp.csr_matrix:
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def csr_arrays(A: sp.csr_matrix):
    """(rowptr int64, col int32, val float64) with sorted column indices."""
    A = A.tocsr()
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64)
