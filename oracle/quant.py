"""16-bit storage of Theta_K's values (test oracle for the mixed-precision form).

Not in the paper (it states no GPU precision).  Rule, written from its
definition:

1. each kept value is first rounded to float32 (the solver's storage);
2. every block of Theta_K gets a power-of-two scale that depends on the row
   subband A only: u_A = 2^(-floor(log2 m_A)), m_A the largest |value| in the
   rows of subband A (u_A = 1 for an empty subband), so the largest scaled
   value of the subband lies in [1, 2);
3. the scaled value v * u_A (exact: a power-of-two scaling) is rounded to the
   16-bit format with round-to-nearest-even: IEEE binary16 ("f16") or bfloat16
   ("bf16", the upper half of a float32);
4. the dequantised value is q / u_A (exact).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .dwt import subband_of


def round_bf16(x32: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); returns float64."""
    bits = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def band_scales(A: sp.csr_matrix, n: int, levels: int) -> np.ndarray:
    """u_A per row subband (canonical order)."""
    A = sp.csr_matrix(A)
    v32 = np.abs(A.data.astype(np.float32)).astype(np.float64)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    band = subband_of(n, levels)[rows]
    nb = int(subband_of(n, levels).max()) + 1
    m = np.zeros(nb)
    np.maximum.at(m, band, v32)
    u = np.ones(nb)
    nz = m > 0
    mant, ex = np.frexp(m[nz])          # m = mant * 2^ex, mant in [0.5, 1)
    u[nz] = np.ldexp(1.0, -(ex - 1))    # 2^-floor(log2 m)
    return u


def quantize(A: sp.csr_matrix, n: int, levels: int, fmt: str) -> sp.csr_matrix:
    """Theta_K with every value replaced by its dequantised 16-bit form."""
    A = sp.csr_matrix(A, copy=True)
    A.sort_indices()
    u = band_scales(A, n, levels)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    ub = u[subband_of(n, levels)[rows]]
    s32 = (A.data.astype(np.float32).astype(np.float64) * ub).astype(np.float32)   # exact scaling
    if fmt == "f16":
        q = s32.astype(np.float16).astype(np.float64)
    elif fmt == "bf16":
        q = round_bf16(s32)
    else:
        raise ValueError(fmt)
    A.data = q / ub
    return A
