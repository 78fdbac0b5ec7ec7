"""Pins for the oracle's 16-bit storage rule (CPU only)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import quant
from oracle.dwt import subband_of


def _bf16_bruteforce(x):
    """Nearest bfloat16 by comparing the two neighbours (ties: even mantissa)."""
    out = []
    for v in np.asarray(x, dtype=np.float32):
        b = int(np.array([v], dtype=np.float32).view(np.uint32)[0])
        lo = b & 0xFFFF0000
        hi = lo + 0x10000
        flo = float(np.array([lo], dtype=np.uint32).view(np.float32)[0])
        fhi = float(np.array([hi], dtype=np.uint32).view(np.float32)[0])
        dlo, dhi = abs(float(v) - flo), abs(fhi - float(v))
        if dlo < dhi or (dlo == dhi and ((lo >> 16) & 1) == 0):
            out.append(flo)
        else:
            out.append(fhi)
    return np.array(out)


def test_bf16_rounding_matches_bruteforce():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(2000).astype(np.float32),
                        np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 3.0, 1e-30], dtype=np.float32)])
    assert np.array_equal(quant.round_bf16(x), _bf16_bruteforce(x))
    # halfway between 1 and 1 + 2^-7: ties to the even mantissa (1.0)
    assert quant.round_bf16(np.array([1.0 + 2 ** -8], dtype=np.float32))[0] == 1.0
    assert quant.round_bf16(np.array([1.0 + 3 * 2 ** -8], dtype=np.float32))[0] == 1.0 + 2 ** -6


def _toy(n=16, J=2, seed=3):
    rng = np.random.default_rng(seed)
    N = n * n
    A = sp.random(N, N, density=0.02, random_state=rng, format="csr")
    A.data = rng.standard_normal(A.nnz) * np.exp(rng.uniform(-8, 0, A.nnz))
    return A


@pytest.mark.parametrize("fmt,rel", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_quantisation_error_bound_and_scales(fmt, rel):
    n, J = 16, 2
    A = _toy(n, J)
    u = quant.band_scales(A, n, J)
    mant, ex = np.frexp(u)
    assert np.all(mant == 0.5)                      # powers of two
    Q = quant.quantize(A, n, J, fmt)
    v32 = A.data.astype(np.float32).astype(np.float64)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    ub = u[subband_of(n, J)[rows]]
    scaled = np.abs(v32 * ub)
    # the largest scaled value of each band lies in [1, 2)
    for band in np.unique(subband_of(n, J)[rows]):
        m = scaled[subband_of(n, J)[rows] == band].max()
        assert 1.0 <= m < 2.0
    err = np.abs(Q.data - v32)
    normal = scaled >= 2.0 ** -14
    assert np.all(err[normal] <= rel * np.abs(v32[normal]))
    if fmt == "f16":                                 # subnormal range: absolute half-ulp bound
        assert np.all(err[~normal] <= 2.0 ** -25 / ub[~normal])
    assert np.array_equal(Q.indices, A.indices) and np.array_equal(Q.indptr, A.indptr)


def test_exact_values_survive():
    n, J = 8, 1
    N = n * n
    A = sp.csr_matrix((np.array([0.75, -0.5, 0.375, 1.5]), (np.array([0, 1, 20, 63]), np.array([3, 4, 5, 6]))),
                      shape=(N, N))
    for fmt in ("f16", "bf16"):
        assert np.array_equal(quant.quantize(A, n, J, fmt).data, A.data)
