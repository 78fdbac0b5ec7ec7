"""The seeded input generators: determinism and the structure the full-size
tests rely on (CPU only)."""
import numpy as np

import synth
from oracle import dwt


def test_local_operator_is_seeded_and_local():
    n, J = 64, 3
    rp, cc, vv = synth.local_operator(n, J, 20, 5)
    rp2, cc2, vv2 = synth.local_operator(n, J, 20, 5)
    assert np.array_equal(rp, rp2) and np.array_equal(cc, cc2) and np.array_equal(vv, vv2)
    N = n * n
    assert rp.size == N + 1 and rp[-1] == cc.size == vv.size
    assert abs(cc.size - 20 * N) <= 0.05 * 20 * N
    rows = np.repeat(np.arange(N), np.diff(rp))
    # sorted, unique columns per row; every row keeps its own coefficient
    key = rows.astype(np.int64) * N + cc
    assert np.all(np.diff(key) > 0)
    assert np.all(np.isin(np.arange(N, dtype=np.int64) * (N + 1), key))
    # entries couple subbands at most one level apart
    lev = dwt.level_of(n, J)
    assert np.all(np.abs(lev[rows] - lev[cc]) <= 1)
    # a different seed changes only the values' signs and noise
    rp3, cc3, vv3 = synth.local_operator(n, J, 20, 6)
    assert np.array_equal(cc3, cc) and not np.array_equal(vv3, vv)
    assert np.allclose(np.abs(vv3), np.abs(vv), rtol=0.5)
