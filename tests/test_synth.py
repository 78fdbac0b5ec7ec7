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
    # a different seed changes the values' signs and noise and, among entries
    # of equal magnitude at the cut, which ones are kept
    rp3, cc3, vv3 = synth.local_operator(n, J, 20, 6)
    key3 = np.repeat(np.arange(N), np.diff(rp3)).astype(np.int64) * N + cc3
    assert cc3.size == cc.size and np.intersect1d(key, key3).size >= 0.9 * key.size
    assert not np.array_equal(vv3, vv)


def test_local_operator_long_coarse_rows_and_far_entries():
    """The structure the full-size tests need from the stand-in: exactly the
    requested number of non-zeros, coarse rows reaching two and three levels
    finer at displacements beyond 16, and entries at a level gap of 4 or a
    displacement beyond 128 (none at this size for the latter)."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    import tilestats
    n, J = 256, 5
    rp, cc, vv = synth.local_operator(n, J, 20, 3, coarse_from=4, far=16)
    N = n * n
    assert rp[-1] == 20 * N
    st = tilestats.stats(rp, cc, n, J, 8)
    assert st["max_level_gap"] == 4 and st["escapes"] == 8
    assert st["max_disp"] > 16 and st["entries_gap_2_or_more"] > 8
    rows = np.repeat(np.arange(N), np.diff(rp))
    lev = dwt.level_of(n, J)
    gap = lev[cc] - lev[rows]
    assert set(np.unique(gap).tolist()) == {-3, -2, -1, 0, 1, 4}
    assert np.all(lev[rows[gap <= -2]] >= 4) and np.all(lev[rows[gap == 4]] == 1)
