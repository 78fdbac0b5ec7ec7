"""Structure statistics of a wavelet-domain sparse operator (test helper).

For every kept entry (a, b) of an N x N operator in the canonical subband
order (approximation first, then per level J..1 the orientations (0,1),
(1,0), (1,1)), this computes what decides how the tiled storage holds it:
the level gap dL = l_b - l_a, and the displacement (di, dj) of b's position
from the point of level l_b whose atom is centred nearest to a's atom
(atoms of level l at index i are centred at 2^l i + (L - 1)(2^l - 1)/2 for a
filter of length L), wrapped to [-s/2, s/2) on b's subband side s.  Rows are
grouped as the storage groups them (8 x 8 position blocks of a subband, or
a whole subband of side below 8) and the distinct (dL, band slot, di, dj)
per group are counted.  Written from the geometry of the transform, for the
tests that compare a stand-in operator's structure with a built one.
"""
from __future__ import annotations

import numpy as np


def positions(idx: np.ndarray, n: int, J: int):
    """(level, orientation 0..2 details / 3 approximation, i, j) of canonical indices."""
    idx = np.asarray(idx, dtype=np.int64)
    lsJ = int(np.log2(n)) - J
    level = np.empty(idx.shape, np.int64)
    orient = np.empty(idx.shape, np.int64)
    i = np.empty(idx.shape, np.int64)
    j = np.empty(idx.shape, np.int64)
    approx = idx < (1 << (2 * lsJ))
    level[approx] = J
    orient[approx] = 3
    i[approx] = idx[approx] >> lsJ
    j[approx] = idx[approx] & ((1 << lsJ) - 1)
    d = ~approx
    r = idx[d]
    ls = np.floor(np.log2(r.astype(np.float64))).astype(np.int64) // 2
    # guard float rounding of log2 on exact powers
    ls = np.where((np.int64(1) << (2 * (ls + 1))) <= r, ls + 1, ls)
    o = (r >> (2 * ls)) - 1
    p = r - (o + 1) * (np.int64(1) << (2 * ls))
    level[d] = int(np.log2(n)) - ls
    orient[d] = o
    i[d] = p >> ls
    j[d] = p & ((np.int64(1) << ls) - 1)
    return level, orient, i, j


def centre(i, la, lb, L1):
    return ((i << (la + 1)) + L1 * ((np.int64(1) << la) - (np.int64(1) << lb)) + (np.int64(1) << lb)) >> (lb + 1)


def entry_codes(rows, cols, n: int, J: int, taps: int):
    """Per entry: level gap, band slot of the column, displacements (di, dj)."""
    la, oa, ia, ja = positions(rows, n, J)
    lb, ob, ib, jb = positions(cols, n, J)
    L1 = taps - 1
    s = np.int64(n) >> lb
    h = s >> 1
    di = ((ib - centre(ia, la, lb, L1) + h) & (s - 1)) - h
    dj = ((jb - centre(ja, la, lb, L1) + h) & (s - 1)) - h
    slot = np.where(ob == 3, 0, ob + 1)
    return lb - la, slot, di, dj


def tile_of(rows, n: int, J: int):
    """Group id of each row: its subband and 8 x 8 block."""
    la, oa, ia, ja = positions(rows, n, J)
    band = np.where(oa == 3, 0, 1 + 3 * (J - la) + oa)
    side = np.int64(n) >> la
    small = side < 8
    bi = np.where(small, 0, ia >> 3)
    bj = np.where(small, 0, ja >> 3)
    return (band * (n // 8 + 1) + bi) * (n // 8 + 1) + bj, la


def stats(rowptr, col, n: int, J: int, taps: int, dmax: int = 128, gmax: int = 3):
    """Summary of an operator's structure as the tiled storage sees it."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    rows = np.repeat(np.arange(rowptr.size - 1, dtype=np.int64), np.diff(rowptr))
    col = np.asarray(col, dtype=np.int64)
    dL, slot, di, dj = entry_codes(rows, col, n, J, taps)
    esc = (np.abs(dL) > gmax) | (di < -dmax) | (di >= dmax) | (dj < -dmax) | (dj >= dmax)
    tid, la = tile_of(rows, n, J)
    ok = ~esc
    code = ((dL + 8) * 4 + slot) * (2 * n) ** 2 + (di + n) * (2 * n) + (dj + n)
    key = np.unique(np.stack([tid[ok], code[ok]]), axis=1)
    _, per_tile = np.unique(key[0], return_counts=True)
    coarse = la >= 3
    ckey = np.unique(np.stack([tid[ok & coarse], code[ok & coarse]]), axis=1)
    _, per_coarse = np.unique(ckey[0], return_counts=True) if ckey.size else (None, np.zeros(1, np.int64))
    return {
        "nnz": int(col.size),
        "max_level_gap": int(np.max(np.abs(dL))) if dL.size else 0,
        "max_disp": int(max(np.max(np.abs(di)), np.max(np.abs(dj)))) if di.size else 0,
        "entries_disp_over_16": int(np.sum((np.abs(di) > 16) | (np.abs(dj) > 16))),
        "entries_gap_2_or_more": int(np.sum(np.abs(dL) >= 2)),
        "escapes": int(np.sum(esc)),
        "max_codes_per_tile": int(per_tile.max()) if per_tile.size else 0,
        "max_codes_per_coarse_tile": int(per_coarse.max()),
        "stored_over_nnz": float(64 * per_tile.sum() / max(col.size, 1)),
    }
