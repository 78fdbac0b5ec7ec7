"""The C-ABI library loads, exports every declared symbol, and its host-only
paths (filter derivation, argument validation) behave — no GPU needed."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wdb.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wdb_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1512_08401_amd import wdb
    return wdb._lib


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), f"{name} declared in wdb.h but not exported"


def test_library_filter_matches_published_table():
    from paper_1512_08401_amd import wavelet_filter
    vals = [float(l) for l in open(os.path.join(ROOT, "tests", "golden", "db4_daubechies_table.txt"))
            if l.strip() and not l.startswith("#")]
    assert np.max(np.abs(wavelet_filter("db4") - np.array(vals))) < 1e-13
    assert np.allclose(wavelet_filter("haar"), [2 ** -0.5] * 2, rtol=1e-15, atol=0)


def test_library_symlet_matches_oracle():
    """The library's Symmlet 6 (own root finder and phase criterion) equals the oracle's."""
    from paper_1512_08401_amd import wavelet_filter
    from oracle import filters
    h = wavelet_filter("sym6")
    assert len(h) == 12 and np.max(np.abs(h - filters.sym6())) < 1e-13


def test_wavelet_filter_honours_the_documented_capacity(lib):
    """The header's buffer contract: 12 doubles hold every filter (sym6 has 12
    taps); a smaller capacity is refused without writing past it, and a
    length query writes nothing."""
    from paper_1512_08401_amd import wdb
    pd = C.POINTER(C.c_double)
    ln = C.c_int32(-1)
    assert lib.wdb_wavelet_filter(wdb.WAVELETS["sym6"], None, 0, C.byref(ln)) == wdb.WDB_OK
    assert ln.value == 12
    buf = np.full(14, 7.0)          # 12 documented doubles plus two guard entries
    assert lib.wdb_wavelet_filter(wdb.WAVELETS["sym6"], buf.ctypes.data_as(pd), 12, C.byref(ln)) == wdb.WDB_OK
    assert ln.value == 12 and np.all(buf[12:] == 7.0) and abs(buf[:12].sum() - 2 ** 0.5) < 1e-14
    small = np.full(10, 7.0)
    assert lib.wdb_wavelet_filter(wdb.WAVELETS["sym6"], small.ctypes.data_as(pd), 8, C.byref(ln)) == wdb.WDB_ERR_ARG
    assert ln.value == 12 and np.all(small == 7.0)
    assert "12 taps" in lib.wdb_last_error().decode()
    for name, taps in (("haar", 2), ("db4", 8)):
        assert lib.wdb_wavelet_filter(wdb.WAVELETS[name], buf.ctypes.data_as(pd), 12, C.byref(ln)) == wdb.WDB_OK
        assert ln.value == taps


def test_host_validation_errors(lib):
    from paper_1512_08401_amd import wdb
    fake = C.c_void_p(16)   # never dereferenced: validation fails first
    h = np.zeros(8)
    ln = C.c_int32()
    assert lib.wdb_wavelet_filter(7, h.ctypes.data_as(C.POINTER(C.c_double)), 8, C.byref(ln)) == wdb.WDB_ERR_ARG
    assert "unknown wavelet" in lib.wdb_last_error().decode()
    assert lib.wdb_dwt(48, 0, 1, fake, C.c_void_p(32), 0, None) == wdb.WDB_ERR_SIZE
    assert lib.wdb_dwt(64, 1, 5, fake, C.c_void_p(32), 0, None) == wdb.WDB_ERR_LEVELS   # 64/16 < 8 taps
    assert lib.wdb_dwt(64, 0, 1, None, C.c_void_p(32), 0, None) == wdb.WDB_ERR_ARG
    assert lib.wdb_dwt(64, 0, 1, fake, fake, 0, None) == wdb.WDB_ERR_ARG                # aliasing
    assert lib.wdb_set_tile_values(None, 1) == wdb.WDB_ERR_ARG
    assert lib.wdb_set_tile_values(fake, 2) == wdb.WDB_ERR_ARG
    assert "kept values" in lib.wdb_last_error().decode()
    big = C.c_void_p(1 << 40)   # far from `fake`: the two batches do not overlap
    assert lib.wdb_dwt_batched(64, 0, 1, 0, fake, big, 0, None) == wdb.WDB_ERR_ARG        # count < 1
    assert lib.wdb_dwt_batched(64, 0, 1, 2, None, big, 0, None) == wdb.WDB_ERR_ARG        # null input
    assert lib.wdb_dwt_batched(48, 0, 1, 2, fake, big, 0, None) == wdb.WDB_ERR_SIZE
    assert lib.wdb_dwt_batched(64, 1, 5, 2, fake, big, 0, None) == wdb.WDB_ERR_LEVELS
    # out starts inside the input batch (two images of 64 x 64 floats)
    assert lib.wdb_dwt_batched(64, 0, 1, 2, fake, C.c_void_p(16 + 4 * 64 * 64), 0, None) == wdb.WDB_ERR_ARG
    assert "overlap" in lib.wdb_last_error().decode()
    out = C.c_void_p()
    rp = np.zeros(4 * 4 + 1, dtype=np.int64)
    rp[-1] = 1
    assert lib.wdb_theta_import(4, 0, 1, 1, C.c_void_p(rp.ctypes.data), None, None, None,
                                C.byref(out)) == wdb.WDB_ERR_ARG
    bad = np.zeros(17, dtype=np.int64)
    bad[5] = 3   # rowptr must end at nnz = 0
    assert lib.wdb_theta_import(4, 0, 1, 0, C.c_void_p(bad.ctypes.data), None, None, None,
                                C.byref(out)) == wdb.WDB_ERR_FORMAT
    col = np.array([2, 1], dtype=np.int32)          # not increasing
    val = np.array([1.0, 2.0])
    rp = np.zeros(17, dtype=np.int64)
    rp[1:] = 2
    assert lib.wdb_theta_import(4, 0, 1, 2, C.c_void_p(rp.ctypes.data), C.c_void_p(col.ctypes.data),
                                C.c_void_p(val.ctypes.data), None, C.byref(out)) == wdb.WDB_ERR_FORMAT
    val = np.array([1.0, np.nan])
    col = np.array([1, 2], dtype=np.int32)
    assert lib.wdb_theta_import(4, 0, 1, 2, C.c_void_p(rp.ctypes.data), C.c_void_p(col.ctypes.data),
                                C.c_void_p(val.ctypes.data), None, C.byref(out)) == wdb.WDB_ERR_NONFINITE


def test_psf_field_validation(lib):
    from paper_1512_08401_amd import wdb
    import synth
    f = synth.psf_isotropic(16, 1.0, 3.0)        # radius 8: 2*8+1 > 16
    st, keep = wdb._field_struct(f)
    out = C.c_void_p()
    assert lib.wdb_build_theta(C.byref(st), 0, 2, 100, None, C.byref(out)) == wdb.WDB_ERR_SIZE
    f = synth.psf_isotropic(32, 1.0, 2.0)
    f.sig_minor[3, 4] = np.nan
    st, keep = wdb._field_struct(f)
    assert lib.wdb_build_theta(C.byref(st), 0, 2, 100, None, C.byref(out)) == wdb.WDB_ERR_NONFINITE
    f = synth.psf_isotropic(32, 1.0, 2.0)
    st, keep = wdb._field_struct(f)
    assert lib.wdb_build_theta(C.byref(st), 0, 2, 0, None, C.byref(out)) == wdb.WDB_ERR_ARG
    assert lib.wdb_build_theta(C.byref(st), 1, 4, 100, None, C.byref(out)) == wdb.WDB_ERR_LEVELS
