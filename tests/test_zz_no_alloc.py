"""The transform entry point that allocates nothing (wdb_dwt_noalloc), called
through the C ABI, against wdb_dwt on the same inputs: bitwise equal outputs,
forward and inverse, on two calls in a row with the second on a smaller
image, and the size limit refused before any GPU work."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def W():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1512_08401_amd import wdb
    return wdb


def _call(W, fn, n, name, J, x, inverse):
    out = torch.full((n * n,), float("nan"), device="cuda", dtype=torch.float32)
    st = getattr(W._lib, fn)(n, W.WAVELETS[name], J, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                             int(inverse), None)
    assert st == W.WDB_OK, (fn, st, W._lib.wdb_last_error())
    torch.cuda.synchronize()
    return out


def test_noalloc_transform_matches_wdb_dwt(W):
    W._lib.wdb_dwt_noalloc.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                       C.c_void_p]
    W._lib.wdb_dwt_noalloc.restype = C.c_int
    for n, name, J in ((1024, "db4", 6), (256, "sym6", 4), (2048, "haar", 3), (64, "db4", 3)):
        print(f"no-alloc transform n={n} {name} J={J}", flush=True)
        x = torch.as_tensor(np.random.default_rng(n).standard_normal(n * n).astype(np.float32)).cuda()
        for inverse in (0, 1):
            a = _call(W, "wdb_dwt", n, name, J, x, inverse)
            b = _call(W, "wdb_dwt_noalloc", n, name, J, x, inverse)
            assert torch.equal(a, b), (n, name, J, inverse)
    big = torch.zeros(16, device="cuda")
    st = W._lib.wdb_dwt_noalloc(4096, W.WAVELETS["db4"], 3, C.c_void_p(big.data_ptr()),
                                C.c_void_p(big.data_ptr() + 64), 0, None)
    assert st == W.WDB_ERR_SIZE
    assert b"2048" in W._lib.wdb_last_error()
