"""MI355X-native wavelet-domain l1-l2 deblurring (Escande & Weiss).

The compute path is libwdb.so (HIP kernels for gfx950 behind the C ABI in
include/wdb.h); :mod:`paper_1512_08401_amd.wdb` is its ctypes binding.  The
binding is loaded on first use of an attribute (so the build script can run
before the library exists); loading fails loudly if libwdb.so is missing.
"""

_EXPORTS = ("Theta", "WdbError", "blur", "build_theta", "dwt", "version", "wavelet_filter", "LIB_PATH")


def __getattr__(name):
    if name in _EXPORTS:
        from . import wdb
        return getattr(wdb, name)
    raise AttributeError(name)
