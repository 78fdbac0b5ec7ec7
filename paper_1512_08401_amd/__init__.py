"""MI355X-native wavelet-domain l1-l2 deblurring (Escande & Weiss).

The compute path is libwdb.so (HIP kernels for gfx950 behind the C ABI in
include/wdb.h); :mod:`paper_1512_08401_amd.wdb` is its ctypes binding.
"""
from .wdb import (Theta, WdbError, blur, build_theta, dwt, version, wavelet_filter,  # noqa: F401
                  LIB_PATH)
