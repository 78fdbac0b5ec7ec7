"""Host-side checks of the tiled pattern storage, compiled from the library's
own sources (tests/native/tiles_host_check.cpp): tile cover, the XCD launch
order as a permutation, the shared group decode against the per-code decode
on every lane, and the tile product against the row-wise product (exact).
Runs on the CPU; needs hipcc to compile the sources that hold the kernels."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_tiled_storage_host_checks(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "tiles_host_check")
    cmd = [hipcc, "-x", "hip", "-O1", "-std=c++17", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "native", "tiles_host_check.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "all checks passed" in run.stdout
