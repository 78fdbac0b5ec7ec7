"""The Ritz step of the library's Lanczos estimate of ||Theta_K||^2 (host
code, tridiag.hpp): the largest eigenvalue of a symmetric tridiagonal matrix
and the last component of its unit eigenvector, against numpy's dense
symmetric eigensolver, on random, nearly diagonal and clustered spectra."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_top_ritz_matches_dense_eigensolver(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "tridiag_check")
    res = subprocess.run([gxx, "-O2", "-std=c++17", os.path.join(ROOT, "tests", "native", "tridiag_check.cpp"),
                          "-o", exe], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0
    lines = out.stdout.strip().splitlines()
    assert len(lines) == 21
    for line in lines:
        left, right = line.split("|")
        f = left.split()
        kind, m = int(f[0]), int(f[1])
        a = np.array([float(v) for v in f[2:2 + m]])
        b = np.array([float(v) for v in f[2 + m:]])
        theta, last = (float(v) for v in right.split())
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        w, V = np.linalg.eigh(T)
        spread = max(np.max(np.abs(w)), 1e-300)
        assert abs(theta - w[-1]) <= 1e-13 * spread, (kind, m, theta, w[-1])
        if m > 1 and w[-1] - w[-2] > 1e-8 * spread:   # the eigenvector is determined
            assert abs(abs(last) - abs(V[-1, -1])) <= 1e-6, (kind, m, last, V[-1, -1])
