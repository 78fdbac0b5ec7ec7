"""Pins of the Alg. 3 oracle: for a convolution, Theta assembled from one
blurred atom per subband equals the definition Psi^* H Psi built densely."""
import numpy as np
import pytest

import synth
from oracle import filters, theta, theta_conv


@pytest.mark.parametrize("n,wavelet,levels,field", [
    (32, "haar", 3, ("iso", 1.5)),
    (32, "db4", 2, ("aniso", 2.5, 1.0, 0.6)),
    (64, "haar", 4, ("aniso", 3.0, 1.2, -1.1)),
])
def test_alg3_equals_dense_definition(n, wavelet, levels, field):
    h = filters.by_name(wavelet)
    f = synth.psf_stationary(n, field[1], field[1]) if field[0] == "iso" else synth.psf_stationary(n, *field[1:])
    T_dense = theta.theta_dense(f, h, levels)
    T_alg3 = theta_conv.theta_convolution(f, h, levels)
    assert np.max(np.abs(T_alg3 - T_dense)) <= 1e-12 * np.max(np.abs(T_dense))


def test_alg3_refuses_a_spatially_varying_field():
    with pytest.raises(ValueError):
        theta_conv.theta_convolution(synth.psf_isotropic(32, 1.0, 2.0), filters.haar(), 2)


def test_alg3_planted_shift_direction_is_caught():
    """Shifting the representative the wrong way (q + r m) must break the pin."""
    n, levels = 32, 2
    h = filters.haar()
    f = synth.psf_stationary(n, 2.0, 1.0, 0.4)
    T_dense = theta.theta_dense(f, h, levels)
    rows, _ = theta_conv.representatives(f, h, levels)
    from oracle import dwt
    bands = dwt.subbands(n, levels)
    _l, _e, offr, sr = bands[1]
    _l, _e, offc, sc = bands[-1]
    r = sc // sr
    rep = rows[1][offc:offc + sc * sc].reshape(sc, sc)
    wrong = np.roll(rep, (-r * 1, -r * 2), (0, 1)).ravel()
    right = np.roll(rep, (r * 1, r * 2), (0, 1)).ravel()
    row = offr + 1 * sr + 2
    assert np.allclose(right, T_dense[row, offc:offc + sc * sc], atol=1e-13)
    assert not np.allclose(wrong, T_dense[row, offc:offc + sc * sc], atol=1e-6)
