"""Pins for the oracle's warm-start network (CPU only): central finite
differences for every parameter block, the circular convolution against an
FFT, identity at zero weights, and the Adam step against its closed form."""
import numpy as np
import pytest

from oracle import cnn


def test_level_slices_cover_the_layout():
    sl = cnn.level_slices(32, 2)
    assert [(o, c, s) for o, c, s in sl] == [(0, 1, 8), (64, 3, 8), (256, 3, 16)]
    assert sum(c * s * s for _, c, s in sl) == 32 * 32


def test_conv_is_circular_correlation():
    rng = np.random.default_rng(0)
    z = rng.standard_normal((2, 3, 8, 8))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = cnn.conv(z, W, b)
    # FFT: correlation with a kernel placed at offsets (di-1, dj-1)
    for o in range(4):
        acc = np.full((2, 8, 8), b[o])
        for c in range(3):
            ker = np.zeros((8, 8))
            for di in range(3):
                for dj in range(3):
                    ker[(1 - di) % 8, (1 - dj) % 8] = W[o, c, di, dj]
            acc += np.real(np.fft.ifft2(np.fft.fft2(z[:, c]) * np.fft.fft2(ker)[None]))
        assert np.max(np.abs(out[:, o] - acc)) < 1e-12


def test_zero_weights_give_identity():
    n, J, F = 16, 1, 4
    x0 = np.random.default_rng(1).standard_normal((3, n * n))
    assert np.array_equal(cnn.forward(np.zeros(cnn.n_params(n, J, F)), x0, n, J, F), x0)


def test_gradient_by_central_differences():
    n, J, F = 16, 1, 4
    rng = np.random.default_rng(2)
    P = cnn.n_params(n, J, F)
    theta = rng.standard_normal(P) * 0.3
    x0 = rng.standard_normal((2, n * n))
    tgt = rng.standard_normal((2, n * n))
    loss, g = cnn.loss_and_grad(theta, x0, tgt, n, J, F)
    idx = np.concatenate([np.arange(0, P, max(1, P // 60)), [P - 1]])
    for i in idx:
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp = cnn.loss_and_grad(tp, x0, tgt, n, J, F)[0]
        lm = cnn.loss_and_grad(tm, x0, tgt, n, J, F)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_planted_relu_mistake_is_caught():
    n, J, F = 16, 1, 4
    rng = np.random.default_rng(3)
    P = cnn.n_params(n, J, F)
    theta = rng.standard_normal(P) * 0.3
    x0, tgt = rng.standard_normal((1, n * n)), rng.standard_normal((1, n * n))
    orig = np.maximum
    try:
        cnn.np.maximum = lambda a, b: a            # relu dropped in the forward pass only
        loss_bad, _ = cnn.loss_and_grad(theta, x0, tgt, n, J, F)
    finally:
        cnn.np.maximum = orig
    loss, g = cnn.loss_and_grad(theta, x0, tgt, n, J, F)
    assert abs(loss_bad - loss) > 1e-6


def test_adam_closed_form_first_step():
    g = np.array([0.5, -2.0, 0.0])
    th, m, v = cnn.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 0.1)
    # after one step m_hat = g, v_hat = g^2: update = -lr * g / (|g| + eps)
    assert np.allclose(th, [-0.1, 0.1, 0.0], atol=1e-8)
