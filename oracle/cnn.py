"""FP64 reference of the warm-start network (test oracle; not in the paper).

The network maps x0 = Psi^* u (canonical coefficient layout) to a predicted
solution.  One stack per wavelet level: the coarsest approximation A_J (1
channel) and the detail subbands of levels J..1 (3 channels each, the three
subbands (0,1), (1,0), (1,1) in layout order, which is already channel-major).
Each stack, on a C-channel s x s input z:

    h1 = relu(conv(z; W1, b1))      C  -> F channels
    h2 = relu(conv(h1; W2, b2))     F  -> F
    out = z + conv(h2; W3, b3)      F  -> C   (residual)

conv is a 3x3 cross-correlation with circular padding (the coefficients live
on the torus):
    conv(z; W, b)[o, i, j] = b[o] + sum_{c, di, dj} W[o, c, di, dj] z[c, (i+di-1) mod s, (j+dj-1) mod s].
Loss: mean squared error over the batch and all N coefficients.

Parameters are flattened stack by stack (A_J, then levels J..1), each as
W1, b1, W2, b2, W3, b3 in C order.
"""
from __future__ import annotations

import numpy as np

from .dwt import subbands


def level_slices(n: int, levels: int):
    """(offset, channels, side) of each stack's input in the coefficient vector."""
    out = []
    bands = subbands(n, levels)
    out.append((bands[0][2], 1, bands[0][3]))
    for k in range(1, len(bands), 3):
        out.append((bands[k][2], 3, bands[k][3]))
    return out


def param_shapes(n: int, levels: int, F: int):
    shapes = []
    for _off, C, _s in level_slices(n, levels):
        shapes += [(F, C, 3, 3), (F,), (F, F, 3, 3), (F,), (C, F, 3, 3), (C,)]
    return shapes


def n_params(n, levels, F):
    return int(sum(np.prod(s) for s in param_shapes(n, levels, F)))


def unpack(theta: np.ndarray, n: int, levels: int, F: int):
    out, pos = [], 0
    for shp in param_shapes(n, levels, F):
        k = int(np.prod(shp))
        out.append(theta[pos:pos + k].reshape(shp))
        pos += k
    return out


def conv(z, W, b):
    """z: (B, C, s, s); W: (O, C, 3, 3) -> (B, O, s, s)."""
    out = np.zeros((z.shape[0], W.shape[0], z.shape[2], z.shape[3])) + b[None, :, None, None]
    for di in range(3):
        for dj in range(3):
            zs = np.roll(z, shift=(-(di - 1), -(dj - 1)), axis=(2, 3))
            out += np.einsum("oc,bcij->boij", W[:, :, di, dj], zs)
    return out


def conv_backward(z, W, g):
    """Gradients of sum(g * conv(z; W, b)) w.r.t. z, W, b."""
    gz = np.zeros_like(z)
    gW = np.zeros_like(W)
    for di in range(3):
        for dj in range(3):
            zs = np.roll(z, shift=(-(di - 1), -(dj - 1)), axis=(2, 3))
            gW[:, :, di, dj] = np.einsum("boij,bcij->oc", g, zs)
            gzs = np.einsum("oc,boij->bcij", W[:, :, di, dj], g)
            gz += np.roll(gzs, shift=(di - 1, dj - 1), axis=(2, 3))
    return gz, gW, g.sum(axis=(0, 2, 3))


def forward(theta, x0, n, levels, F, keep=False):
    """x0: (B, N) -> prediction (B, N); optional activations for backward."""
    params = unpack(theta, n, levels, F)
    B = x0.shape[0]
    pred = np.array(x0, dtype=np.float64, copy=True)
    acts = []
    for k, (off, C, s) in enumerate(level_slices(n, levels)):
        W1, b1, W2, b2, W3, b3 = params[6 * k:6 * k + 6]
        z = x0[:, off:off + C * s * s].reshape(B, C, s, s).astype(np.float64)
        a1 = conv(z, W1, b1)
        h1 = np.maximum(a1, 0)
        a2 = conv(h1, W2, b2)
        h2 = np.maximum(a2, 0)
        out = z + conv(h2, W3, b3)
        pred[:, off:off + C * s * s] = out.reshape(B, -1)
        acts.append((z, a1, h1, a2, h2))
    return (pred, acts) if keep else pred


def loss_and_grad(theta, x0, target, n, levels, F):
    """(MSE, gradient w.r.t. the flat parameter vector)."""
    B, N = x0.shape
    pred, acts = forward(theta, x0, n, levels, F, keep=True)
    diff = pred - target
    loss = float(np.sum(diff * diff)) / (B * N)
    gpred = 2.0 * diff / (B * N)
    params = unpack(theta, n, levels, F)
    grads = []
    for k, (off, C, s) in enumerate(level_slices(n, levels)):
        W1, b1, W2, b2, W3, b3 = params[6 * k:6 * k + 6]
        z, a1, h1, a2, h2 = acts[k]
        g = gpred[:, off:off + C * s * s].reshape(B, C, s, s)
        gh2, gW3, gb3 = conv_backward(h2, W3, g)
        ga2 = gh2 * (a2 > 0)
        gh1, gW2, gb2 = conv_backward(h1, W2, ga2)
        ga1 = gh1 * (a1 > 0)
        _, gW1, gb1 = conv_backward(z, W1, ga1)
        grads += [gW1, gb1, gW2, gb2, gW3, gb3]
    return loss, np.concatenate([g.ravel() for g in grads])


def adam_step(theta, m, v, grad, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
