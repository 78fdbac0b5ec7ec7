"""GPU parity of the warm-start network kernels against the FP64 oracle, and
an end-to-end check that a trained network lowers the solver's iteration
count (the solver still runs to the same tolerance from the prediction)."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import blur, cnn as ocnn, dwt, filters, fista, theta

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def W():
    assert torch.cuda.is_available()
    from paper_1512_08401_amd import wdb
    return wdb


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("n,J", [(32, 2), (64, 2)])
def test_forward_and_gradient_match_oracle(W, n, J):
    """n = 32: stacks of side 8 (vector kernels) and 16 (matrix-core kernels,
    16-wide tiles); n = 64: every stack on the matrix cores, the 1-channel
    approximation stack included, with 32-wide tiles at side 32."""
    F = 32
    net = W.Cnn(n, J, F, seed=5)
    rng = np.random.default_rng(1)
    p = (rng.standard_normal(net.nparam) * 0.05).astype(np.float32)
    net.set_params(p)
    pr = net.get_params(rounded=True).astype(np.float64)     # the bfloat16 values the kernels use
    assert np.max(np.abs(pr - p)) <= 2.0 ** -8 * np.max(np.abs(p))
    B = 3
    x0 = rng.standard_normal((B, n * n)).astype(np.float32)
    tgt = rng.standard_normal((B, n * n)).astype(np.float32)
    pred = net.predict(dev(x0).reshape(-1)).cpu().numpy().reshape(B, -1)
    pred_o = ocnn.forward(pr, x0.astype(np.float64), n, J, F)
    assert np.max(np.abs(pred - pred_o)) <= 1e-5 * np.max(np.abs(pred_o))
    loss, g = net.loss_grad(dev(x0).reshape(-1), dev(tgt).reshape(-1))
    loss_o, g_o = ocnn.loss_and_grad(pr, x0.astype(np.float64), tgt.astype(np.float64), n, J, F)
    assert abs(loss - loss_o) <= 1e-6 * loss_o
    scale = np.max(np.abs(g_o))
    assert np.max(np.abs(g - g_o)) <= 1e-4 * scale
    # block by block (every W and b of every stack is exercised)
    pos = 0
    for shp in ocnn.param_shapes(n, J, F):
        k = int(np.prod(shp))
        blk, blk_o = g[pos:pos + k], g_o[pos:pos + k]
        assert np.linalg.norm(blk - blk_o) <= 1e-4 * max(np.linalg.norm(blk_o), 1e-3 * scale)
        pos += k


def test_adam_step_matches_closed_form(W):
    n, J, F = 32, 2, 32
    net = W.Cnn(n, J, F, seed=6)
    rng = np.random.default_rng(2)
    p = (rng.standard_normal(net.nparam) * 0.05).astype(np.float32)
    net.set_params(p)
    x0 = dev(rng.standard_normal((2, n * n))).reshape(-1)
    tgt = dev(rng.standard_normal((2, n * n))).reshape(-1)
    _, g = net.loss_grad(x0, tgt)
    net.train_step(x0, tgt, 1e-3)
    p1 = net.get_params()
    exp, _, _ = ocnn.adam_step(p.astype(np.float64), np.zeros(p.size), np.zeros(p.size), g.astype(np.float64), 1, 1e-3)
    assert np.max(np.abs(p1 - exp)) <= 1e-6


def test_trained_warm_start_reduces_iterations(W):
    """Train on targets the solver itself produces (64x64, Haar, 3 levels),
    then compare iterations to a relative objective of 1e-5,
    (E(x_k) - E*) / E(0) <= 1e-5, from the prediction and from zero on
    held-out images (checked after every iteration; E* from a long solve)."""
    n, J, lam = 64, 3, 2e-3
    field = synth.psf_isotropic(n, 1.0, 3.0)
    th = W.build_theta(field, "haar", J, 40 * n * n)
    th.lipschitz(synth.power_start(n * n, 3))
    H = blur.blur_matrix(field)

    def obs(seed):
        return (blur.blur(None, synth.piecewise_image(n, seed), H) + synth.noise(n, 0.01, seed + 7)).astype(np.float32)

    train_u = [dev(obs(1000 + i)).reshape(-1) for i in range(96)]
    test_u = [dev(obs(5000 + i)).reshape(-1) for i in range(16)]
    xs, _ = W.solve_batched([(th, u, lam) for u in train_u], 4000, check_every=50, tol=1e-5)
    X0 = torch.stack([W.dwt(u, "haar", J) for u in train_u])
    T = torch.stack(xs)
    net = W.Cnn(n, J, 32, seed=11)
    first = None
    for epoch in range(60):
        perm = torch.randperm(96, generator=torch.Generator().manual_seed(epoch))
        for b in range(0, 96, 16):
            idx = perm[b:b + 16].cuda()
            loss = net.train_step(X0[idx].reshape(-1).contiguous(), T[idx].reshape(-1).contiguous(), 2e-3)
            first = loss if first is None else first
    assert loss < 0.5 * first
    Xt = torch.stack([W.dwt(u, "haar", J) for u in test_u])
    pred = net.predict(Xt.reshape(-1).contiguous()).reshape(16, -1)
    _, star = W.solve_batched([(th, u, lam) for u in test_u], 6000, check_every=100, tol=1e-8)
    E0 = 0.5 * (Xt.double() ** 2).sum(dim=1).cpu().numpy()
    tgt = [star[i]["objective"] + 1e-5 * E0[i] for i in range(16)]
    _, cold = W.solve_batched([(th, u, lam, None, tgt[i]) for i, u in enumerate(test_u)], 4000, check_every=1)
    _, warm = W.solve_batched([(th, u, lam, pred[i].contiguous(), tgt[i]) for i, u in enumerate(test_u)], 4000,
                              check_every=1)
    it_cold = np.array([r["iters"] for r in cold])
    it_warm = np.array([r["iters"] for r in warm])
    print(f"iterations to rel. objective 1e-5: zero start {it_cold.mean():.1f}, warm start {it_warm.mean():.1f}")
    assert all(r["converged"] for r in warm) and all(r["converged"] for r in cold)
    assert it_warm.mean() < it_cold.mean()
