"""Training loop for the warm-start network (loop control only: each step is
one wdb_cnn_train_step call that runs the forward, backward and Adam kernels).

The network predicts an initial iterate; the solver always runs from it to
its own tolerance, so the prediction can only change the iteration count.
"""
from __future__ import annotations


def train(net, X0, T, epochs: int, batch: int, lr: float, seed: int = 0, log=None, final_lr=None):
    """Adam on (X0, T) pairs (device tensors [count, N]); returns per-epoch mean
    losses.  With ``final_lr`` the step size follows a cosine from ``lr`` at the
    first step down to ``final_lr`` at the last."""
    import math
    import torch
    count = X0.shape[0]
    gen = torch.Generator().manual_seed(seed)
    per_epoch = max((count - batch) // batch + 1, 0)
    total = max(epochs * per_epoch - 1, 1)
    hist = []
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(count, generator=gen).to(X0.device)
        tot, steps = 0.0, 0
        for b in range(0, count - batch + 1, batch):
            idx = perm[b:b + batch]
            step_lr = lr
            if final_lr is not None:
                step_lr = final_lr + 0.5 * (lr - final_lr) * (1 + math.cos(math.pi * k / total))
            tot += net.train_step(X0[idx].reshape(-1).contiguous(), T[idx].reshape(-1).contiguous(), step_lr)
            steps += 1
            k += 1
        hist.append(tot / max(steps, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean training loss {hist[-1]:.4e}")
    return hist
