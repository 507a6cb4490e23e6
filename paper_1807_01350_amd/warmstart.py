"""Training of the warm-start network with the library's own kernels.

Pairs (features of the previous replica columns and the sketch of the new
batch, the columns after ALS to a tight tolerance) come from running the
method itself through the C ABI; the network is then fitted with Adam by
octen_mlp_train_step.  torch only holds the tensors and draws minibatches.
"""
from __future__ import annotations

import numpy as np

from . import octen as oc


def collect_pairs(eng, batches, Ws, init, tol=1e-8, max_iters=500, first_iters=50):
    """Run one stream through compress -> update -> ALS and return the
    training pairs of every update batch.  eng: an Octen handle with a sketch
    set (octen_warmstart_set, network optional); batches: device slice
    tensors [t][I][J] (the first is the initial summary); Ws: device W rows
    per batch; init: device [P][3][Q][R] start of the first ALS."""
    feats, targs = [], []
    for b, (X, W) in enumerate(zip(batches, Ws)):
        eng.compress_batch(X, W)
        eng.update_replicas()
        if b == 0:
            eng.cp_als_replicas(first_iters, init=init)
            eng.cp_als_replicas(max_iters, tol=tol)
            continue
        feats.append(eng.warmstart_features())
        eng.cp_als_replicas(max_iters, tol=tol)
        targs.append(eng.warmstart_targets())
    return feats, targs


def train(mlp, X, T, steps, batch=512, lr=1e-3, seed=0, lr_final=None):
    """Adam on minibatches drawn uniformly without replacement per epoch;
    returns the loss of every step.  lr decays linearly to lr_final."""
    torch = mlp.torch
    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    n = X.shape[0]
    losses = []
    perm = torch.randperm(n, generator=g, device=X.device)
    pos = 0
    for s in range(steps):
        if pos + batch > n:
            perm = torch.randperm(n, generator=g, device=X.device)
            pos = 0
        idx = perm[pos:pos + min(batch, n)]
        pos += batch
        cur = lr if lr_final is None else lr + (lr_final - lr) * s / max(1, steps - 1)
        losses.append(mlp.train_step(X[idx].contiguous(), T[idx].contiguous(), cur))
    return np.array(losses)


def evaluate_loss(mlp, X, T):
    Y = mlp.forward(X)
    return float(((Y - T) ** 2).mean())
