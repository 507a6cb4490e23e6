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


def dense_stream_batches(torch, c, cid):
    """Seeded small dense stream (the synthetic protocol of the dense
    workloads) as device tensors: slices per batch, W rows, first init."""
    from . import synth
    A, B, C, X = synth.dense_stream(c["I"], c["J"], c["K"], c["R"], c.get("sigma", 0.01), cid,
                                    dtype=np.float32)
    U, V = synth.compression_UV(c["I"], c["J"], c["P"], c["Q"], c["S"], cid)
    M1 = c["S"] + c["P"] * (c["Q"] - c["S"])
    tX = torch.from_numpy(X).cuda()
    out, k0 = [], 0
    for b, t in enumerate(c["batches"]):
        out.append(tX[k0:k0 + t])
        k0 += t
    Ws = [torch.from_numpy(synth.temporal_W(t, M1, cid, b)).cuda()
          for b, t in enumerate(c["batches"])]
    init = torch.from_numpy(synth.als_init(c["P"], c["Q"], c["R"], cid)).cuda()
    return torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda(), out, Ws, init


def experiment(c, train_ids, test_ids, D=32, hidden=256, steps=600, lr=1e-3, tol=1e-6,
               max_iters=200, budgets=(5, 10, 20), log=None):
    """Train a warm-start network on streams train_ids and compare, on
    streams test_ids, three starts of every update's ALS: the plain warm
    start (previous factors), the untrained network (its skip connection
    alone: [a; b; c + u]) and the trained network, each judged against the
    plain start.  Reports ALS sweeps to reach tol and the fit of the
    recovered factors after fixed sweep budgets.  c: dict with I, J, K, R, P,
    Q, S, batches (dense FP32 streams, FP32 compression)."""
    import torch
    from . import synth
    Q, P, R = c["Q"], c["P"], c["R"]
    G = torch.from_numpy(synth.sketch_matrix(D, Q, 900)).cuda()
    n_in = 4 * Q + D

    def handle(U, V):
        return oc.Octen(c["I"], c["J"], R, P, Q, c["S"], U, V, x_dtype="f32", compress_dtype="f32")

    feats, targs = [], []
    for cid in train_ids:
        U, V, xs, Ws, init = dense_stream_batches(torch, c, cid)
        eng = handle(U, V)
        eng.warmstart_set(None, G, D)
        f, t = collect_pairs(eng, xs, Ws, init, tol=1e-8, max_iters=500)
        feats += f
        targs += t
        eng.close()
    Xtr = torch.cat(feats)
    Ttr = torch.cat(targs)
    p0 = torch.from_numpy(synth.mlp_params(n_in, hidden, 3 * Q, 901)).cuda()
    skip = oc.Mlp(n_in, hidden, 3 * Q, p0)
    net = oc.Mlp(n_in, hidden, 3 * Q, p0)
    base = evaluate_loss(net, Xtr, Ttr)
    ident = float(((Xtr[:, :3 * Q] - Ttr) ** 2).mean())
    train(net, Xtr, Ttr, steps, batch=min(512, Xtr.shape[0]), lr=lr, lr_final=lr / 10)
    trained = evaluate_loss(net, Xtr, Ttr)
    if log:
        log(f"training: {Xtr.shape[0]} pairs, loss {base:.4g} (skip only) -> {trained:.4g}")
    nets = {"plain": None, "skip": skip, "trained": net}
    res = {"pairs": int(Xtr.shape[0]), "loss_skip": base, "loss_trained": trained,
           "loss_previous_columns": ident,
           "sweeps": {k: [] for k in nets}, "kept": {k: 0 for k in nets}, "judged": 0,
           "fit_budget": {b: {k: [] for k in nets} for b in budgets}}
    A = torch.empty((c["I"], R), dtype=torch.float64, device="cuda")
    B = torch.empty((c["J"], R), dtype=torch.float64, device="cuda")
    C = torch.empty((c["K"], R), dtype=torch.float64, device="cuda")
    for cid in test_ids:
        U, V, xs, Ws, init = dense_stream_batches(torch, c, cid)
        engs = {}
        for run in ["tol"] + list(budgets):
            for k, m in nets.items():
                e = handle(U, V)
                e.warmstart_set(m, G, D)
                engs[(run, k)] = e
        for bi, (X, W) in enumerate(zip(xs, Ws)):
            for (run, k), e in engs.items():
                e.compress_batch(X, W)
                e.update_replicas()
                if bi == 0:
                    e.cp_als_replicas(50, init=init)
                    e.cp_als_replicas(500, tol=1e-8)
                    continue
                learned = nets[k] is not None
                if run == "tol":
                    it = e.cp_als_replicas(max_iters, tol=tol, learned=learned, want_iters=True)
                    res["sweeps"][k].append(int(it.sum()))
                    if learned:
                        res["kept"][k] += int(e.state(oc.OCTEN_STATE_WARM_KEEP).cpu().sum())
                    elif k == "plain":
                        res["judged"] += P
                else:
                    e.cp_als_replicas(run, learned=learned)
                    e.recover_factors(A, B, C)
                    sse, nx = e.fit_terms(torch.cat(xs[:bi + 1]), 0, A, B, C)
                    res["fit_budget"][run][k].append(1.0 - float(np.sqrt(sse / nx)))
        for e in engs.values():
            e.close()
    skip.close()
    net.close()
    res["sweeps_total"] = {k: int(sum(v)) for k, v in res["sweeps"].items()}
    res["kept_rate"] = {k: res["kept"][k] / max(1, res["judged"]) for k in nets if k != "plain"}
    res["fit_budget_mean"] = {b: {k: float(np.mean(v)) for k, v in res["fit_budget"][b].items()}
                              for b in budgets}
    if log:
        log(f"sweeps to tol {tol}: {res['sweeps_total']}; network start kept: {res['kept_rate']}; "
            f"fit after budgets: {res['fit_budget_mean']}")
    return res
