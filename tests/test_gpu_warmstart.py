"""GPU checks of the learned warm start through the C ABI: network forward,
gradients and Adam against the FP64 oracle (BF16 products: 2e-2 normwise),
features, sketch, targets and the judge against the oracle on the same
factors, and the gain of a trained network over the plain warm start."""
import sys

import numpy as np
import pytest

from paper_1807_01350_amd import synth
from tests.stream_helpers import rel

pytestmark = pytest.mark.gpu


def _split(flat, n_in, n_h, n_out):
    from oracle.warmstart import mlp_param_shapes
    out, o = [], 0
    for shp in mlp_param_shapes(n_in, n_h, n_out):
        k = int(np.prod(shp))
        out.append(np.asarray(flat[o:o + k], np.float64).reshape(shp))
        o += k
    return out


def _net(n_in, n_h, n_out, cid, last_scale=0.5):
    import torch
    from paper_1807_01350_amd import octen as oc
    p = synth.mlp_params(n_in, n_h, n_out, cid, last_scale=last_scale)
    return oc.Mlp(n_in, n_h, n_out, torch.from_numpy(p).cuda()), p


DIMS = [(92, 64, 60, 37), (272, 256, 240, 320)]


@pytest.mark.parametrize("n_in,n_h,n_out,n", DIMS)
def test_forward_matches_oracle(n_in, n_h, n_out, n):
    """The network is a BF16 network: every product takes bfloat16 operands
    with float32 sums.  The oracle evaluates that definition (rounded
    operands, exact sums) from the same inputs: within 5e-4 normwise; the
    plain FP64 network is within 2e-2.  The bar: a hidden value lies within
    float32-summation distance (about 2^-24 sqrt(K) relative, K the inner
    length) of a bfloat16 rounding boundary with probability about
    2^-16 sqrt(K), and then rounds to the neighbouring bfloat16 value (2^-8
    relative) on one side only; over a layer that is 2^-8 sqrt(2^-16 sqrt(K))
    normwise, 6e-5 at K = 272, and two hidden layers feed the output."""
    import torch
    from oracle.precision import round_bf16
    from oracle.warmstart import mlp_forward
    net, p = _net(n_in, n_h, n_out, 31)
    X = np.random.default_rng(1).standard_normal((n, n_in)).astype(np.float32)
    Y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    params = _split(p, n_in, n_h, n_out)
    Yb, _ = mlp_forward(params, X, n_out, rnd=round_bf16)
    Yr, _ = mlp_forward(params, X, n_out)
    # compare the learned part (the residual is exact)
    assert rel(Y - X[:, :n_out], Yb - X[:, :n_out]) <= 5e-4
    assert rel(Y - X[:, :n_out], Yr - X[:, :n_out]) <= 2e-2
    assert np.array_equal(Y.shape, (n, n_out))
    net.close()


@pytest.mark.parametrize("n_in,n_h,n_out,n", DIMS)
def test_gradients_match_oracle(n_in, n_h, n_out, n):
    """Gradients of the mean squared error against the oracle's own forward
    and backward pass of the BF16 network (bfloat16 operands in every
    product, exact sums, rectifier masks from the oracle's forward): within
    1e-3 normwise per parameter array.  The GPU's loss is also within 1e-2 of
    the plain FP64 network's."""
    import torch
    from oracle.precision import round_bf16
    from oracle.warmstart import mlp_backward, mlp_forward, mse_loss
    net, p = _net(n_in, n_h, n_out, 32)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((n, n_in)).astype(np.float32)
    T = rng.standard_normal((n, n_out)).astype(np.float32)
    g, loss = net.gradients(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    params = _split(p, n_in, n_h, n_out)
    Yb, cache = mlp_forward(params, X, n_out, rnd=round_bf16)
    Lb, dY = mse_loss(Yb, T.astype(np.float64))
    gr = mlp_backward(params, cache, dY, rnd=round_bf16)
    assert abs(loss - Lb) <= 1e-5 * Lb
    Lx = mse_loss(mlp_forward(params, X, n_out)[0], T.astype(np.float64))[0]
    assert abs(loss - Lx) <= 1e-2 * Lx
    got = _split(g.cpu().numpy(), n_in, n_h, n_out)
    for name, a, b in zip(("W1", "b1", "W2", "b2", "W3", "b3"), got, gr):
        print(f"[warm] grad {name} rel {rel(a, b):.2e}", file=sys.stderr, flush=True)
        assert rel(a, b) <= 1e-3, (name, rel(a, b))
    net.close()


def test_adam_matches_oracle():
    import torch
    from oracle.warmstart import adam_step
    n_in, n_h, n_out = 40, 32, 30
    net, p = _net(n_in, n_h, n_out, 33)
    params = _split(p, n_in, n_h, n_out)
    m = [np.zeros_like(w) for w in params]
    v = [np.zeros_like(w) for w in params]
    rng = np.random.default_rng(3)
    for step in (1, 2, 3):
        gflat = rng.standard_normal(p.size).astype(np.float32)
        net.adam(torch.from_numpy(gflat).cuda(), 1e-3)
        adam_step(params, _split(gflat, n_in, n_h, n_out), m, v, step, 1e-3)
    got = net.params().cpu().numpy().astype(np.float64)
    want = np.concatenate([w.reshape(-1) for w in params])
    assert np.max(np.abs(got - want)) <= 2e-6
    net.close()


def test_training_fits_a_teacher():
    import torch
    from paper_1807_01350_amd import warmstart
    n_in, n_h, n_out, n = 92, 128, 60, 4096
    teacher, _ = _net(n_in, n_h, n_out, 34, last_scale=1.0)
    X = torch.randn((n, n_in), generator=torch.Generator(device="cuda").manual_seed(5),
                    device="cuda")
    T = teacher.forward(X)
    student, _ = _net(n_in, n_h, n_out, 35, last_scale=0.0)
    before = warmstart.evaluate_loss(student, X, T)
    losses = warmstart.train(student, X, T, steps=400, batch=512, lr=3e-3, seed=1)
    after = warmstart.evaluate_loss(student, X, T)
    print(f"[warmstart] teacher fit: loss {before:.4g} -> {after:.4g}", file=sys.stderr)
    assert np.all(np.isfinite(losses))
    assert after < 0.2 * before
    teacher.close()
    student.close()


def _small_stream(cid, batches=(30, 10, 10), I=60, J=55, R=4, P=4, Q=20, S=3):
    from tests.stream_helpers import Case, make_inputs
    c = Case(f"ws{cid}", I, J, R, P, Q, S, batches, iters=30, config_id=cid)
    X, U, V, Ws, init = make_inputs(c)
    return c, X, U, V, Ws, init


def test_features_targets_and_judge_match_oracle():
    """Features, sketch and targets from the GPU factors, and the choice of
    start, against the oracle fed the same factors and summaries."""
    import torch
    from oracle.warmstart import (candidate_init, judge, sketch, warmstart_features,
                                  warmstart_targets)
    from paper_1807_01350_amd import octen as oc
    c, X, U, V, Ws, init = _small_stream(41)
    D = 32
    G = synth.sketch_matrix(D, c.Q, 41)
    net, p = _net(4 * c.Q + D, 64, 3 * c.Q, 42, last_scale=0.3)
    eng = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, torch.from_numpy(U).cuda(),
                   torch.from_numpy(V).cuda())
    eng.warmstart_set(net, torch.from_numpy(G).cuda(), D)
    tX = torch.from_numpy(X).cuda()
    eng.compress_batch(tX[:30], torch.from_numpy(Ws[0]).cuda())
    eng.update_replicas()
    eng.cp_als_replicas(30, init=torch.from_numpy(init).cuda())
    F0 = eng.state(oc.OCTEN_STATE_FACTORS).cpu().numpy()
    lam0 = eng.state(oc.OCTEN_STATE_LAMBDA).cpu().numpy()
    eng.compress_batch(tX[30:40], torch.from_numpy(Ws[1]).cuda())
    Z = eng.state(oc.OCTEN_STATE_Z).cpu().numpy()
    eng.update_replicas()
    Ysum = eng.state(oc.OCTEN_STATE_Y).cpu().numpy()
    feats = eng.warmstart_features().cpu().numpy()
    sk = sketch(Z, G.astype(np.float64))
    fr, signs = warmstart_features(F0, lam0, sk, Z)
    assert rel(feats, fr) <= 1e-6
    # the signs are decided in FP64 on both sides: compare them exactly
    gsig = np.sign(feats[:, :3 * c.Q])
    osig = np.sign(fr[:, :3 * c.Q])
    assert np.array_equal(gsig[np.abs(fr[:, :3 * c.Q]) > 1e-6], osig[np.abs(fr[:, :3 * c.Q]) > 1e-6])
    # the learned start: network on the GPU features, judge on the oracle side
    Yn = net.forward(torch.from_numpy(feats).cuda()).cpu().numpy().astype(np.float64)
    cand = candidate_init(Yn, signs, c.Q)
    chosen, keep = judge(Ysum, cand, F0, lam0)
    eng.cp_als_replicas(1, learned=True)
    gkeep = eng.state(oc.OCTEN_STATE_WARM_KEEP).cpu().numpy()
    gfits = eng.state(oc.OCTEN_STATE_WARM_FITS).cpu().numpy()
    from oracle.warmstart import replica_fit_of
    c3 = np.cbrt(lam0)[:, None, :]
    ofits = np.array([[replica_fit_of(Ysum[q], *(F0[q] * c3[q][None])),
                       replica_fit_of(Ysum[q], *cand[q])] for q in range(c.P)])
    assert np.max(np.abs(gfits - ofits)) <= 1e-10
    margin = np.abs(ofits[:, 1] - ofits[:, 0])
    sure = margin > 1e-9
    assert np.array_equal(gkeep.astype(bool)[sure], keep[sure])
    # targets after a converged ALS, with the stored signs
    eng.cp_als_replicas(200, tol=1e-10)
    F1 = eng.state(oc.OCTEN_STATE_FACTORS).cpu().numpy()
    lam1 = eng.state(oc.OCTEN_STATE_LAMBDA).cpu().numpy()
    T = eng.warmstart_targets().cpu().numpy()
    assert rel(T, warmstart_targets(F1, lam1, signs)) <= 1e-6
    eng.close()
    net.close()


def test_trained_network_saves_sweeps():
    """What the trained network gains over the method without it: 24 small
    dense streams give the training pairs (ALS to 1e-8), 3 others are the
    test.  On the test streams the judged learned start must need fewer ALS
    sweeps to reach 1e-6 than the plain warm start and give a higher fit of
    the recovered factors after 5 sweeps; the untrained network (skip
    connection only) is reported alongside."""
    from paper_1807_01350_amd import warmstart
    c = dict(I=60, J=55, K=78, R=4, P=4, Q=20, S=3, batches=(30,) + (6,) * 8)
    res = warmstart.experiment(c, list(range(100, 124)), list(range(200, 203)), steps=800,
                               log=lambda m: print("[warmstart]", m, file=sys.stderr))
    sw = res["sweeps_total"]
    fb = res["fit_budget_mean"]
    assert res["loss_trained"] < 0.2 * res["loss_skip"]
    assert sw["trained"] < 0.9 * sw["plain"], sw
    assert fb[5]["trained"] > fb[5]["plain"], fb
    assert fb[20]["trained"] >= fb[20]["plain"], fb
