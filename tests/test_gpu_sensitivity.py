"""Points of the parameter sensitivity experiment (Sec. 5.4.3, Eq. 8) through
the GPU path against the oracle: a dense FP64 stream (I = J = K = 100, rank
5, 10 initial slices then batches of 10) for p = 3 (Eq. 8 fails, modes 1-2
under-determined) and p = 8 (Eq. 8 holds), Q = 20, S = 4, two seeds each.
The GPU fit equals the oracle's within 1e-8, and on these seeds the
determined setting fits better, the trend Eq. 8 predicts."""
import sys

import numpy as np
import pytest

from paper_1807_01350_amd import synth

pytestmark = pytest.mark.gpu

I = J = K = 100
R, SIGMA, T0, T = 5, 0.01, 10, 10


def _run(P, Q, S, cid, X):
    import torch
    from oracle import OctenOracle, fit_dense
    from paper_1807_01350_amd import octen as oc
    M1 = S + P * (Q - S)
    U, V = synth.compression_UV(I, J, P, Q, S, cid)
    init = synth.als_init(P, Q, R, cid)
    o = OctenOracle(I, J, R, P, Q, S, U, V)
    eng = oc.Octen(I, J, R, P, Q, S, torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda())
    outs = [torch.empty((n, R), dtype=torch.float64, device="cuda") for n in (I, J, K)]
    tX = torch.from_numpy(X).cuda()
    k0, b = 0, 0
    while k0 < K:
        t = T0 if b == 0 else T
        W = synth.temporal_W(t, M1, cid, b)
        o.compress_batch(X[k0:k0 + t], W); o.update_replicas()
        o.cp_als_replicas(30, init=init if b == 0 else None)
        Ao, Bo, Co = o.recover_factors()
        eng.compress_batch(tX[k0:k0 + t], torch.from_numpy(W).cuda())
        eng.update_replicas()
        eng.cp_als_replicas(30, init=torch.from_numpy(init).cuda() if b == 0 else None)
        eng.recover_factors(*outs)
        k0 += t
        b += 1
    sse, nx = eng.fit_terms(tX, 0, *outs)
    eng.close()
    return 1.0 - np.sqrt(sse / nx), fit_dense(X, Ao, Bo, Co)[0]


def test_sensitivity_points_match_oracle():
    _, _, _, X = synth.dense_stream(I, J, K, R, SIGMA, 5)
    fits = {}
    for P in (3, 8):
        for seed in (0, 1):
            g, o = _run(P, 20, 4, 500 + seed, X)
            print(f"[sens] p={P} seed={seed}: gpu {g:.6f} oracle {o:.6f}", file=sys.stderr,
                  flush=True)
            assert abs(g - o) <= 1e-8, (P, seed, g, o)
            fits.setdefault(P, []).append(o)
    assert min(fits[8]) > max(fits[3])
