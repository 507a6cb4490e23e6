"""The long-stream setting of the scalability experiment (Sec. 5.4.2): small
slices, many batches of 10 slices after an initial summary of 10 % of the
stream.  The FP64 path follows the oracle batch after batch (factors within
1e-10, the recovered C over all slices seen, the fit), and the same stream
stepped as a captured graph per batch (compress + update + ALS replayed)
gives exactly the eager results."""
import sys

import numpy as np
import pytest

from tests.stream_helpers import Case, make_inputs, rel

pytestmark = pytest.mark.gpu

CASE = Case("long20", 20, 20, 3, 2, 12, 3, (60,) + (10,) * 30, iters=20, config_id=61)


def test_long_stream_follows_oracle_and_graph_is_identical():
    import torch
    from oracle import OctenOracle, fit_dense
    from paper_1807_01350_amd import octen as oc
    c = CASE
    X, U, V, Ws, init = make_inputs(c)
    o = OctenOracle(c.I, c.J, c.R, c.P, c.Q, c.S, U, V)
    tU, tV = torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda()
    eager = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, tU, tV)
    graph = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, tU, tV, flags=oc.OCTEN_FLAG_ALS_ONE_WG)
    outs = {e: [torch.empty((n, c.R), dtype=torch.float64, device="cuda") for n in (c.I, c.J, c.K)]
            for e in ("eager", "graph")}
    tX = torch.from_numpy(X).cuda()
    tinit = torch.from_numpy(init).cuda()
    group = None
    xb = torch.empty((10, c.I, c.J), dtype=torch.float64, device="cuda")
    wb = torch.empty((10, c.M1), dtype=torch.float64, device="cuda")
    k0 = 0
    for b, t in enumerate(c.batches):
        tW = torch.from_numpy(Ws[b]).cuda()
        o.compress_batch(X[k0:k0 + t], Ws[b]); o.update_replicas()
        o.cp_als_replicas(c.iters, init=init if b == 0 else None)
        Ao, Bo, Co = o.recover_factors()
        eager.compress_batch(tX[k0:k0 + t], tW)
        eager.update_replicas()
        eager.cp_als_replicas(c.iters, init=tinit if b == 0 else None)
        K = eager.recover_factors(*outs["eager"])
        if b == 0:
            graph.compress_batch(tX[k0:k0 + t], tW)
            graph.update_replicas()
            graph.cp_als_replicas(c.iters, init=tinit)
            group = oc.Group([graph])
        else:
            xb.copy_(tX[k0:k0 + t])
            wb.copy_(tW)
            group.step([(xb, wb)], c.iters)
        assert graph.recover_factors(*outs["graph"]) == K == o.K
        k0 += t
        A, B, C = (x.cpu().numpy() for x in outs["eager"])
        C = C[:K]
        assert rel(A, Ao) <= 1e-10 and rel(B, Bo) <= 1e-10 and rel(C, Co) <= 1e-10, b
        if b > 0:
            # the eager cooperative ALS and the graph's one-workgroup ALS sum
            # in different orders: same results within FP64 rounding
            for x, y in zip(outs["eager"], outs["graph"]):
                assert rel(y[:K].cpu().numpy(), x[:K].cpu().numpy()) <= 1e-10, b
        sse, nx = eager.fit_terms(tX[:K], 0, *outs["eager"])
        fit = 1.0 - np.sqrt(sse / nx)
        fit_o = fit_dense(X[:K], Ao, Bo, Co)[0]
        assert abs(fit - fit_o) <= 1e-10, (b, fit, fit_o)
    print(f"[long] K={K} fit {fit:.6f}", file=sys.stderr, flush=True)
    group.close()
    eager.close()
    graph.close()
