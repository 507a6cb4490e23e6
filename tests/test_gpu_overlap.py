"""GPU: the overlapped compression (octen_compress_batch_async) gives the
same stream as the plain call order, bit for bit: the next batch's
compression runs on the handle's second stream while the current batch's
cooperative ALS and recovery run on the handle stream (Sec. 4.1 steps of
consecutive batches; only the compression is independent of the ALS)."""
import sys

import numpy as np
import pytest

from tests.stream_helpers import Case, make_inputs

pytestmark = pytest.mark.gpu

CASE = Case("overlap", 300, 280, 6, 12, 60, 3, (40, 10, 10, 10), iters=20, config_id=31)


def _run(form, overlap):
    import torch
    from paper_1807_01350_amd import octen as oc
    c = CASE
    X, U, V, Ws, init = make_inputs(c, x_dtype=np.float32)
    dev = "cuda"
    tX = torch.from_numpy(np.ascontiguousarray(X)).to(dev)
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    eng = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, torch.from_numpy(U).to(dev),
                   torch.from_numpy(V).to(dev), x_dtype="f32", compress_dtype=form)
    A = torch.empty((c.I, c.R), dtype=torch.float64, device=dev)
    B = torch.empty((c.J, c.R), dtype=torch.float64, device=dev)
    C = torch.empty((c.K, c.R), dtype=torch.float64, device=dev)
    tinit = torch.from_numpy(init).to(dev)
    offs = np.concatenate([[0], np.cumsum(c.batches)])
    xb = [tX[offs[b]:offs[b + 1]] for b in range(len(c.batches))]
    outs = []
    eng.compress_batch(xb[0], tW[0])
    eng.update_replicas()
    for b in range(len(c.batches)):
        print(f"[overlap] {form} overlap={overlap} batch {b}", file=sys.stderr, flush=True)
        last = b + 1 == len(c.batches)
        if overlap and not last:
            eng.compress_batch_async(xb[b + 1], tW[b + 1])
        eng.cp_als_replicas(c.iters, init=tinit if b == 0 else None)
        K = eng.recover_factors(A, B, C)
        torch.cuda.synchronize()
        outs.append(dict(F=eng.state(oc.OCTEN_STATE_FACTORS).cpu().numpy(),
                         A=A.cpu().numpy().copy(), B=B.cpu().numpy().copy(),
                         C=C[:K].cpu().numpy().copy()))
        if not last:
            if not overlap:
                eng.compress_batch(xb[b + 1], tW[b + 1])
            eng.update_replicas()
            outs[-1]["Y"] = eng.state(oc.OCTEN_STATE_Y).cpu().numpy()
    eng.close()
    return outs


@pytest.mark.parametrize("form", ["bf16", "f32"])
def test_overlapped_compression_is_bit_identical(form):
    seq = _run(form, False)
    ovl = _run(form, True)
    assert len(seq) == len(ovl)
    for b, (s, o) in enumerate(zip(seq, ovl)):
        for key in s:
            assert np.array_equal(s[key], o[key]), (form, b, key)


def test_overlapped_compression_state_reads_join():
    """A state read right after the overlapped call sees the new batch's Z
    (the handle stream waits for the second stream first)."""
    import torch
    from paper_1807_01350_amd import octen as oc
    c = CASE
    X, U, V, Ws, init = make_inputs(c, x_dtype=np.float32)
    dev = "cuda"
    tX = torch.from_numpy(np.ascontiguousarray(X)).to(dev)
    eng = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, torch.from_numpy(U).to(dev),
                   torch.from_numpy(V).to(dev), x_dtype="f32", compress_dtype="f32")
    t0, t1 = c.batches[0], c.batches[1]
    W1 = torch.from_numpy(Ws[1]).to(dev)
    eng.compress_batch(tX[t0:t0 + t1], W1)
    Zs = eng.state(oc.OCTEN_STATE_Z).cpu().numpy()
    eng.compress_batch(tX[:t0], torch.from_numpy(Ws[0]).to(dev))
    eng.compress_batch_async(tX[t0:t0 + t1], W1)
    Za = eng.state(oc.OCTEN_STATE_Z).cpu().numpy()
    assert np.array_equal(Zs, Za)
    eng.close()
