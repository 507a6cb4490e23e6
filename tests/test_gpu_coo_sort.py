"""Sparse batches that do not arrive in (k, i, j) order (the sparse input of
Sec. 4.1): the library sorts them on the device (stable radix sort) before
the segments and the compression.  Against the oracle on the same
unordered input: the segments of the sorted batch bit-exact
(oracle.sort_coo then oracle.coo_segments), the compressed batch within the
bars of the ordered path (FP64 1e-12, FP32 1e-5).  With unique coordinates
the sorted batch is unique, so an unordered batch gives exactly the ordered
batch's results."""
import sys

import numpy as np
import pytest

from paper_1807_01350_amd import synth
from tests.stream_helpers import rel
from tests.test_gpu_parity_coo import CASES, CooCase, _dev, _engine

pytestmark = pytest.mark.gpu

SORT_CASES = CASES + [
    # several sort tiles (4096 entries each) and a ragged last one, the
    # sparse workload's mode sizes
    CooCase("wide_1e5", 100_000, 100_000, 6, 2, 20, 3, 4, 6000, 27),
    # one slice
    CooCase("one_slice", 500, 400, 4, 2, 12, 2, 1, 3000, 28),
]


def _shuffle(c, x, seed):
    order = np.random.Generator(np.random.PCG64(seed)).permutation(x[0].size)
    return [a[order].copy() for a in x]


def _gpu(c, U, V, W, form, k, i, j, v):
    from paper_1807_01350_amd import octen as oc
    eng = _engine(c, U, V, form)
    tk, ti, tj, tv, tW = _dev(k, i, j, v, W)
    eng.compress_batch_coo(tk, ti, tj, tv, c.t, tW)
    Z = eng.state(oc.OCTEN_STATE_Z).cpu().numpy()
    segs = [x.cpu().numpy() for x in eng.coo_segments()]
    eng.close()
    return Z, segs


@pytest.mark.parametrize("c", SORT_CASES, ids=[c.name for c in SORT_CASES])
def test_unordered_batch(c):
    from oracle import compress_coo, coo_segments, sort_coo
    print(f"[coo-sort] case {c.name}", file=sys.stderr, flush=True)
    k, i, j, v, U, V, W = c.inputs()
    ks, is_, js, vs = _shuffle(c, (k, i, j, v), 7 + c.cid)
    assert k.size > 1 and not all(np.array_equal(a, b) for a, b in ((ks, k), (is_, i), (js, j)))
    ref_segs = coo_segments(*sort_coo(ks, is_, js, vs)[:2], c.t)
    Zref = compress_coo(ks, is_, js, vs, c.t, U, V, W, c.P, c.Q, c.S)
    for form, bar in (("f64", 1e-12), ("f32", 1e-5)):
        Z, segs = _gpu(c, U, V, W, form, ks, is_, js, vs)
        for got, want in zip(segs, ref_segs):
            assert np.array_equal(got.astype(np.int64), want), (form, got[:8], want[:8])
        assert rel(Z, Zref) <= bar, (form, rel(Z, Zref))
        if not c.dup:
            # unique coordinates: the sorted batch is the ordered batch
            Z0, _ = _gpu(c, U, V, W, form, k, i, j, v)
            assert np.array_equal(Z, Z0), form


def test_duplicates_keep_input_order():
    """Equal coordinates with different values, interleaved with others:
    the stable sort keeps them in input order, so the segment sums run in
    the oracle's order; FP64 Z within 1e-12 and segments exact."""
    from oracle import compress_coo, coo_segments, sort_coo
    c = CooCase("dups", 60, 50, 3, 2, 10, 2, 3, 200, 29)
    k, i, j, v, U, V, W = c.inputs()
    g = np.random.Generator(np.random.PCG64(11))
    extra = g.integers(0, k.size, k.size)
    k2, i2, j2 = (np.concatenate([x, x[extra]]) for x in (k, i, j))
    v2 = np.concatenate([v, g.standard_normal(extra.size).astype(np.float32)])
    k2, i2, j2, v2 = _shuffle(c, (k2, i2, j2, v2), 12)
    Z, segs = _gpu(c, U, V, W, "f64", k2, i2, j2, v2)
    for got, want in zip(segs, coo_segments(*sort_coo(k2, i2, j2, v2)[:2], c.t)):
        assert np.array_equal(got.astype(np.int64), want)
    assert rel(Z, compress_coo(k2, i2, j2, v2, c.t, U, V, W, c.P, c.Q, c.S)) <= 1e-12


def test_reversed_batch_then_ordered_batch_on_one_handle():
    from oracle import compress_coo
    from paper_1807_01350_amd import octen as oc
    c = CASES[2]
    k, i, j, v, U, V, W = c.inputs()
    eng = _engine(c, U, V, "f32")
    tW = _dev(W)[0]
    for kk, ii, jj, vv in ((k[::-1], i[::-1], j[::-1], v[::-1]), (k, i, j, v)):
        tk, ti, tj, tv = _dev(kk, ii, jj, vv)
        eng.compress_batch_coo(tk, ti, tj, tv, c.t, tW)
        Z = eng.state(oc.OCTEN_STATE_Z).cpu().numpy()
        assert rel(Z, compress_coo(k, i, j, v, c.t, U, V, W, c.P, c.Q, c.S)) <= 1e-5
    eng.close()
