"""GPU parity of the sparse (COO) path against the oracle through the C ABI:
bookkeeping (bit-exact), compression of a sparse batch (Sec. 4.1) in FP64
(1e-12) and FP32 (1e-5), the whole update on a sparse stream, and the sparse
fitness identity (Sec. 5.1).  Inputs: seeded truncated-Zipf(1.2) coordinates
in modes 1 and 2, uniform slices, rank-R CP values plus N(0, 0.01^2) noise."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1807_01350_amd import synth
from tests.stream_helpers import rel

pytestmark = pytest.mark.gpu


class CooCase:
    def __init__(self, name, I, J, R, P, Q, S, t, per_slice, cid, empty=(), dup=False):
        self.name, self.I, self.J, self.R, self.P, self.Q, self.S = name, I, J, R, P, Q, S
        self.t, self.per_slice, self.cid, self.empty, self.dup = t, per_slice, cid, empty, dup

    @property
    def M1(self):
        return self.S + self.P * (self.Q - self.S)

    def inputs(self):
        _, _, _, k, i, j, v = synth.coo_stream(self.I, self.J, self.t, self.R, self.per_slice,
                                               0.01, self.cid)
        keep = ~np.isin(k, list(self.empty))
        k, i, j, v = k[keep], i[keep], j[keep], v[keep]
        if self.dup:
            # every third nonzero appears twice (adjacent, so the order holds)
            rep = np.where(np.arange(k.size) % 3 == 0, 2, 1)
            k, i, j, v = (np.repeat(x, rep) for x in (k, i, j, v))
            v = (v * np.where(np.arange(v.size) % 2 == 0, 1.0, 0.5)).astype(np.float32)
        U, V = synth.compression_UV(self.I, self.J, self.P, self.Q, self.S, self.cid)
        W = synth.temporal_W(self.t, self.M1, self.cid, 0)
        return k, i, j, v, U, V, W


CASES = [
    # one 32-column tile per replica side (Q = 20), slices without nonzeros
    # in the middle and at the end
    CooCase("q20_gaps", 300, 280, 5, 4, 20, 3, 9, 400, 21, empty=(2, 5, 8)),
    # two tiles (Q = 40), heavy Zipf rows: segments longer than a wavefront
    CooCase("q40", 2000, 1800, 8, 5, 40, 3, 12, 3000, 22),
    # three tiles (Q = 80, the sparse workload's replica side), ragged t
    CooCase("q80", 900, 1000, 10, 3, 80, 3, 7, 2500, 23),
    # four tiles (Q = 128, the largest replica side), duplicated coordinates
    CooCase("q128_dup", 400, 350, 6, 2, 128, 4, 3, 1500, 24, dup=True),
]


def _engine(c, U, V, compress_dtype):
    import torch
    from paper_1807_01350_amd import octen as oc
    x_dtype = "f64" if compress_dtype == "f64" else "f32"
    return oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, torch.from_numpy(U).cuda(),
                    torch.from_numpy(V).cuda(), x_dtype=x_dtype, compress_dtype=compress_dtype)


def _dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


_cache = {}


def _run(c, compress_dtype):
    key = (c.name, compress_dtype)
    if key not in _cache:
        from oracle import compress_coo, coo_segments
        from paper_1807_01350_amd import octen as oc
        print(f"[parity-coo] case {c.name} {compress_dtype}", file=sys.stderr, flush=True)
        k, i, j, v, U, V, W = c.inputs()
        ref = _cache.get((c.name, "oracle"))
        if ref is None:
            ref = (compress_coo(k, i, j, v, c.t, U, V, W, c.P, c.Q, c.S), coo_segments(k, i, c.t))
            _cache[(c.name, "oracle")] = ref
        eng = _engine(c, U, V, compress_dtype)
        tk, ti, tj, tv, tW = _dev(k, i, j, v, W)
        eng.compress_batch_coo(tk, ti, tj, tv, c.t, tW)
        Z = eng.state(oc.OCTEN_STATE_Z).cpu().numpy()
        segs = [x.cpu().numpy() for x in eng.coo_segments()]
        eng.close()
        _cache[key] = (ref, Z, segs)
    return _cache[key]


@pytest.mark.parametrize("c", CASES, ids=[c.name for c in CASES])
def test_coo_bookkeeping_bit_exact(c):
    (Zref, segref), _, segs = _run(c, "f64")
    for got, want in zip(segs, segref):
        assert np.array_equal(got.astype(np.int64), want), (got[:10], want[:10])


@pytest.mark.parametrize("c", CASES, ids=[c.name for c in CASES])
def test_coo_compression_f64(c):
    (Zref, _), Z, _ = _run(c, "f64")
    assert rel(Z, Zref) <= 1e-12, rel(Z, Zref)


@pytest.mark.parametrize("form", ["f32", "bf16"])
@pytest.mark.parametrize("c", CASES, ids=[c.name for c in CASES])
def test_coo_compression_f32(c, form):
    # both narrow forms gather in FP32 and accumulate with FP32 MFMA
    (Zref, segref), Z, segs = _run(c, form)
    assert rel(Z, Zref) <= 1e-5, rel(Z, Zref)
    for got, want in zip(segs, segref):
        assert np.array_equal(got.astype(np.int64), want)


def test_coo_empty_batch():
    from paper_1807_01350_amd import octen as oc
    import torch
    c = CASES[0]
    _, _, _, _, U, V, W = c.inputs()
    for form in ("f64", "f32"):
        eng = _engine(c, U, V, form)
        e = torch.zeros(0, dtype=torch.int32, device="cuda")
        ev = torch.zeros(0, dtype=torch.float32, device="cuda")
        eng.compress_batch_coo(e, e, e, ev, c.t, _dev(W)[0])
        Z = eng.state(oc.OCTEN_STATE_Z).cpu().numpy()
        assert np.all(Z == 0)
        seg_start, seg_row, slice_seg = (x.cpu().numpy() for x in eng.coo_segments())
        assert seg_start.tolist() == [0] and seg_row.size == 0
        assert slice_seg.tolist() == [0] * (c.t + 1)
        eng.close()


def test_coo_rejects_bad_coordinates_then_recovers():
    from paper_1807_01350_amd import octen as oc
    c = CASES[0]
    k, i, j, v, U, V, W = c.inputs()
    eng = _engine(c, U, V, "f64")
    tW = _dev(W)[0]
    # out of range in each mode (also when the order is broken as well)
    bad_i = i.copy(); bad_i[len(i) // 2] = c.I
    bad_j = j.copy(); bad_j[-1] = -1
    bad_k = k.copy(); bad_k[0] = c.t
    rev = [x[::-1].copy() for x in (k, bad_i, j)]
    for kk, ii, jj in ((k, bad_i, j), (k, i, bad_j), (bad_k, i, j), tuple(rev)):
        tk, ti, tj, tv = _dev(kk, ii, jj, v)
        st = oc.octen_compress_batch_coo(eng.h, v.size, tk, ti, tj, tv, c.t, tW)
        assert st == oc.OCTEN_ERR_ARG, oc.octen_status_str(st)
    # a good batch still works on the same handle
    from oracle import compress_coo
    tk, ti, tj, tv = _dev(k, i, j, v)
    eng.compress_batch_coo(tk, ti, tj, tv, c.t, tW)
    Z = eng.state(oc.OCTEN_STATE_Z).cpu().numpy()
    assert rel(Z, compress_coo(k, i, j, v, c.t, U, V, W, c.P, c.Q, c.S)) <= 1e-12
    eng.close()


@pytest.mark.parametrize("shape", [(700, 650, 4, 5, 30, 3, 1500, 25),
                                   (20000, 17000, 3, 3, 12, 2, 3000, 26)],
                         ids=["small", "tall_recovery"])
def test_coo_stream_update_and_fit_f64(shape):
    """Three sparse batches through compress -> update -> ALS -> recover, and
    the sparse fitness identity, against the oracle on the same inputs.  The
    second shape has enough rows for the MFMA product of the mode-1 and
    mode-2 recovery and for the many-block column statistics."""
    import torch
    from oracle import OctenOracle, fit_coo_identity
    from paper_1807_01350_amd import octen as oc
    I, J, R, P, Q, S, per, cid = shape
    batches = (20, 8, 6)
    K = sum(batches)
    _, _, _, k, i, j, v = synth.coo_stream(I, J, K, R, per, 0.01, cid)
    U, V = synth.compression_UV(I, J, P, Q, S, cid)
    M1 = S + P * (Q - S)
    init = synth.als_init(P, Q, R, cid)
    o = OctenOracle(I, J, R, P, Q, S, U, V)
    eng = oc.Octen(I, J, R, P, Q, S, torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda())
    A = torch.empty((I, R), dtype=torch.float64, device="cuda")
    B = torch.empty((J, R), dtype=torch.float64, device="cuda")
    C = torch.empty((K, R), dtype=torch.float64, device="cuda")
    tinit = torch.from_numpy(init).cuda()
    k0 = 0
    for b, t in enumerate(batches):
        sel = (k >= k0) & (k < k0 + t)
        kb, ib, jb, vb = k[sel] - k0, i[sel], j[sel], v[sel]
        W = synth.temporal_W(t, M1, cid, b)
        print(f"[parity-coo] stream batch {b} t={t} nnz={vb.size}", file=sys.stderr, flush=True)
        o.compress_batch_coo(kb, ib, jb, vb, t, W)
        o.update_replicas()
        o.cp_als_replicas(25, init=init if b == 0 else None)
        Ar, Br, Cr = o.recover_factors()
        tk, ti, tj, tv, tW = _dev(kb.astype(np.int32), ib, jb, vb, W)
        eng.compress_batch_coo(tk, ti, tj, tv, t, tW)
        assert rel(eng.state(oc.OCTEN_STATE_Z).cpu().numpy(), o.Z) <= 1e-12
        eng.update_replicas()
        eng.cp_als_replicas(25, init=tinit if b == 0 else None)
        Kn = eng.recover_factors(A, B, C)
        assert Kn == o.K
        assert rel(A.cpu().numpy(), Ar) <= 1e-10
        assert rel(B.cpu().numpy(), Br) <= 1e-10
        assert rel(C[:Kn].cpu().numpy(), Cr) <= 1e-10
        k0 += t
    # sparse fitness over every slice seen, fed in two pieces
    sel = k < k0
    fit_ref, sse_ref, nx_ref = fit_coo_identity(k[sel], i[sel], j[sel], v[sel], Ar, Br, Cr)
    acc = (0.0, 0.0, 0.0)
    cut = int(np.count_nonzero(k < 10))
    for lo, hi, kk0 in ((0, cut, 0), (cut, int(np.count_nonzero(sel)), 10)):
        tk, ti, tj, tv = _dev((k[lo:hi] - kk0).astype(np.int32), i[lo:hi], j[lo:hi], v[lo:hi])
        acc = eng.fit_coo_terms(tk, ti, tj, tv, kk0, A, B, C, k0, acc=acc)
    nx, inner, gram = acc
    sse = max(nx - 2 * inner + gram, 0.0)
    fit = 1.0 - np.sqrt(sse / nx)
    assert abs(nx - nx_ref) <= 1e-10 * nx_ref
    assert abs(sse - sse_ref) <= 1e-8 * nx_ref
    assert abs(fit - fit_ref) <= 1e-10
    # values sit on a sparse Zipf support, so a rank-R model of the whole
    # tensor (zeros included) fits it poorly: only the range is checked (with
    # M1 far below I, J the recovered factors are minimum-norm and the fit
    # can drop below zero)
    assert fit <= 1.0
    if I * J < 10**7:
        assert fit >= 0.0
    eng.close()


def test_coo_full_size_batch_sampled():
    """One batch of the sparse workload at full size (10^5 x 10^5, 100 slices
    of 10^5 nonzeros, P = 16 replicas of 80^3, S = 3) in the FP32 form:
    bookkeeping bit-exact, and sampled fibres Z_p[a, b, :] computed entry by
    entry by the oracle."""
    import torch
    from oracle import compress_coo_entries, coo_segments
    from paper_1807_01350_amd import octen as oc
    I = J = 100_000
    R, P, Q, S, t, per = 20, 16, 80, 3, 100, 100_000
    cid = 3
    print("[parity-coo] full-size batch: generating", file=sys.stderr, flush=True)
    _, _, _, k, i, j, v = synth.coo_stream(I, J, t, R, per, 0.01, cid)
    U, V = synth.compression_UV(I, J, P, Q, S, cid)
    M1 = S + P * (Q - S)
    W = synth.temporal_W(t, M1, cid, 1)
    print(f"[parity-coo] full-size batch: nnz={v.size}, gpu", file=sys.stderr, flush=True)
    eng = oc.Octen(I, J, R, P, Q, S, torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda(),
                   x_dtype="f32", compress_dtype="bf16")
    tk, ti, tj, tv, tW = _dev(k, i, j, v, W)
    eng.compress_batch_coo(tk, ti, tj, tv, t, tW)
    Z = eng.state(oc.OCTEN_STATE_Z).cpu().numpy()
    segs = [x.cpu().numpy() for x in eng.coo_segments()]
    eng.close()
    del tk, ti, tj, tv
    torch.cuda.empty_cache()
    print("[parity-coo] full-size batch: oracle", file=sys.stderr, flush=True)
    for got, want in zip(segs, coo_segments(k, i, t)):
        assert np.array_equal(got.astype(np.int64), want)
    rng = np.random.default_rng(7)
    picks = [(0, 0, 0), (0, 2, 1), (P - 1, Q - 1, Q - 1), (5, 3, 40)]
    picks += [(int(rng.integers(P)), int(rng.integers(Q)), int(rng.integers(Q))) for _ in range(6)]
    ref = compress_coo_entries(k, i, j, v, t, U, V, W, P, Q, S, picks)
    got = np.array([Z[p, a, b, :] for p, a, b in picks])
    assert rel(got, ref) <= 1e-5, rel(got, ref)


def test_coo_stream_sparse_workload_replicas():
    """The sparse workload's replica shape (P = 16 replicas of 80^3, S = 3,
    rank 20) on a 5000 x 5000 stream of truncated-Zipf coordinates, three
    batches through the whole update: the FP64 handle within 1e-10 of the
    oracle (factors) and its fit within 1e-10; the FP32-gather handle of the
    two-term form with its fit within 1e-3 of the oracle's."""
    import torch
    from oracle import OctenOracle, fit_coo_identity
    from paper_1807_01350_amd import octen as oc
    I = J = 5000
    R, P, Q, S, per, cid = 20, 16, 80, 3, 4000, 27
    batches = (20, 10, 10)
    iters = 10
    K = sum(batches)
    _, _, _, k, i, j, v = synth.coo_stream(I, J, K, R, per, 0.01, cid)
    U, V = synth.compression_UV(I, J, P, Q, S, cid)
    M1 = S + P * (Q - S)
    init = synth.als_init(P, Q, R, cid)
    Ws = [synth.temporal_W(t, M1, cid, b) for b, t in enumerate(batches)]
    o = OctenOracle(I, J, R, P, Q, S, U, V)
    engs = {"f64": oc.Octen(I, J, R, P, Q, S, torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda()),
            "bf16x2": oc.Octen(I, J, R, P, Q, S, torch.from_numpy(U).cuda(),
                               torch.from_numpy(V).cuda(), x_dtype="f32", compress_dtype="bf16x2")}
    outs = {f: [torch.empty((n, R), dtype=torch.float64, device="cuda") for n in (I, J, K)]
            for f in engs}
    tinit = torch.from_numpy(init).cuda()
    k0 = 0
    for b, t in enumerate(batches):
        sel = (k >= k0) & (k < k0 + t)
        kb, ib, jb, vb = k[sel] - k0, i[sel], j[sel], v[sel]
        print(f"[parity-coo] P=16 Q=80 R=20 batch {b} nnz={vb.size}", file=sys.stderr, flush=True)
        o.compress_batch_coo(kb, ib, jb, vb, t, Ws[b])
        o.update_replicas()
        o.cp_als_replicas(iters, init=init if b == 0 else None)
        Ar, Br, Cr = o.recover_factors()
        tk, ti, tj, tv, tW = _dev(kb.astype(np.int32), ib, jb, vb, Ws[b])
        for f, eng in engs.items():
            eng.compress_batch_coo(tk, ti, tj, tv, t, tW)
            eng.update_replicas()
            eng.cp_als_replicas(iters, init=tinit if b == 0 else None)
            assert eng.recover_factors(*outs[f]) == o.K
        A, B, C = (x.cpu().numpy() for x in outs["f64"])
        assert rel(A, Ar) <= 1e-10 and rel(B, Br) <= 1e-10 and rel(C[:o.K], Cr) <= 1e-10, b
        k0 += t
        sel = k < k0
        fit_ref = fit_coo_identity(k[sel], i[sel], j[sel], v[sel], Ar, Br, Cr)[0]
        tk, ti, tj, tv = _dev(k[sel].astype(np.int32), i[sel], j[sel], v[sel])
        fits = {}
        for f, eng in engs.items():
            nx, inner, gram = eng.fit_coo_terms(tk, ti, tj, tv, 0, *outs[f], k0)
            fits[f] = 1.0 - np.sqrt(max(nx - 2 * inner + gram, 0.0) / nx)
        print(f"[parity-coo] batch {b}: fit oracle {fit_ref:.6f} f64 {fits['f64']:.6f} "
              f"bf16x2 {fits['bf16x2']:.6f}", file=sys.stderr, flush=True)
        assert abs(fits["f64"] - fit_ref) <= 1e-10
        assert abs(fits["bf16x2"] - fit_ref) <= 1e-3
    for eng in engs.values():
        eng.close()
