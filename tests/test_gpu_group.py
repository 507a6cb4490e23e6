"""GPU checks of batched steps and the autotuner through the C ABI.

A group runs compress -> update -> ALS of several streams of uneven shapes as
one captured HIP graph; every round must give exactly the results of the same
calls made handle by handle (the kernels and their order are the same), also
on replays with eager work and synchronisation between them.  FP64 streams in
a group are also compared with the oracle."""
import sys

import numpy as np
import pytest

from paper_1807_01350_amd import synth
from tests.stream_helpers import Case, make_inputs, rel

pytestmark = pytest.mark.gpu

# uneven streams: (I, J, R, P, Q, S, t0, t, form)
SHAPES = [
    (90, 70, 4, 4, 20, 3, 24, 8, "f32"),
    (130, 160, 6, 6, 36, 3, 30, 12, "bf16"),
    (64, 64, 3, 3, 24, 3, 20, 5, "f32"),
    (200, 120, 8, 5, 40, 3, 40, 16, "bf16"),
    (150, 97, 5, 4, 24, 3, 24, 8, "bf16x2"),
]
ROUNDS = 4


def _streams(shapes, seed0):
    import torch
    out = []
    for q, (I, J, R, P, Q, S, t0, t, form) in enumerate(shapes):
        c = Case(f"g{q}", I, J, R, P, Q, S, (t0,) + (t,) * ROUNDS, iters=20,
                 config_id=seed0 + q)
        X, U, V, Ws, init = make_inputs(c, x_dtype=np.float32 if form != "f64" else np.float64)
        out.append((c, form, torch.from_numpy(X).cuda(), torch.from_numpy(U).cuda(),
                    torch.from_numpy(V).cuda(), [torch.from_numpy(w).cuda() for w in Ws],
                    torch.from_numpy(init).cuda()))
    return out


def _engine(c, form, U, V):
    from paper_1807_01350_amd import octen as oc
    x = "f64" if form == "f64" else "f32"
    return oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, U, V, x_dtype=x, compress_dtype=form,
                    flags=oc.OCTEN_FLAG_ALS_ONE_WG)


def _run(shapes, seed0, iters=15, tol=0.0):
    """Group and twin handles on the same streams; returns per round the
    (group, eager) states and whether the group replayed."""
    import torch
    from paper_1807_01350_amd import octen as oc
    streams = _streams(shapes, seed0)
    grp_engs, twin_engs, bufs = [], [], []
    for c, form, X, U, V, Ws, init in streams:
        g, e = _engine(c, form, U, V), _engine(c, form, U, V)
        t0 = c.batches[0]
        for eng in (g, e):
            eng.compress_batch(X[:t0], Ws[0])
            eng.update_replicas()
            eng.cp_als_replicas(iters, init=init)
            eng.recover_factors(torch.empty((c.I, c.R), dtype=torch.float64, device="cuda"),
                                torch.empty((c.J, c.R), dtype=torch.float64, device="cuda"),
                                torch.empty((c.K, c.R), dtype=torch.float64, device="cuda"))
        # fixed batch buffers, rewritten in place every round
        bufs.append((torch.empty_like(X[t0:t0 + c.batches[1]]), torch.empty_like(Ws[1])))
        grp_engs.append(g)
        twin_engs.append(e)
    group = oc.Group(grp_engs)
    rounds = []
    for r in range(1, ROUNDS + 1):
        print(f"[group] round {r}", file=sys.stderr, flush=True)
        for (c, form, X, U, V, Ws, init), (xb, wb) in zip(streams, bufs):
            k0 = sum(c.batches[:r])
            xb.copy_(X[k0:k0 + c.batches[r]])
            wb.copy_(Ws[r])
        replayed = group.step(bufs, iters, tol)
        for e, (xb, wb) in zip(twin_engs, bufs):
            e.compress_batch(xb, wb)
            e.update_replicas()
            e.cp_als_replicas(iters, tol=tol)
        torch.cuda.synchronize()
        # eager work between replays
        _ = (torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")).sum()
        torch.cuda.synchronize()
        res = []
        for g, e, (c, *_rest) in zip(grp_engs, twin_engs, streams):
            A = torch.empty((c.I, c.R), dtype=torch.float64, device="cuda")
            B = torch.empty((c.J, c.R), dtype=torch.float64, device="cuda")
            C = torch.empty((c.K, c.R), dtype=torch.float64, device="cuda")
            A2, B2, C2 = torch.empty_like(A), torch.empty_like(B), torch.empty_like(C)
            K = g.recover_factors(A, B, C)
            assert e.recover_factors(A2, B2, C2) == K
            C, C2 = C[:K], C2[:K]
            res.append({
                "Y": (g.state(oc.OCTEN_STATE_Y).cpu().numpy(), e.state(oc.OCTEN_STATE_Y).cpu().numpy()),
                "F": (g.state(oc.OCTEN_STATE_FACTORS).cpu().numpy(),
                      e.state(oc.OCTEN_STATE_FACTORS).cpu().numpy()),
                "A": (A.cpu().numpy(), A2.cpu().numpy()), "C": (C.cpu().numpy(), C2.cpu().numpy())})
        rounds.append((replayed, res))
    group.close()
    for e in grp_engs + twin_engs:
        e.close()
    return rounds


def test_group_step_equals_handle_by_handle_calls():
    rounds = _run(SHAPES, 60)
    assert [rp for rp, _ in rounds] == [False] + [True] * (ROUNDS - 1)
    for r, (_, res) in enumerate(rounds):
        for q, item in enumerate(res):
            for key, (a, b) in item.items():
                assert np.array_equal(a, b), (r, q, key, float(np.max(np.abs(a - b))))


def test_group_fp64_streams_match_oracle():
    """Two FP64 streams in a group against the oracle (ALS with a fixed number
    of sweeps, one workgroup per replica)."""
    import torch
    from oracle import OctenOracle
    from paper_1807_01350_amd import octen as oc
    cases = [Case("gf0", 50, 50, 5, 4, 20, 3, (30, 10, 10), iters=25, config_id=71),
             Case("gf1", 70, 60, 3, 3, 16, 2, (20, 7, 7), iters=25, config_id=72)]
    ins = [make_inputs(c) for c in cases]
    engs, oras, bufs = [], [], []
    for c, (X, U, V, Ws, init) in zip(cases, ins):
        e = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, torch.from_numpy(U).cuda(),
                     torch.from_numpy(V).cuda(), flags=oc.OCTEN_FLAG_ALS_ONE_WG)
        o = OctenOracle(c.I, c.J, c.R, c.P, c.Q, c.S, U, V)
        t0 = c.batches[0]
        e.compress_batch(torch.from_numpy(X[:t0]).cuda(), torch.from_numpy(Ws[0]).cuda())
        e.update_replicas()
        e.cp_als_replicas(c.iters, init=torch.from_numpy(init).cuda())
        o.compress_batch(X[:t0], Ws[0]); o.update_replicas(); o.cp_als_replicas(c.iters, init=init)
        engs.append(e); oras.append(o)
        bufs.append((torch.empty((c.batches[1], c.I, c.J), dtype=torch.float64, device="cuda"),
                     torch.empty((c.batches[1], c.M1), dtype=torch.float64, device="cuda")))
    group = oc.Group(engs)
    for r in (1, 2):
        for c, (X, U, V, Ws, init), (xb, wb), o in zip(cases, ins, bufs, oras):
            k0 = sum(c.batches[:r])
            xb.copy_(torch.from_numpy(X[k0:k0 + c.batches[r]]))
            wb.copy_(torch.from_numpy(Ws[r]))
            o.compress_batch(X[k0:k0 + c.batches[r]], Ws[r]); o.update_replicas()
            o.cp_als_replicas(c.iters)
        group.step(bufs, cases[0].iters)
        torch.cuda.synchronize()
        for e, o in zip(engs, oras):
            assert rel(e.state(oc.OCTEN_STATE_Y).cpu().numpy(), o.Y) <= 1e-12
            assert rel(e.state(oc.OCTEN_STATE_FACTORS).cpu().numpy(), o.F) <= 1e-10
    group.close()
    for e in engs:
        e.close()


def test_group_narrow_streams_fit_gate():
    """Three float32 streams of uneven shapes (FP32 and two-term BF16
    compression) stepped as one group: after every round the fit of each
    (Sec. 5.1, over all slices seen) lies within 1e-3 of the FP64 oracle's
    on the same slices."""
    import torch
    from oracle import OctenOracle, fit_dense
    from paper_1807_01350_amd import octen as oc
    spec = [(Case("gn0", 160, 140, 6, 6, 30, 3, (40, 10, 10, 10), iters=20, config_id=74), "f32"),
            (Case("gn1", 210, 130, 8, 8, 36, 3, (50, 12, 12, 12), iters=20, config_id=75), "bf16x2"),
            (Case("gn2", 120, 123, 5, 5, 24, 3, (30, 8, 8, 8), iters=20, config_id=76), "bf16x2")]
    engs, oras, bufs, ins, outs = [], [], [], [], []
    for c, form in spec:
        X, U, V, Ws, init = make_inputs(c, x_dtype=np.float32)
        ins.append((X, U, V, Ws, init))
        e = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, torch.from_numpy(U).cuda(),
                     torch.from_numpy(V).cuda(), x_dtype="f32", compress_dtype=form,
                     flags=oc.OCTEN_FLAG_ALS_ONE_WG)
        o = OctenOracle(c.I, c.J, c.R, c.P, c.Q, c.S, U, V)
        t0 = c.batches[0]
        e.compress_batch(torch.from_numpy(X[:t0]).cuda(), torch.from_numpy(Ws[0]).cuda())
        e.update_replicas()
        e.cp_als_replicas(c.iters, init=torch.from_numpy(init).cuda())
        o.compress_batch(X[:t0].astype(np.float64), Ws[0]); o.update_replicas()
        o.cp_als_replicas(c.iters, init=init)
        out = [torch.empty((n, c.R), dtype=torch.float64, device="cuda") for n in (c.I, c.J, c.K)]
        e.recover_factors(*out); o.recover_factors()
        engs.append(e); oras.append(o); outs.append(out)
        bufs.append((torch.empty((c.batches[1], c.I, c.J), dtype=torch.float32, device="cuda"),
                     torch.empty((c.batches[1], c.M1), dtype=torch.float64, device="cuda")))
    group = oc.Group(engs)
    for r in (1, 2, 3):
        for (c, form), (X, U, V, Ws, init), (xb, wb), o in zip(spec, ins, bufs, oras):
            k0 = sum(c.batches[:r])
            xb.copy_(torch.from_numpy(X[k0:k0 + c.batches[r]]))
            wb.copy_(torch.from_numpy(Ws[r]))
            o.compress_batch(X[k0:k0 + c.batches[r]].astype(np.float64), Ws[r])
            o.update_replicas(); o.cp_als_replicas(c.iters); o.recover_factors()
        group.step(bufs, spec[0][0].iters)
        for (c, form), (X, *_), e, o, out in zip(spec, ins, engs, oras, outs):
            K = e.recover_factors(*out)
            assert K == o.K
            sse, nx = e.fit_terms(torch.from_numpy(X[:K]).cuda(), 0, *out)
            fit = 1.0 - np.sqrt(sse / nx)
            fit_o = fit_dense(X[:K].astype(np.float64), o.A, o.B, o.C)[0]
            print(f"[group] round {r} {c.name} {form}: fit {fit:.6f} oracle {fit_o:.6f}",
                  file=sys.stderr, flush=True)
            assert abs(fit - fit_o) <= 1e-3, (r, c.name, fit, fit_o)
    group.close()
    for e in engs:
        e.close()


def test_group_recaptures_when_descriptors_change():
    import torch
    from paper_1807_01350_amd import octen as oc
    streams = _streams(SHAPES[:2], 80)
    engs, bufs = [], []
    for c, form, X, U, V, Ws, init in streams:
        e = _engine(c, form, U, V)
        e.compress_batch(X[:c.batches[0]], Ws[0]); e.update_replicas()
        e.cp_als_replicas(10, init=init)
        e.recover_factors(torch.empty((c.I, c.R), dtype=torch.float64, device="cuda"),
                          torch.empty((c.J, c.R), dtype=torch.float64, device="cuda"),
                          torch.empty((c.batches[0] + 6 * c.batches[1], c.R), dtype=torch.float64,
                                      device="cuda"))
        engs.append(e)
        bufs.append((X[c.batches[0]:c.batches[0] + c.batches[1]].clone(), Ws[1].clone()))
    group = oc.Group(engs)
    outs = []
    for c, *_ in streams:
        outs.append((torch.empty((c.I, c.R), dtype=torch.float64, device="cuda"),
                     torch.empty((c.J, c.R), dtype=torch.float64, device="cuda"),
                     torch.empty((c.batches[0] + 6 * c.batches[1], c.R), dtype=torch.float64,
                                 device="cuda")))

    def step(b, iters):
        rep = group.step(b, iters)
        for e, (A, B, C) in zip(engs, outs):
            e.recover_factors_async(A, B, C)   # pending slices back to zero
        return rep

    flags = [step(bufs, 10), step(bufs, 10), step(bufs, 12)]   # then another sweep count
    other = [(x.clone(), w) for x, w in bufs]                  # other buffers
    flags += [step(other, 12), step(other, 12)]
    assert flags == [False, True, False, False, True]
    group.close()
    for e in engs:
        e.close()


@pytest.mark.parametrize("form,J", [("bf16", 1000), ("f32", 1000), ("bf16", 998)])
def test_autotune_keeps_results_within_tolerance(form, J):
    import torch
    from oracle import compress_dense
    from paper_1807_01350_amd import octen as oc
    I, R, P, Q, S, t = 300, 6, 12, 60, 3, 6
    c = Case("tune", I, J, R, P, Q, S, (t,), config_id=90)
    X, U, V, Ws, init = make_inputs(c, x_dtype=np.float32)
    tX, tW = torch.from_numpy(X).cuda(), torch.from_numpy(Ws[0]).cuda()
    e = oc.Octen(I, J, R, P, Q, S, torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda(),
                 x_dtype="f32", compress_dtype=form)
    choice = e.autotune(tX)
    G, variant = divmod(choice, 10)
    assert 1 <= G <= P and variant in ((0, 1, 2, 3) if form == "bf16" else (0, 1, 2))
    if J % 4:
        assert variant == 2
    e.compress_batch(tX, tW)
    Z = e.state(oc.OCTEN_STATE_Z).cpu().numpy()
    Zr = compress_dense(X.astype(np.float64), U, V, Ws[0], P, Q, S)
    assert rel(Z, Zr) <= (2e-2 if form == "bf16" else 1e-5)
    print(f"[autotune] {form} J={J}: choice {choice}", file=sys.stderr)
    e.close()


@pytest.mark.parametrize("J", [1000, 998])
def test_compress_variants_agree(J):
    """Every compression variant of a BF16 handle gives the oracle's summary
    within the BF16 bar; the half-chunk variant (3) accumulates the same k
    steps in the same order as the pipelined one (0), so the two agree bit
    for bit.  With J % 4 != 0 the 16-byte variants fall back to the scalar
    kernel."""
    import torch
    from oracle import compress_dense
    from paper_1807_01350_amd import octen as oc
    I, R, P, Q, S, t = 600, 6, 12, 60, 3, 5
    c = Case("variants", I, J, R, P, Q, S, (t,), config_id=91)
    X, U, V, Ws, init = make_inputs(c, x_dtype=np.float32)
    tX, tW = torch.from_numpy(X).cuda(), torch.from_numpy(Ws[0]).cuda()
    e = oc.Octen(I, J, R, P, Q, S, torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda(),
                 x_dtype="f32", compress_dtype="bf16")
    Zr = compress_dense(X.astype(np.float64), U, V, Ws[0], P, Q, S)
    Zs = {}
    for v in (0, 1, 2, 3):
        e.compress_variant(v)
        e.compress_batch(tX, tW)
        Zs[v] = e.state(oc.OCTEN_STATE_Z).cpu().numpy()
        assert rel(Zs[v], Zr) <= 2e-2, (v, rel(Zs[v], Zr))
    assert np.array_equal(Zs[0], Zs[3])
    with pytest.raises(oc.OctenError):
        e.compress_variant(4)
    e.close()


def test_small_group_runs_cooperative_als_after_the_join():
    """With few replicas the group runs each ALS on the handle's cooperative
    kernel after its branches join: results equal the handle-by-handle calls
    of handles without OCTEN_FLAG_ALS_ONE_WG."""
    import torch
    from paper_1807_01350_amd import octen as oc
    shapes = [(300, 280, 6, 12, 60, 3, 40, 10, "bf16"), (200, 240, 5, 8, 40, 3, 30, 8, "f32")]
    streams = _streams(shapes, 95)
    grp, twin, bufs = [], [], []
    for c, form, X, U, V, Ws, init in streams:
        pair = [oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, U, V, x_dtype="f32", compress_dtype=form)
                for _ in range(2)]
        for e in pair:
            e.compress_batch(X[:c.batches[0]], Ws[0]); e.update_replicas()
            e.cp_als_replicas(20, init=init)
            e.recover_factors(torch.empty((c.I, c.R), dtype=torch.float64, device="cuda"),
                              torch.empty((c.J, c.R), dtype=torch.float64, device="cuda"),
                              torch.empty((c.K, c.R), dtype=torch.float64, device="cuda"))
        grp.append(pair[0]); twin.append(pair[1])
        bufs.append((torch.empty_like(X[:c.batches[1]]), torch.empty_like(Ws[1])))
    group = oc.Group(grp)
    flags = []
    for r in (1, 2, 3):
        for (c, form, X, U, V, Ws, init), (xb, wb) in zip(streams, bufs):
            k0 = sum(c.batches[:r])
            xb.copy_(X[k0:k0 + c.batches[r]]); wb.copy_(Ws[r])
        flags.append(group.step(bufs, 20, 1e-7))
        for e, (xb, wb) in zip(twin, bufs):
            e.compress_batch(xb, wb); e.update_replicas(); e.cp_als_replicas(20, tol=1e-7)
        for g, e, (c, *_r) in zip(grp, twin, streams):
            for what in (oc.OCTEN_STATE_Y, oc.OCTEN_STATE_FACTORS, oc.OCTEN_STATE_ITERS):
                a, b = g.state(what).cpu().numpy(), e.state(what).cpu().numpy()
                assert np.array_equal(a, b), (r, what)
            for e2 in (g, e):
                e2.recover_factors(torch.empty((c.I, c.R), dtype=torch.float64, device="cuda"),
                                   torch.empty((c.J, c.R), dtype=torch.float64, device="cuda"),
                                   torch.empty((c.K, c.R), dtype=torch.float64, device="cuda"))
    assert flags == [False, True, True]
    group.close()
    for e in grp + twin:
        e.close()


def test_group_packs_cooperative_als_of_equal_kernels():
    """After the join, handles whose ALS runs the same kernel share one
    cooperative launch (four float-summary FP64-solve handles of ranks 5, 6,
    9 and 13, three rank classes, each member taking its own class's
    inverse; two of them with the fewest workgroups per replica); a
    two-term handle takes a launch of its own.  Every replica's result
    equals the handle-by-handle cooperative calls bit for bit (the
    convergence test on, so members may stop at different sweeps), and so
    does the group's recovery of all handles at once (octen_group_recover)."""
    import torch
    from paper_1807_01350_amd import octen as oc
    shapes = [(120, 100, 5, 4, 20, 3, 24, 6, "bf16x2"), (140, 90, 6, 6, 24, 3, 30, 8, "bf16x2"),
              (100, 130, 9, 8, 22, 3, 20, 5, "f32"), (90, 110, 13, 5, 26, 3, 24, 6, "bf16"),
              (110, 96, 5, 4, 24, 3, 20, 5, "bf16x2")]
    als = ["f64", "f64", "f64", "f64", "bf16x2"]
    streams = _streams(shapes, 120)
    grp, twin, bufs = [], [], []
    for q, ((c, form, X, U, V, Ws, init), ad) in enumerate(zip(streams, als)):
        fl = oc.OCTEN_FLAG_ALS_FEW_WG if q in (1, 3) else 0
        pair = [oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, U, V, x_dtype="f32", compress_dtype=form,
                         als_dtype=ad, flags=fl) for _ in range(2)]
        for e in pair:
            e.compress_batch(X[:c.batches[0]], Ws[0]); e.update_replicas()
            e.cp_als_replicas(20, init=init)
            e.recover_factors(torch.empty((c.I, c.R), dtype=torch.float64, device="cuda"),
                              torch.empty((c.J, c.R), dtype=torch.float64, device="cuda"),
                              torch.empty((c.K, c.R), dtype=torch.float64, device="cuda"))
        grp.append(pair[0]); twin.append(pair[1])
        bufs.append((torch.empty_like(X[:c.batches[1]]), torch.empty_like(Ws[1])))
    group = oc.Group(grp)
    flags, iters = [], set()
    for r in (1, 2, 3):
        print(f"[group] packed ALS round {r}", file=sys.stderr, flush=True)
        for (c, form, X, U, V, Ws, init), (xb, wb) in zip(streams, bufs):
            k0 = sum(c.batches[:r])
            xb.copy_(X[k0:k0 + c.batches[r]]); wb.copy_(Ws[r])
        flags.append(group.step(bufs, 20, 1e-6))
        for e, (xb, wb) in zip(twin, bufs):
            e.compress_batch(xb, wb); e.update_replicas(); e.cp_als_replicas(20, tol=1e-6)
        torch.cuda.synchronize()
        _ = (torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")).sum()
        torch.cuda.synchronize()
        for q, (g, e, (c, *_r)) in enumerate(zip(grp, twin, streams)):
            for what in (oc.OCTEN_STATE_Y, oc.OCTEN_STATE_FACTORS, oc.OCTEN_STATE_LAMBDA,
                         oc.OCTEN_STATE_ITERS, oc.OCTEN_STATE_FLAGS):
                a, b = g.state(what).cpu().numpy(), e.state(what).cpu().numpy()
                assert np.array_equal(a, b), (r, q, what)
            iters.update(int(v) for v in g.state(oc.OCTEN_STATE_ITERS).cpu().numpy())
            assert not g.state(oc.OCTEN_STATE_FLAGS).cpu().numpy().any(), (r, q)
        # the group's recovery (handles on their own streams) against the
        # handle-by-handle calls
        outs = [tuple(torch.full((n, c.R), float("nan"), dtype=torch.float64, device="cuda")
                      for n in (c.I, c.J, c.K)) for (c, *_r) in streams]
        group.recover(outs)
        for q, (g, e, (c, *_r)) in enumerate(zip(grp, twin, streams)):
            ref = [torch.empty((n, c.R), dtype=torch.float64, device="cuda") for n in (c.I, c.J, c.K)]
            K = e.recover_factors(*ref)
            assert g.K == K, (r, q)
            (A, B, C), (A2, B2, C2) = outs[q], ref
            for what, a, b in (("A", A, A2), ("B", B, B2), ("C", C[:K], C2[:K])):
                assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), (r, q, what)
    assert flags == [False, True, True]
    assert group.als_launches() == 2
    print(f"[group] sweep counts seen: {sorted(iters)}", file=sys.stderr, flush=True)
    group.close()
    for e in grp + twin:
        e.close()
