"""GPU parity of the N-mode extension (supplement, higher-order tensors)
against the N-mode oracle, step by step, through the C ABI: compression of
the N modes, the summary update, the replica ALS over N modes, matching with
lambda^(1/N), the per-mode recovery of Eq. 7 and the temporal rows with the
carried history removed, and the fit.

Bars (FP64 on both sides, no step is approximated): compression and
summaries within 1e-12 normwise relative; replica factors and weights within
1e-10 (ALS sweeps amplify rounding differences a little, as in the three-mode
FP64 parity); matching margins within 1e-9 absolute; permutations and
pairings bit-exact; recovered factors within 1e-10; fit within 1e-10
absolute."""
import sys
from dataclasses import dataclass

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@dataclass(frozen=True)
class NCase:
    name: str
    dims: tuple
    R: int
    P: int
    Q: int
    S: int
    batches: tuple
    iters: int
    sigma: float = 0.01
    config_id: int = 40
    min_fit: float = -np.inf     # the oracle's fit is at least this (a recovered stream)


CASES = [
    # four modes, every mode determined (M1 = 20 >= I_n)
    NCase("n4", (20, 18, 16), 3, 3, 8, 2, (12, 5, 5), 30, config_id=41, min_fit=0.9),
    # five modes
    NCase("n5", (9, 8, 7, 6), 2, 2, 6, 2, (8, 4), 25, config_id=42),
    # six modes, Q^6 = 15625
    NCase("n6", (5, 4, 4, 3, 3), 2, 2, 5, 2, (6, 3), 20, config_id=43),
    # three modes through the N-mode path
    NCase("n3", (30, 25), 4, 3, 10, 3, (20, 6, 6), 30, config_id=44),
    # under-determined non-temporal modes (M1 = 16 < 40, 33), a batch wider
    # than M1 (the temporal minimum-norm branch), ragged sizes, a singleton
    NCase("n4_ragged", (40, 33, 7), 3, 2, 9, 2, (20, 1, 17), 25, config_id=45),
    # rank one, one anchor column
    NCase("n4_rank1", (11, 10, 9), 1, 3, 5, 1, (6, 6), 15, config_id=46),
    # ranks past 8 and past 16 (the 16- and 32-column instances of the ALS)
    NCase("n4_r10", (12, 10, 9), 10, 3, 12, 2, (12, 6), 20, config_id=51),
    NCase("n3_r20", (30, 28), 20, 2, 24, 2, (25, 8), 15, config_id=52),
    # 130 replicas: one workgroup per replica (no cooperative launch)
    NCase("n3_many", (6, 5), 2, 130, 5, 2, (5, 3), 10, config_id=49),
    # the benchmark's four-mode stream at full size (100^3 slices, P = 10
    # replicas of 16^4, 50 sweeps): its first two batches, every output
    NCase("nmode4_full", (100, 100, 100), 5, 10, 16, 4, (20, 10), 50, config_id=50),
]


def _inputs(case):
    from paper_1807_01350_amd import synth
    K = sum(case.batches)
    fac, C = synth.nmode_factors(case.dims, K, case.R, case.config_id)
    Us = synth.compression_Us(case.dims, case.P, case.Q, case.S, case.config_id)
    M1 = case.S + case.P * (case.Q - case.S)
    Xs, Ws = [], []
    k0 = 0
    for b, t in enumerate(case.batches):
        Xs.append(synth.nmode_slices(fac, C, k0, t, case.sigma, case.config_id, b))
        Ws.append(synth.temporal_W(t, M1, case.config_id, b))
        k0 += t
    N = len(case.dims) + 1
    init = synth.nmode_als_init(case.P, N, case.Q, case.R, case.config_id)
    return Xs, Us, Ws, init


def _oracle(case, Xs, Us, Ws, init):
    from oracle.nmode import OctenNOracle, fit_dense_n
    o = OctenNOracle(case.dims, case.R, case.P, case.Q, case.S, Us)
    out = []
    for b, (X, W) in enumerate(zip(Xs, Ws)):
        Z = o.compress_batch(X, W).copy()
        Y = o.update_replicas().copy()
        F, lam = o.cp_als_replicas(case.iters, init=init if b == 0 else None)
        As, C = o.recover_factors()
        last = o.last
        out.append(dict(Z=Z, Y=Y, F=F.copy(), lam=lam.copy(), perm=last["perm"].copy(),
                        margins=last["margins"].copy(), rhs=np.stack(last["rhs"]),
                        tperm=np.asarray(last["tperm"]).copy(), H=o.H.copy(),
                        A=[a.copy() for a in As], C=C.copy()))
    X_all = np.concatenate(Xs)
    out[-1]["fit"] = fit_dense_n(X_all, out[-1]["A"], out[-1]["C"])
    return out


def _gpu(case, Xs, Us, Ws, init):
    import torch
    from paper_1807_01350_amd import octen as oc
    dev = "cuda"
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)
    eng = oc.OctenN(case.dims, case.R, case.P, case.Q, case.S, [T(u) for u in Us])
    K = sum(case.batches)
    As = [torch.zeros((d, case.R), dtype=torch.float64, device=dev) for d in case.dims]
    C = torch.zeros((K, case.R), dtype=torch.float64, device=dev)
    out = []
    try:
        for b, (X, W) in enumerate(zip(Xs, Ws)):
            eng.compress_batch(T(X), T(W))
            Z = eng.state(oc.OCTEN_STATE_Z).cpu().numpy()
            eng.update_replicas()
            Y = eng.state(oc.OCTEN_STATE_Y).cpu().numpy()
            eng.cp_als_replicas(case.iters, init=T(init) if b == 0 else None)
            F = eng.state(oc.OCTEN_STATE_FACTORS).cpu().numpy()
            lam = eng.state(oc.OCTEN_STATE_LAMBDA).cpu().numpy()
            flags = eng.state(oc.OCTEN_STATE_FLAGS).cpu().numpy()
            Kn = eng.recover_factors(As, C)
            out.append(dict(
                Z=Z, Y=Y, F=F, lam=lam, flags=flags, K=Kn,
                perm=eng.state(oc.OCTEN_STATE_PERM).cpu().numpy(),
                margins=eng.state(oc.OCTEN_STATE_MARGIN).cpu().numpy(),
                rhs=eng.state(oc.OCTEN_STATE_RHS).cpu().numpy(),
                tperm=eng.state(oc.OCTEN_STATE_TPERM).cpu().numpy(),
                H=eng.state(oc.OCTEN_STATE_H).cpu().numpy(),
                A=[a.cpu().numpy().copy() for a in As], C=C[:Kn].cpu().numpy().copy()))
        acc = (0.0, 0.0)
        k0 = 0
        for X in Xs:
            acc = eng.fit_terms(T(X), k0, As, C, acc)
            k0 += X.shape[0]
        out[-1]["fit_terms"] = acc
    finally:
        eng.close()
    return out


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


_cache = {}


def _run(case):
    if case.name not in _cache:
        print(f"[nmode] case {case.name} dims={case.dims} R={case.R} P={case.P} Q={case.Q}",
              file=sys.stderr, flush=True)
        Xs, Us, Ws, init = _inputs(case)
        _cache[case.name] = (_oracle(case, Xs, Us, Ws, init), _gpu(case, Xs, Us, Ws, init))
    return _cache[case.name]


@pytest.fixture(params=CASES, ids=[c.name for c in CASES])
def result(request):
    return request.param, _run(request.param)


def test_compression_and_update(result):
    case, (ref, got) = result
    for r, g in zip(ref, got):
        assert rel(g["Z"], r["Z"]) <= 1e-12
        assert rel(g["Y"], r["Y"]) <= 1e-12


def test_replica_als(result):
    case, (ref, got) = result
    for r, g in zip(ref, got):
        assert not g["flags"].any()
        assert rel(g["F"], r["F"]) <= 1e-10
        assert rel(g["lam"], r["lam"]) <= 1e-10


def test_matching(result):
    case, (ref, got) = result
    for r, g in zip(ref, got):
        np.testing.assert_array_equal(g["perm"], r["perm"])
        fin = np.isfinite(r["margins"])
        np.testing.assert_array_equal(np.isfinite(g["margins"]), fin)
        np.testing.assert_allclose(g["margins"][fin], r["margins"][fin], rtol=0, atol=1e-9)
        assert rel(g["rhs"], r["rhs"]) <= 1e-10


def test_recovery(result):
    case, (ref, got) = result
    for r, g in zip(ref, got):
        np.testing.assert_array_equal(g["tperm"], r["tperm"])
        for a, b in zip(g["A"], r["A"]):
            assert rel(a, b) <= 1e-10
        assert g["K"] == r["C"].shape[0]
        assert rel(g["C"], r["C"]) <= 1e-10
        assert rel(g["H"], r["H"]) <= 1e-10


def test_fit(result):
    case, (ref, got) = result
    sse, nx = got[-1]["fit_terms"]
    fit = 1.0 - np.sqrt(sse) / np.sqrt(nx)
    assert abs(fit - ref[-1]["fit"][0]) <= 1e-10
    assert ref[-1]["fit"][0] >= case.min_fit


def test_invalid_state_and_arguments():
    import torch
    from paper_1807_01350_amd import octen as oc
    from paper_1807_01350_amd import synth
    dims, R, P, Q, S = (10, 9, 8), 2, 2, 5, 2
    Us = [torch.as_tensor(u, device="cuda")
          for u in synth.compression_Us(dims, P, Q, S, 47)]
    eng = oc.OctenN(dims, R, P, Q, S, Us)
    try:
        with pytest.raises(oc.OctenError) as e:
            eng.update_replicas()
        assert e.value.status == oc.OCTEN_ERR_STATE
        with pytest.raises(oc.OctenError) as e:
            eng.cp_als_replicas(5)
        assert e.value.status == oc.OCTEN_ERR_STATE
        X = torch.zeros((0,) + dims, dtype=torch.float64, device="cuda")
        W = torch.zeros((0, eng.M1), dtype=torch.float64, device="cuda")
        with pytest.raises(oc.OctenError) as e:
            eng.compress_batch(X, W)
        assert e.value.status == oc.OCTEN_ERR_ARG
        buf = torch.empty(1, dtype=torch.float64, device="cuda")
        assert oc.octen_nm_get_state(eng.h, oc.OCTEN_STATE_Y, buf, 8) == oc.OCTEN_ERR_ARG
        assert oc.octen_nm_get_state(eng.h, 99, buf, 8) == oc.OCTEN_ERR_ARG
        # recovery before ALS, then a C too small for the rows
        X = torch.rand((4,) + dims, dtype=torch.float64, device="cuda")
        W = torch.randn((4, eng.M1), dtype=torch.float64, device="cuda")
        eng.compress_batch(X, W)
        eng.update_replicas()
        As = [torch.zeros((d, R), dtype=torch.float64, device="cuda") for d in dims]
        with pytest.raises(oc.OctenError) as e:
            eng.recover_factors(As, torch.zeros((4, R), dtype=torch.float64, device="cuda"))
        assert e.value.status == oc.OCTEN_ERR_STATE
        init = torch.randn((P, 4, Q, R), dtype=torch.float64, device="cuda")
        eng.cp_als_replicas(3, init=init)
        with pytest.raises(oc.OctenError) as e:
            eng.recover_factors(As, torch.zeros((3, R), dtype=torch.float64, device="cuda"))
        assert e.value.status == oc.OCTEN_ERR_ARG
        assert eng.recover_factors(As, torch.zeros((4, R), dtype=torch.float64, device="cuda")) == 4
    finally:
        eng.close()


def test_rank_deficient_compression_matrix_rejected():
    """A non-temporal compression matrix without full row rank (a zero row in
    the mode with I_n <= M1 = 8) makes the normal matrix of its
    least-squares operator singular (an exactly zero pivot): init reports
    OCTEN_ERR_NUMERIC."""
    import torch
    from paper_1807_01350_amd import octen as oc
    from paper_1807_01350_amd import synth
    dims, R, P, Q, S = (10, 9, 8), 2, 2, 5, 2
    Us = synth.compression_Us(dims, P, Q, S, 47)
    Us[2] = Us[2].copy()
    Us[2][3] = 0.0
    with pytest.raises(oc.OctenError) as e:
        oc.OctenN(dims, R, P, Q, S, [torch.as_tensor(u, device="cuda") for u in Us])
    assert e.value.status == oc.OCTEN_ERR_NUMERIC


def test_nonfinite_batch_leaves_summaries():
    """A batch with a NaN: every replica is flagged and left out of the
    update; the recovery reports OCTEN_ERR_NUMERIC."""
    import torch
    from paper_1807_01350_amd import octen as oc
    from paper_1807_01350_amd import synth
    case = NCase("nan", (10, 9, 8), 2, 2, 5, 2, (6, 4), 10, config_id=48)
    Xs, Us, Ws, init = _inputs(case)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    eng = oc.OctenN(case.dims, case.R, case.P, case.Q, case.S, [T(u) for u in Us])
    try:
        As = [torch.zeros((d, case.R), dtype=torch.float64, device="cuda") for d in case.dims]
        C = torch.zeros((10, case.R), dtype=torch.float64, device="cuda")
        eng.compress_batch(T(Xs[0]), T(Ws[0]))
        eng.update_replicas()
        eng.cp_als_replicas(case.iters, init=T(init))
        eng.recover_factors(As, C)
        Y0 = eng.state(oc.OCTEN_STATE_Y).cpu().numpy()
        X1 = Xs[1].copy()
        X1[1, 2, 3, 4] = np.nan
        eng.compress_batch(T(X1), T(Ws[1]))
        eng.update_replicas()
        np.testing.assert_array_equal(eng.state(oc.OCTEN_STATE_Y).cpu().numpy(), Y0)
        eng.cp_als_replicas(case.iters)
        with pytest.raises(oc.OctenError) as e:
            eng.recover_factors(As, C)
        assert e.value.status == oc.OCTEN_ERR_NUMERIC
    finally:
        eng.close()
