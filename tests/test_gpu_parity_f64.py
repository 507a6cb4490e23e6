"""GPU parity of the FP64 path against the oracle, step by step, through the
C ABI: compression and update (Sec. 4.1, Eq. 1-2), replica ALS (Sec. 4.1),
matching (Sec. 4.2) and recovery (Sec. 4.3), and the fit (Sec. 5.1).

Bars: FP64 steps within 1e-10 normwise relative; matching margins within
1e-9 absolute; permutations, pairings and
iteration counts bit-exact; fit within 1e-10 absolute."""
import sys

import numpy as np
import pytest

from tests.stream_helpers import Case, make_inputs, run_gpu, run_oracle, rel

pytestmark = pytest.mark.gpu

CASES = [
    # the 50^3 FP64 stream: 30 initial slices then two batches of 10
    Case("dense50", 50, 50, 5, 4, 20, 3, (30, 10, 10), iters=50),
    # several GEMM tiles with ragged tails, under-determined modes 1-2
    # (M1 = 108 < I, J), and a singleton batch
    Case("ragged", 137, 151, 6, 5, 24, 3, (40, 17, 1), iters=30, config_id=11),
    # more slices in a batch than compression columns (M1 = 17 < t = 30):
    # the temporal solve takes the minimum-norm branch
    Case("wide_t", 40, 40, 3, 2, 10, 3, (30, 5), iters=40, config_id=12),
    # rank one (matching is trivial) with two anchors
    Case("rank1", 30, 30, 1, 3, 8, 2, (12, 6), iters=20, config_id=13),
    # large replicas: ALS spreads each replica over several workgroups
    Case("wideq", 90, 90, 4, 3, 40, 3, (20, 8), iters=30, config_id=14),
    # nine replicas of 64^3 at rank 16: the FP64 slab of a workgroup does not
    # fit in LDS next to the factor state, so the ALS reads it from global
    # memory (16 workgroups per replica, two replicas on some XCDs)
    Case("gx_slab", 120, 110, 16, 9, 64, 3, (30, 10), iters=20, config_id=15),
    # the ranks of the sparse and batched workloads: R = 20 with Q = 80 (the
    # sparse stream's replica side; slab in global memory) and R = 24 with the
    # slab in LDS, both on the 24-wide inverse; R = 30 with Q = 64 (global
    # memory) and Q = 32 (LDS) on the 32-wide inverse
    Case("r20_q80", 120, 120, 20, 4, 80, 3, (40, 10), iters=15, config_id=16),
    Case("r24_lds", 100, 100, 24, 4, 40, 3, (40, 10), iters=15, config_id=17),
    Case("r30_q64", 110, 110, 30, 4, 64, 3, (40, 10), iters=12, config_id=18),
    Case("r30_lds", 100, 100, 30, 4, 32, 3, (40, 10), iters=15, config_id=19),
]

_cache = {}


def _run(case):
    if case.name not in _cache:
        print(f"[parity-f64] case {case.name}", file=sys.stderr, flush=True)
        X, U, V, Ws, init = make_inputs(case)
        ref = run_oracle(case, X, U, V, Ws, init)
        got = run_gpu(case, X, U, V, Ws, init, compress_dtype="f64", x_dtype="f64", log=True)
        _cache[case.name] = (ref, got)
    return _cache[case.name]


@pytest.fixture(params=CASES, ids=[c.name for c in CASES])
def result(request):
    return request.param, _run(request.param)


def test_compression_and_update(result):
    case, (ref, got) = result
    for b, (r, g) in enumerate(zip(ref, got)):
        assert rel(g["Z"], r["Z"]) <= 1e-12, (b, rel(g["Z"], r["Z"]))
        assert rel(g["Y"], r["Y"]) <= 1e-12, (b, rel(g["Y"], r["Y"]))


def test_replica_als(result):
    case, (ref, got) = result
    for b, (r, g) in enumerate(zip(ref, got)):
        assert np.array_equal(g["iters"], r["iters"])
        assert rel(g["F"], r["F"]) <= 1e-10, (b, rel(g["F"], r["F"]))
        assert rel(g["lam"], r["lam"]) <= 1e-10, (b, rel(g["lam"], r["lam"]))
        assert not np.any(g["flags"])


def test_matching_permutation_exact(result):
    case, (ref, got) = result
    for b, (r, g) in enumerate(zip(ref, got)):
        ok = r["margins"] > 1e-6
        assert np.array_equal(g["perm"][ok], r["perm"][ok]), b
        # a margin is a difference of two products of three |cos| of unit
        # columns, each product within a few 1e-10 of the oracle's when the
        # factors are (the FP64 bar): the bar is absolute
        fin = np.isfinite(r["margins"])
        assert np.allclose(g["margins"][fin], r["margins"][fin], rtol=1e-8, atol=1e-9)
        assert np.array_equal(g["tperm"], r["tperm"]), b


def test_aligned_and_stacked(result):
    case, (ref, got) = result
    for b, (r, g) in enumerate(zip(ref, got)):
        assert rel(g["aligned"], r["aligned"]) <= 1e-10, (b, rel(g["aligned"], r["aligned"]))
        assert rel(g["rhs"], r["rhs"]) <= 1e-10, (b, rel(g["rhs"], r["rhs"]))


def test_recovered_factors(result):
    case, (ref, got) = result
    for b, (r, g) in enumerate(zip(ref, got)):
        assert g["K"] == r["K"]
        for key in ("A", "B", "C", "H"):
            assert rel(g[key], r[key]) <= 1e-10, (b, key, rel(g[key], r[key]))


def test_fit(result):
    case, (ref, got) = result
    for b, (r, g) in enumerate(zip(ref, got)):
        assert abs(g["fit"] - r["fit"]) <= 1e-10, (b, g["fit"], r["fit"])


def test_reference_kernels_agree():
    """The plain reference kernels (no MFMA, one workgroup per replica) give
    the same stream as the default kernels, both within the oracle's bars."""
    from paper_1807_01350_amd import octen as oc
    case = CASES[4]
    X, U, V, Ws, init = make_inputs(case)
    a = _run(case)[1]
    b = run_gpu(case, X, U, V, Ws, init, flags=oc.OCTEN_FLAG_REFERENCE_PATH)
    for x, y in zip(a, b):
        for key in ("F", "A", "B", "C"):
            assert rel(x[key], y[key]) <= 1e-10, key


def test_deterministic_rerun():
    case = CASES[4]
    X, U, V, Ws, init = make_inputs(case)
    a = run_gpu(case, X, U, V, Ws, init)
    b = run_gpu(case, X, U, V, Ws, init)
    for x, y in zip(a, b):
        for key in ("Z", "Y", "F", "A", "B", "C"):
            assert np.array_equal(x[key], y[key]), key


@pytest.mark.parametrize("idx", [4, 5], ids=["wideq", "gx_slab"])
def test_device_sync_barriers_give_identical_als(idx):
    """Replicas spread over several workgroups: the barriers that keep the
    slot exchange inside one XCD's L2 and the ones that write back and
    invalidate the L2 at every step give bit-identical ALS results (the slot
    sums run in a fixed order either way), with and without a tolerance."""
    from paper_1807_01350_amd import octen as oc
    case = CASES[idx]
    X, U, V, Ws, init = make_inputs(case)
    for tol in (0.0, 1e-9):
        a = run_gpu(case, X, U, V, Ws, init, tol=tol)
        b = run_gpu(case, X, U, V, Ws, init, tol=tol, flags=oc.OCTEN_FLAG_ALS_DEVICE_SYNC)
        for x, y in zip(a, b):
            assert np.array_equal(x["iters"], y["iters"])
            for key in ("F", "lam", "A", "B", "C"):
                assert np.array_equal(x[key], y[key]), (tol, key)
            assert not np.any(x["flags"]) and not np.any(y["flags"])
