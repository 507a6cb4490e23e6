"""The replica ALS (Sec. 4.1) with its two slab contractions in the two-term
bfloat16 form (als_dtype BF16X2), through the C ABI, against the oracle's
definition of that form (oracle.precision.cp_als_two_term: the same sweep
with the contractions' products exact and their sums exact) and against the
plain FP64 ALS.

One sweep from given factors on the float32 summaries the GPU holds:

  * GPU vs the definition: the only difference is the float32 accumulation
    of the products on the matrix cores (blocks of 32 exact products, float32
    additions between blocks; the mode-3 partials of a replica's workgroups
    added in FP64).  That error and the form's own representation error (up
    to 2^-16 per product: the dropped lo*lo term and each operand's
    unrepresented tail) both scale with the cancellation in the sums, and
    the first is the smaller: 0.1 to 0.3 of the second on these cases.  The
    bar is half of the definition's distance from the FP64 sweep (both sides
    go through the same solves), which still tells the form apart from its
    plausible mistakes: FP64 arithmetic gives a ratio of 1, one-term
    bfloat16 operands or a dropped cross term ratios above 100.
  * GPU vs FP64: within 2e-2 relative, the bar stated for bfloat16 work.

Over a whole stream the form is held to the fit gate (test_gpu_fit_gate)."""
import sys

import numpy as np
import pytest

from paper_1807_01350_amd import synth
from tests.stream_helpers import Case, make_inputs, rel

pytestmark = pytest.mark.gpu

CASES = [
    # the replica shape of the dense 1000^3 workload
    Case("q60_r10", 300, 300, 10, 4, 60, 3, (100,), config_id=21),
    # rank 20 at Q = 80 (the sparse workload's replica shape)
    Case("q80_r20", 200, 200, 20, 2, 80, 3, (60,), config_id=22),
    # the 32-wide inverse at Q = 32
    Case("q32_r30", 200, 200, 30, 2, 32, 3, (60,), config_id=23),
    # a small rank (6-wide inverse), Q not a multiple of 16
    Case("q20_r5", 60, 60, 5, 3, 20, 3, (30,), config_id=24),
    # Q = 120: the slab of a workgroup stays in global memory
    Case("q120_r16", 300, 300, 16, 2, 120, 3, (60,), config_id=25),
]

RATIO = 0.5
BF16_BAR = 2e-2


def _one_sweep(case):
    import torch
    from oracle import cp_als
    from oracle.precision import cp_als_two_term
    from paper_1807_01350_amd import octen as oc
    print(f"[als-two-term] case {case.name}", file=sys.stderr, flush=True)
    X, U, V, Ws, init = make_inputs(case, x_dtype=np.float32)
    eng = oc.Octen(case.I, case.J, case.R, case.P, case.Q, case.S, torch.from_numpy(U).cuda(),
                   torch.from_numpy(V).cuda(), x_dtype="f32", compress_dtype="f32",
                   als_dtype="bf16x2")
    eng.compress_batch(torch.from_numpy(X).cuda(), torch.from_numpy(Ws[0]).cuda())
    eng.update_replicas()
    eng.cp_als_replicas(1, init=torch.from_numpy(init).cuda())
    torch.cuda.synchronize()
    Y = eng.state(oc.OCTEN_STATE_Y).cpu().numpy()
    F = eng.state(oc.OCTEN_STATE_FACTORS).cpu().numpy()
    lam = eng.state(oc.OCTEN_STATE_LAMBDA).cpu().numpy()
    flags = eng.state(oc.OCTEN_STATE_FLAGS).cpu().numpy()
    eng.close()
    assert Y.dtype == np.float32
    out = []
    for p in range(case.P):
        Fd, ld, _, _ = cp_als_two_term(Y[p], init[p], 1)
        F8, l8, _, _ = cp_als(Y[p].astype(np.float64), init[p], 1)
        out.append((F[p], lam[p], np.stack(Fd), ld, np.stack(F8), l8))
    return out, flags


@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_one_sweep(case):
    out, flags = _one_sweep(case)
    assert not np.any(flags), flags
    for p, (Fg, lg, Fd, ld, F8, l8) in enumerate(out):
        d_def = rel(Fg, Fd)
        d_form = rel(Fd, F8)
        d_f64 = rel(Fg, F8)
        print(f"[als-two-term] {case.name} replica {p}: |gpu - def| {d_def:.2e}  "
              f"|def - f64| {d_form:.2e}  |gpu - f64| {d_f64:.2e}  "
              f"lambda {rel(lg, ld):.2e}", file=sys.stderr, flush=True)
        assert d_def <= RATIO * d_form, (p, d_def, d_form)
        # lambda holds the column norms of the unnormalised C: its error is
        # bounded by the factors'
        assert rel(lg, ld) <= RATIO * d_form, p
        assert d_f64 <= BF16_BAR and rel(lg, l8) <= BF16_BAR, p


def test_needs_narrow_summaries_and_cooperative_als():
    import torch
    from paper_1807_01350_amd import octen as oc
    I, J, R, P, Q, S = 40, 36, 4, 3, 12, 3
    U, V = synth.compression_UV(I, J, P, Q, S, 77)
    tU, tV = torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda()
    for kw in (dict(compress_dtype="f64", x_dtype="f64"),
               dict(compress_dtype="f32", x_dtype="f32", flags=oc.OCTEN_FLAG_ALS_ONE_WG),
               dict(compress_dtype="f32", x_dtype="f32", flags=oc.OCTEN_FLAG_REFERENCE_PATH)):
        with pytest.raises(oc.OctenError) as ei:
            oc.Octen(I, J, R, P, Q, S, tU, tV, als_dtype="bf16x2", **kw)
        assert ei.value.status == oc.OCTEN_ERR_UNSUPPORTED, kw
