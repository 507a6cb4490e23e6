"""GPU parity of the matrix-core compression (Sec. 4.1, Eq. 1) on f32 slices:
FP32 inputs within 1e-5 and BF16 inputs within 2e-2 of the FP64 oracle
(normwise per replica), and BF16 within 1e-4 of the BF16-emulating oracle.
Shapes cover several row blocks and column blocks with ragged tails, the
scalar-load path (J not a multiple of 4), and Q > 64.

The bar against the emulation follows from the one place the two differ: the
kernel rounds its FP32-accumulated X_k V to bfloat16, the emulation rounds the
exact sum.  With non-negative slices the FP32 sum of J terms is off by up to
about J * 2^-24 relative, so a fraction of about 2 * J * 2^-24 / 2^-7 of the
rounded values land one bfloat16 step (2^-7 relative at most) apart, a
normwise effect of about sqrt(J * 2^-16) * 2^-7; the bar is three times that.
"""
import sys

import numpy as np
import pytest

from oracle import compress_dense
from oracle.precision import compress_dense_bf16_emulated
from paper_1807_01350_amd import synth
from tests.stream_helpers import rel

pytestmark = pytest.mark.gpu

SHAPES = [
    # name, I, J, t, P, Q, S
    ("c2_like", 300, 260, 7, 12, 60, 3),       # 3 column blocks, ragged rows and j
    ("odd_j", 150, 97, 5, 5, 24, 3),           # J % 4 != 0: scalar loads
    ("q80", 200, 200, 4, 4, 80, 3),            # three 32-wide tiles per replica side
    ("single_slice", 129, 64, 1, 2, 20, 2),    # t = 1, one row past a block
]


def emu_bar(J):
    return 3 * 2.0 ** -7 * np.sqrt(J * 2.0 ** -16)


def _inputs(I, J, t, P, Q, S, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    M1 = S + P * (Q - S)
    X = g.random((t, I, J)).astype(np.float32)
    U = g.standard_normal((I, M1))
    V = g.standard_normal((J, M1))
    W = g.standard_normal((t, M1))
    return X, U, V, W


def _gpu_Z(I, J, P, Q, S, X, U, V, W, dtype, scale=None):
    import torch
    from paper_1807_01350_amd import octen as oc
    eng = oc.Octen(I, J, min(Q, 5), P, Q, S, torch.from_numpy(U).cuda(), torch.from_numpy(V).cuda(),
                   x_dtype="f32", compress_dtype=dtype)
    sc = None if scale is None else torch.from_numpy(scale).cuda()
    eng.compress_batch(torch.from_numpy(X).cuda(), torch.from_numpy(W).cuda(), sc)
    Z = eng.state(oc.OCTEN_STATE_Z).cpu().numpy()
    eng.close()
    return Z


@pytest.mark.parametrize("shape", SHAPES, ids=[s[0] for s in SHAPES])
def test_fp32_and_bf16_compression(shape):
    name, I, J, t, P, Q, S = shape
    print(f"[mfma] {name}", file=sys.stderr, flush=True)
    X, U, V, W = _inputs(I, J, t, P, Q, S, 7 + I)
    ref = compress_dense(X.astype(np.float64), U, V, W, P, Q, S)
    z32 = _gpu_Z(I, J, P, Q, S, X, U, V, W, "f32")
    zbf = _gpu_Z(I, J, P, Q, S, X, U, V, W, "bf16")
    emu = compress_dense_bf16_emulated(X, U, V, W, P, Q, S)
    e32 = max(rel(z32[p], ref[p]) for p in range(P))
    ebf = max(rel(zbf[p], ref[p]) for p in range(P))
    eem = max(rel(zbf[p], emu[p]) for p in range(P))
    print(f"[mfma] {name}: f32 {e32:.2e} bf16 {ebf:.2e} bf16-vs-emulation {eem:.2e}",
          file=sys.stderr, flush=True)
    for p in range(P):
        assert rel(z32[p], ref[p]) <= 1e-5, (p, rel(z32[p], ref[p]))
        assert rel(zbf[p], ref[p]) <= 2e-2, (p, rel(zbf[p], ref[p]))
        assert rel(zbf[p], emu[p]) <= emu_bar(J), (p, rel(zbf[p], emu[p]))


def test_power_of_two_slice_scale_is_exact():
    I, J, t, P, Q, S = 140, 96, 3, 4, 20, 3
    X, U, V, W = _inputs(I, J, t, P, Q, S, 5)
    scale = np.array([2.0 ** -3, 1.0, 2.0 ** 5], dtype=np.float32)
    for dt in ("f32", "bf16"):
        a = _gpu_Z(I, J, P, Q, S, X, U, V, W, dt)
        b = _gpu_Z(I, J, P, Q, S, X, U, V, W, dt, scale)
        assert np.array_equal(a, b), dt


def test_full_size_batch_dense1000():
    """One update batch of the 1000 x 1000 stream (t = 50 slices, P = 12,
    Q = 60, S = 3) against the FP64 oracle, every replica."""
    c = synth.C2
    t = 50
    g = np.random.Generator(np.random.PCG64(synth.seed_of(2, 1)))
    A = g.random((c.I, c.R)); B = g.random((c.J, c.R)); C = g.random((t, c.R))
    X = (np.einsum("ir,jr,kr->kij", A, B, C) + 0.01 * g.standard_normal((t, c.I, c.J))).astype(np.float32)
    U, V = synth.compression_UV(c.I, c.J, c.P, c.Q, c.S, c.config_id)
    W = synth.temporal_W(t, c.M1, c.config_id, 1)
    print("[mfma] full-size oracle", file=sys.stderr, flush=True)
    ref = compress_dense(X.astype(np.float64), U, V, W, c.P, c.Q, c.S)
    for dt, tol in (("f32", 1e-5), ("bf16", 2e-2)):
        z = _gpu_Z(c.I, c.J, c.P, c.Q, c.S, X, U, V, W, dt)
        errs = [rel(z[p], ref[p]) for p in range(c.P)]
        print(f"[mfma] full-size {dt} max rel {max(errs):.3e}", file=sys.stderr, flush=True)
        assert max(errs) <= tol, (dt, errs)
