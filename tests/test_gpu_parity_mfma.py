"""GPU parity of the matrix-core compression (Sec. 4.1, Eq. 1) on f32 slices.

Every form is checked twice:
  * entrywise against its own definition (the FP64 compression of its
    rounded inputs, `oracle.precision.compress_rounded`) within the stated
    rounding-error bound of its arithmetic (`oracle.precision.error_bound`:
    float32 accumulation of both sums, the carry of the intermediate
    product, Higham-Mary probabilistic constants at lambda = 8);
  * normwise per replica against the FP64 oracle: FP32 within 1e-5, BF16
    within 2e-2, the two-term BF16 form within 1e-4 (its inputs carry 16
    significant bits: 2^-16 relative, far inside that bar for these data).
Shapes cover several row and column blocks with ragged tails, the
register-staged path (J not a multiple of 4: 16-byte loads inside a row,
guarded scalar loads at its end) at one, two and three 32-wide tiles per
replica side, Q > 64 and a single slice.  The compression matrices are on the bfloat16 grid, as
the two-term form requires.
"""
import sys

import numpy as np
import pytest

from oracle import compress_dense
from oracle.precision import compress_rounded, error_bound
from paper_1807_01350_amd import synth
from tests.stream_helpers import rel

pytestmark = pytest.mark.gpu

SHAPES = [
    # name, I, J, t, P, Q, S
    ("c2_like", 300, 260, 7, 12, 60, 3),       # 3 column blocks, ragged rows and j
    ("odd_j", 150, 97, 5, 5, 24, 3),           # J % 4 != 0: register-staged loads
    ("odd_j_split", 140, 203, 3, 16, 20, 3),   # J % 4 != 0, 14 replicas per tile (two-term: 4 passes)
    ("odd_j_q50", 120, 131, 3, 6, 50, 3),      # J % 4 != 0, two 32-wide tiles (two-term: 2 passes)
    ("odd_j_q80", 100, 77, 2, 3, 80, 3),       # J % 4 != 0, three 32-wide tiles
    ("q80", 200, 200, 4, 4, 80, 3),            # three 32-wide tiles per replica side
    ("single_slice", 129, 64, 1, 2, 20, 2),    # t = 1, one row past a block
]

NORM_BAR = {"f32": 1e-5, "bf16": 2e-2, "bf16x2": 1e-4}


def _inputs(I, J, t, P, Q, S, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    M1 = S + P * (Q - S)
    X = g.random((t, I, J)).astype(np.float32)
    U = synth.to_bf16_grid(g.standard_normal((I, M1)))
    V = synth.to_bf16_grid(g.standard_normal((J, M1)))
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
@pytest.mark.parametrize("form", ["f32", "bf16", "bf16x2"])
def test_compression_forms(shape, form):
    name, I, J, t, P, Q, S = shape
    print(f"[mfma] {name} {form}", file=sys.stderr, flush=True)
    X, U, V, W = _inputs(I, J, t, P, Q, S, 7 + I)
    ref = compress_dense(X.astype(np.float64), U, V, W, P, Q, S)
    dfn = compress_rounded(form, X, U, V, W, P, Q, S)
    bnd = error_bound(form, X, U, V, W, P, Q, S)
    z = _gpu_Z(I, J, P, Q, S, X, U, V, W, form)
    ratio = np.max(np.abs(z - dfn) / bnd)
    nrm = max(rel(z[p], ref[p]) for p in range(P))
    print(f"[mfma] {name} {form}: error / bound {ratio:.3f}, normwise vs FP64 {nrm:.2e}",
          file=sys.stderr, flush=True)
    assert np.all(np.abs(z - dfn) <= bnd), ratio
    for p in range(P):
        assert rel(z[p], ref[p]) <= NORM_BAR[form], (p, rel(z[p], ref[p]))


def test_power_of_two_slice_scale_is_exact():
    I, J, t, P, Q, S = 140, 96, 3, 4, 20, 3
    X, U, V, W = _inputs(I, J, t, P, Q, S, 5)
    scale = np.array([2.0 ** -3, 1.0, 2.0 ** 5], dtype=np.float32)
    for dt in ("f32", "bf16", "bf16x2"):
        a = _gpu_Z(I, J, P, Q, S, X, U, V, W, dt)
        b = _gpu_Z(I, J, P, Q, S, X, U, V, W, dt, scale)
        assert np.array_equal(a, b), dt


def test_two_term_form_needs_bf16_grid():
    """Compression matrices off the bfloat16 grid are refused by the
    two-term form (it would round them) and accepted by the others."""
    import torch
    from paper_1807_01350_amd import octen as oc
    g = np.random.Generator(np.random.PCG64(3))
    I, J, P, Q, S = 40, 36, 2, 8, 2
    M1 = S + P * (Q - S)
    U = torch.from_numpy(g.standard_normal((I, M1))).cuda()
    V = torch.from_numpy(synth.to_bf16_grid(g.standard_normal((J, M1)))).cuda()
    with pytest.raises(oc.OctenError) as ei:
        oc.Octen(I, J, 2, P, Q, S, U, V, x_dtype="f32", compress_dtype="bf16x2")
    assert ei.value.status == oc.OCTEN_ERR_ARG
    oc.Octen(I, J, 2, P, Q, S, U, V, x_dtype="f32", compress_dtype="bf16").close()


def test_full_size_batch_dense1000():
    """One update batch of the 1000 x 1000 stream (t = 50 slices, P = 12,
    Q = 60, S = 3) against the FP64 oracle, every replica, every form."""
    c = synth.C2
    t = 50
    g = np.random.Generator(np.random.PCG64(synth.seed_of(2, 1)))
    A = g.random((c.I, c.R)); B = g.random((c.J, c.R)); C = g.random((t, c.R))
    X = (np.einsum("ir,jr,kr->kij", A, B, C) + 0.01 * g.standard_normal((t, c.I, c.J))).astype(np.float32)
    U, V = synth.compression_UV(c.I, c.J, c.P, c.Q, c.S, c.config_id)
    W = synth.temporal_W(t, c.M1, c.config_id, 1)
    print("[mfma] full-size oracle", file=sys.stderr, flush=True)
    ref = compress_dense(X.astype(np.float64), U, V, W, c.P, c.Q, c.S)
    for dt in ("f32", "bf16", "bf16x2"):
        z = _gpu_Z(c.I, c.J, c.P, c.Q, c.S, X, U, V, W, dt)
        errs = [rel(z[p], ref[p]) for p in range(c.P)]
        print(f"[mfma] full-size {dt} max rel {max(errs):.3e}", file=sys.stderr, flush=True)
        assert max(errs) <= NORM_BAR[dt], (dt, errs)
