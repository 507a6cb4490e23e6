"""End-to-end fit gate of the narrow compression forms: the whole update
(Algorithm 1: compress, add, replica ALS, match, recover) of a float32 stream
with the replica shape of the dense 1000^3 workload (P = 12, Q = 60, S = 3,
R = 10) at I = J = 600 (three row blocks and three column blocks of the
compression kernels), 200 initial slices then three batches of 50.  After
every batch the fitness of Sec. 5.1 of the GPU form must lie within 1e-3 of
the FP64 oracle's on the same inputs.

The FP32 and the two-term BF16 forms meet that bar, the latter also with
the ALS slab contractions in the two-term form.  The plain BF16 form
does not: rounding the slices to 8 significant bits moves the replica ALS,
which runs a fixed 50 sweeps from the same start, to a different point,
and the recovered fit differs by 1e-2 (it is reported, not gated).
"""
import sys

import numpy as np
import pytest

from tests.stream_helpers import Case, make_inputs, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

CASE = Case("gate600", I=600, J=600, R=10, P=12, Q=60, S=3, batches=(200, 50, 50, 50),
            config_id=2)
GATE = 1e-3

_cache = {}


def _oracle():
    if "o" not in _cache:
        X, U, V, Ws, init = make_inputs(CASE, x_dtype=np.float32)
        print("[gate] oracle run", file=sys.stderr, flush=True)
        _cache["in"] = (X, U, V, Ws, init)
        _cache["o"] = run_oracle(CASE, X.astype(np.float64), U, V, Ws, init)
    return _cache["in"], _cache["o"]


def _gap(form, als="f64"):
    (X, U, V, Ws, init), ref = _oracle()
    print(f"[gate] gpu run {form} (ALS contractions {als})", file=sys.stderr, flush=True)
    got = run_gpu(CASE, X, U, V, Ws, init, compress_dtype=form, x_dtype="f32", log=True,
                  als_dtype=als)
    gaps = []
    for b, (g, o) in enumerate(zip(got, ref)):
        gaps.append(abs(g["fit"] - o["fit"]))
        print(f"[gate] {form}/{als} batch {b}: fit {g['fit']:.6f} oracle {o['fit']:.6f} "
              f"|dfit| {gaps[-1]:.2e}", file=sys.stderr, flush=True)
    return gaps


@pytest.mark.parametrize("form,als", [("f32", "f64"), ("bf16x2", "f64"), ("bf16x2", "bf16x2")])
def test_fit_within_gate(form, als):
    gaps = _gap(form, als)
    assert max(gaps) <= GATE, gaps


def test_plain_bf16_reported():
    gaps = _gap("bf16")
    print(f"[gate] plain bf16 largest |dfit| {max(gaps):.2e} (bar {GATE:.0e}, not gated)",
          file=sys.stderr, flush=True)
    assert np.all(np.isfinite(gaps))
