"""Pins of the bfloat16 emulation used to check the matrix-core path."""
import numpy as np

from oracle.precision import round_bf16, compress_dense_bf16_emulated
from oracle import compress_dense


def test_round_bf16_known_values():
    # exactly representable values are unchanged
    for v in (0.0, 1.0, -2.5, 0.15625, 3.0 * 2 ** -100):
        assert round_bf16(v) == np.float32(v)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to even (1.0)
    assert round_bf16(1 + 2 ** -8) == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6
    assert round_bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    # just above halfway rounds up
    assert round_bf16(np.float32(1 + 2 ** -8 + 2 ** -20)) == 1 + 2 ** -7


def test_round_bf16_relative_error_bound(rng):
    x = rng.standard_normal(10000).astype(np.float32)
    r = round_bf16(x)
    assert np.all(np.abs(r - x) <= 2 ** -8 * np.abs(x) + 1e-45)   # unit roundoff 2^-8
    # 8 significant bits: the low 16 bits of the float32 pattern are zero
    assert np.all((r.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


def test_emulation_close_to_exact(rng):
    I, J, t, P, Q, S = 20, 18, 3, 2, 5, 2
    M1 = S + P * (Q - S)
    X = rng.standard_normal((t, I, J)).astype(np.float32)
    U, V, W = rng.standard_normal((I, M1)), rng.standard_normal((J, M1)), rng.standard_normal((t, M1))
    e = compress_dense_bf16_emulated(X, U, V, W, P, Q, S)
    z = compress_dense(X.astype(np.float64), U, V, W, P, Q, S)
    err = np.linalg.norm(e - z) / np.linalg.norm(z)
    assert 1e-4 < err < 2e-2
