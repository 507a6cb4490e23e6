"""Pins of the narrow-type definitions and of the rounding-error bound used to
check the matrix-core compression (Sec. 4.1, Eq. 1)."""
import numpy as np
import pytest

from oracle import compress_dense
from oracle.precision import (U_BF16, compress_rounded, error_bound, gamma, round_bf16,
                              rounded_inputs, split_bf16)
from oracle.octen_oracle import replica_cols


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
    assert np.all(np.abs(r - x) <= U_BF16 * np.abs(x) + 1e-45)
    # 8 significant bits: the low 16 bits of the float32 pattern are zero
    assert np.all((r.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


def test_split_bf16_holds_sixteen_bits(rng):
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32)
    hi, lo = split_bf16(x)
    # both parts are bfloat16 values
    for part in (hi, lo):
        assert np.all((part.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)
    # |x - hi - lo| <= 2^-16 |x| (two nearest roundings of 8 bits each)
    assert np.all(np.abs(x - hi - lo) <= 2.0 ** -16 * np.abs(x) * (1 + 2 ** -8))
    # a float32 value with at most 16 significant bits is split exactly
    y = np.float32(1 + 2 ** -3 + 2 ** -15)
    h, l = split_bf16(y)
    assert h + l == np.float64(y)
    assert h == 1.125 and l == 2.0 ** -15


def test_f32_definition_is_the_plain_compression(rng):
    I, J, t, P, Q, S = 9, 7, 2, 2, 4, 1
    M1 = S + P * (Q - S)
    X = rng.standard_normal((t, I, J)).astype(np.float32)
    U = round_bf16(rng.standard_normal((I, M1)))
    V = round_bf16(rng.standard_normal((J, M1)))
    W = rng.standard_normal((t, M1))
    a = compress_rounded("f32", X, U, V, W, P, Q, S)
    b = compress_dense(X.astype(np.float64), U, V, W, P, Q, S)
    assert np.array_equal(a, b)
    # the bf16x2 inputs sit within 2^-16 of the f32 ones
    Xr, _, _ = rounded_inputs("bf16x2", X, U, V)
    assert np.all(np.abs(Xr - X) <= 2.0 ** -16 * np.abs(X) * (1 + 2 ** -8))


def test_gamma_small_and_monotone():
    u = 2.0 ** -24
    assert gamma(1, 8.0, u) == pytest.approx(8 * u, rel=1e-6)
    assert gamma(100, 8.0, u) < gamma(400, 8.0, u) < 2 * gamma(100, 8.0, u) * 1.01


def _simulated_kernel(form, X, U, V, W, P, Q, S, rng, drop_lo=False):
    """The prescribed arithmetic, literally, in float32 scalar sums in a
    random order: T = x_hat V (float32 accumulation), carried in float32, as a
    bfloat16 value or as a bfloat16 pair, then M = U^T T in float32, then
    mode 3 in float64, stored as float32."""
    t, I, J = X.shape
    Xf = np.asarray(X, np.float32)
    if form == "bf16x2":
        hi, lo = split_bf16(Xf)
        parts = [hi.astype(np.float32)] + ([] if drop_lo else [lo.astype(np.float32)])
    elif form == "bf16":
        parts = [round_bf16(Xf).astype(np.float32)]
    else:
        parts = [Xf]
    Ur = (round_bf16(U) if form != "f32" else U).astype(np.float32)
    Vr = (round_bf16(V) if form != "f32" else V).astype(np.float32)
    Z = np.zeros((P, Q, Q, Q))
    for p in range(P):
        c = replica_cols(P, Q, S, p)
        M = np.zeros((t, Q, Q))
        for k in range(t):
            T = np.zeros((I, Q), np.float32)
            for i in range(I):
                for b in range(Q):
                    prods = np.concatenate([pp[k, i, :] * Vr[:, c[b]] for pp in parts])
                    acc = np.float32(0)
                    for v in prods[rng.permutation(prods.size)]:
                        acc = np.float32(acc + v)
                    T[i, b] = acc
            if form == "bf16":
                carried = [round_bf16(T).astype(np.float32)]
            elif form == "bf16x2":
                th, tl = split_bf16(T)
                carried = [th.astype(np.float32), tl.astype(np.float32)]
            else:
                carried = [T]
            for a in range(Q):
                for b in range(Q):
                    prods = np.concatenate([Ur[:, c[a]] * cc[:, b] for cc in carried])
                    acc = np.float32(0)
                    for v in prods[rng.permutation(prods.size)]:
                        acc = np.float32(acc + v)
                    M[k, a, b] = acc
        Z[p] = np.tensordot(M, W[:, c], axes=([0], [0])).astype(np.float32)
    return Z


@pytest.mark.parametrize("form", ["f32", "bf16", "bf16x2"])
def test_bound_covers_the_prescribed_arithmetic(form, rng):
    """Brute force: the arithmetic the bound is stated for, run literally in
    float32 with random summation orders, stays within the bound."""
    I, J, t, P, Q, S = 12, 40, 2, 2, 4, 1
    M1 = S + P * (Q - S)
    X = rng.random((t, I, J)).astype(np.float32)
    U = round_bf16(rng.standard_normal((I, M1)))
    V = round_bf16(rng.standard_normal((J, M1)))
    W = rng.standard_normal((t, M1))
    ref = compress_rounded(form, X, U, V, W, P, Q, S)
    bnd = error_bound(form, X, U, V, W, P, Q, S)
    for trial in range(2):
        z = _simulated_kernel(form, X, U, V, W, P, Q, S, rng)
        assert np.all(np.abs(z - ref) <= bnd), (form, trial, np.max(np.abs(z - ref) / bnd))


def test_bound_catches_a_dropped_low_part(rng):
    """A plausible mistake in a two-term kernel (the low part of x never
    multiplied) lands far outside the bf16x2 bound."""
    I, J, t, P, Q, S = 12, 40, 2, 2, 4, 1
    M1 = S + P * (Q - S)
    X = rng.random((t, I, J)).astype(np.float32)
    U = round_bf16(rng.standard_normal((I, M1)))
    V = round_bf16(rng.standard_normal((J, M1)))
    W = rng.standard_normal((t, M1))
    ref = compress_rounded("bf16x2", X, U, V, W, P, Q, S)
    bnd = error_bound("bf16x2", X, U, V, W, P, Q, S)
    z = _simulated_kernel("bf16x2", X, U, V, W, P, Q, S, rng, drop_lo=True)
    assert np.mean(np.abs(z - ref) > bnd) > 0.5
