"""Pins of the oracle's two-term bfloat16 replica ALS (Sec. 4.1, the
per-replica CP-ALS, with the slab contractions on two-term operands)."""
import struct

import numpy as np

from oracle import cp_als
from oracle.precision import cp_als_two_term, two_term_product


def _bf16(v):
    """Nearest bfloat16 (ties to even) of the float32 value of v, from the
    IEEE bit pattern: keep the top 16 bits after adding half an ulp."""
    b = struct.unpack("<I", struct.pack("<f", v))[0]
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return struct.unpack("<f", struct.pack("<I", b))[0]


def _pair(v):
    f = struct.unpack("<f", struct.pack("<f", v))[0]     # float32 value
    hi = _bf16(f)
    lo = _bf16(struct.unpack("<f", struct.pack("<f", f - hi))[0])
    return hi, lo


def _tt(x, y):
    xh, xl = _pair(x)
    yh, yl = _pair(y)
    return xh * yh + xl * yh + xh * yl


def test_two_term_product_brute_force(rng):
    X = rng.standard_normal((3, 4)) * np.exp(rng.uniform(-3, 3, (3, 4)))
    B = rng.standard_normal((4, 2))
    got = two_term_product(X, B)
    for i in range(3):
        for r in range(2):
            want = sum(_tt(float(X[i, k]), float(B[k, r])) for k in range(4))
            assert abs(got[i, r] - want) <= 1e-15 * sum(abs(X[i, k] * B[k, r]) for k in range(4))


def test_two_term_product_error_bound(rng):
    # each operand keeps 16 significant bits (|x - hi - lo| <= 2^-16 |x|) and
    # the dropped lo*lo term is below 2^-16 |x y|: at most 3 * 2^-16 per
    # product, plus the float32 rounding of the operands
    X = rng.standard_normal((50, 40))
    B = rng.standard_normal((40, 30))
    err = np.abs(two_term_product(X, B) - X @ B)
    bound = (3 * 2.0 ** -16 + 2 * 2.0 ** -24) * (np.abs(X) @ np.abs(B))
    assert np.all(err <= bound)
    # the bound tells the cross terms apart: dropping one of them, or both,
    # breaks it
    from oracle.precision import split_bf16
    xh, xl = split_bf16(X.astype(np.float32))
    bh, bl = split_bf16(B.astype(np.float32))
    for wrong in (xh @ bh, xh @ bh + xl @ bh, xh @ bh + xh @ bl):
        assert np.any(np.abs(wrong - X @ B) > bound)


def _sweep_brute(Y, init):
    """One Gauss-Seidel sweep written with explicit loops (Q, R tiny)."""
    Q = Y.shape[0]
    R = init[0].shape[1]
    A, B, C = [np.array(f, dtype=np.float64) for f in init]

    def solve(M, G):
        X = np.linalg.solve(G, M.T).T
        n = np.sqrt((X * X).sum(axis=0))
        return X / n, n

    T = np.zeros((Q, Q, R))
    for a in range(Q):
        for b in range(Q):
            for r in range(R):
                T[a, b, r] = sum(_tt(float(Y[a, b, c]), float(C[c, r])) for c in range(Q))
    M1 = np.array([[sum(T[a, b, r] * B[b, r] for b in range(Q)) for r in range(R)]
                   for a in range(Q)])
    A, _ = solve(M1, (B.T @ B) * (C.T @ C))
    M2 = np.array([[sum(T[a, b, r] * A[a, r] for a in range(Q)) for r in range(R)]
                   for b in range(Q)])
    B, _ = solve(M2, (A.T @ A) * (C.T @ C))
    M3 = np.zeros((Q, R))
    for c in range(Q):
        for r in range(R):
            M3[c, r] = sum(_tt(float(Y[a, b, c]), float(np.float32(A[a, r] * B[b, r])))
                           for a in range(Q) for b in range(Q))
    C, lam = solve(M3, (A.T @ A) * (B.T @ B))
    return [A, B, C], lam


def test_one_sweep_brute_force(rng):
    Q, R = 4, 2
    Y = rng.standard_normal((Q, Q, Q)).astype(np.float32)
    init = [rng.standard_normal((Q, R)) for _ in range(3)]
    F, lam, done, fb = cp_als_two_term(Y, init, 1)
    Fb, lamb = _sweep_brute(Y, init)
    assert done == 1 and not fb
    for f, g in zip(F, Fb):
        assert np.allclose(f, g, rtol=1e-11, atol=1e-13)
    assert np.allclose(lam, lamb, rtol=1e-11)


def test_converges_with_the_fp64_als(rng):
    # an exactly rank-R replica: both forms recover it, and agree to the
    # two-term precision
    Q, R = 12, 3
    A, B, C = [rng.standard_normal((Q, R)) for _ in range(3)]
    Y = np.einsum("ar,br,cr->abc", A, B, C).astype(np.float32)
    init = [f + 0.3 * rng.standard_normal((Q, R)) for f in (A, B, C)]
    F1, l1, _, _ = cp_als(Y.astype(np.float64), init, 40)
    F2, l2, _, _ = cp_als_two_term(Y, init, 40)
    X1 = np.einsum("r,ar,br,cr->abc", l1, *F1)
    X2 = np.einsum("r,ar,br,cr->abc", l2, *F2)
    nY = np.linalg.norm(Y)
    assert np.linalg.norm(X1 - Y) / nY < 1e-6
    assert np.linalg.norm(X2 - Y) / nY < 1e-4
    for f, g in zip(F1, F2):
        assert np.linalg.norm(f - g) / np.linalg.norm(f) < 1e-3


def test_tolerance_stops_early(rng):
    Q, R = 8, 2
    A, B, C = [rng.standard_normal((Q, R)) for _ in range(3)]
    Y = np.einsum("ar,br,cr->abc", A, B, C).astype(np.float32)
    init = [f + 0.1 * rng.standard_normal((Q, R)) for f in (A, B, C)]
    _, _, done, _ = cp_als_two_term(Y, init, 200, tol=1e-6)
    assert 2 <= done < 200
