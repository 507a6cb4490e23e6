"""Pins of the fitness measure (Sec. 5.1) and of the identifiability checks
(Eq. 4, Eq. 8 with the worked example of Sec. 5.4.3)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import fit_dense, fit_coo_identity, identifiability, p_min_bound

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_fit_exact_model_is_one(rng):
    A = rng.random((6, 2)); B = rng.random((5, 2)); C = rng.random((4, 2))
    X = np.einsum("ir,jr,kr->kij", A, B, C)
    f, sse, nx = fit_dense(X, A, B, C)
    assert abs(f - 1.0) <= 1e-7 and sse <= 1e-25 * nx + 1e-28


def test_fit_zero_model_is_zero(rng):
    X = rng.standard_normal((3, 4, 5))
    Z = np.zeros((4, 2)), np.zeros((5, 2)), np.zeros((3, 2))
    f, sse, nx = fit_dense(X, *Z)
    assert f == pytest.approx(0.0, abs=1e-15) and sse == pytest.approx(nx)


def test_fit_slices_with_offset(rng):
    A = rng.random((6, 2)); B = rng.random((5, 2)); C = rng.random((9, 2))
    X = np.einsum("ir,jr,kr->kij", A, B, C) + 0.1 * rng.standard_normal((9, 6, 5))
    f_all, sse_all, nx_all = fit_dense(X, A, B, C)
    _, s1, n1 = fit_dense(X[:4], A, B, C, k0=0)
    _, s2, n2 = fit_dense(X[4:], A, B, C, k0=4)
    assert s1 + s2 == pytest.approx(sse_all, rel=1e-13)
    assert n1 + n2 == pytest.approx(nx_all, rel=1e-13)


def test_sparse_identity_equals_dense_direct(rng):
    I, J, K, R = 9, 8, 5, 3
    A = rng.random((I, R)); B = rng.random((J, R)); C = rng.random((K, R))
    mask = rng.random((K, I, J)) < 0.2
    X = np.where(mask, rng.standard_normal((K, I, J)), 0.0)
    k, i, j = np.nonzero(X)
    f_s, sse_s, nx_s = fit_coo_identity(k, i, j, X[k, i, j], A, B, C)
    f_d, sse_d, nx_d = fit_dense(X, A, B, C)
    assert sse_s == pytest.approx(sse_d, rel=1e-10)
    assert f_s == pytest.approx(f_d, abs=1e-10)


def test_fit_noise_floor(rng):
    """The true factors fit a noisy tensor at about 1 - ||N|| / ||X||."""
    A = rng.random((20, 3)); B = rng.random((20, 3)); C = rng.random((20, 3))
    Xc = np.einsum("ir,jr,kr->kij", A, B, C)
    N = 0.01 * rng.standard_normal(Xc.shape)
    f, _, _ = fit_dense(Xc + N, A, B, C)
    assert f == pytest.approx(1 - np.linalg.norm(N) / np.linalg.norm(Xc + N), abs=1e-12)


def test_eq8_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "eq8_worked_example.json")))
    x = g["inputs"]
    ratios = [a / b for a, b in g["printed_fractions"]]
    pmin = p_min_bound(x["I"], x["J"], x["K"], x["Q"], x["shared"])
    assert pmin == pytest.approx(max(ratios), abs=1e-12)
    assert math.ceil(pmin) == g["p_min_printed_approx"]


def test_identifiability_bits():
    # 50^3, P=4, Q=20, S=3: M1 = 71 >= 50, Eq. 8 bound 2.76 -> 3 <= 4
    bits, pmin = identifiability(50, 50, 50, 10, 5, 4, 20, 3)
    assert bits == 0b11111 and math.ceil(pmin) == 3
    # 1000^3, P=12, Q=60: M1 = 687 < 1000, bound 16.9 -> 17 > 12
    bits, pmin = identifiability(1000, 1000, 1000, 50, 10, 12, 60, 3)
    assert bits & 1 == 0 and bits & 2 == 0 and bits & 4 == 0 and bits & 8
    # Eq. 4: 3 * min(Q, R) >= 2R + 2 fails for R = 1
    bits, _ = identifiability(50, 50, 50, 10, 1, 4, 20, 3)
    assert bits & 16 == 0
