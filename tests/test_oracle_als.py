"""Pins of the oracle's per-replica CP-ALS (Sec. 4.1 decomposition step, CP
model of Sec. 2) against loops, a library least-squares routine, the ALS
descent property, planted data and the rank-1 power method."""
import numpy as np
import pytest

from oracle import mttkrp, gram_hadamard, solve_normal, cp_als, replica_fit


def _cp(F, lam=None):
    R = F[0].shape[1]
    lam = np.ones(R) if lam is None else lam
    X = np.zeros((F[0].shape[0], F[1].shape[0], F[2].shape[0]))
    for r in range(R):
        X += lam[r] * F[0][:, r][:, None, None] * F[1][:, r][None, :, None] * F[2][:, r][None, None, :]
    return X


def test_mttkrp_matches_loops(rng):
    Q, R = 4, 3
    X = rng.standard_normal((Q, Q + 1, Q + 2))
    F = [rng.standard_normal((Q, R)), rng.standard_normal((Q + 1, R)), rng.standard_normal((Q + 2, R))]
    for n in range(3):
        M = mttkrp(X, F, n)
        ref = np.zeros((X.shape[n], R))
        for a in range(X.shape[0]):
            for b in range(X.shape[1]):
                for c in range(X.shape[2]):
                    idx = (a, b, c)
                    for r in range(R):
                        prod = X[a, b, c]
                        for m in range(3):
                            if m != n:
                                prod *= F[m][idx[m], r]
                        ref[idx[n], r] += prod
        assert np.max(np.abs(M - ref)) <= 1e-12


def test_mode_update_equals_library_lstsq(rng):
    """One mode update solves min ||X_(n) - F_n KR^T||: compare with
    numpy.linalg.lstsq on the explicitly unfolded problem."""
    Q, R = 6, 3
    X = rng.standard_normal((Q, Q, Q))
    F = [rng.standard_normal((Q, R)) for _ in range(3)]
    for n in range(3):
        others = [m for m in range(3) if m != n]
        # Khatri-Rao rows indexed by the pair of the two other indices
        KR = np.zeros((Q * Q, R))
        Xn = np.zeros((Q, Q * Q))
        row = 0
        for x in range(Q):
            for y in range(Q):
                KR[row] = F[others[0]][x] * F[others[1]][y]
                idx = [0, 0, 0]
                idx[others[0]] = x; idx[others[1]] = y
                for q in range(Q):
                    idx[n] = q
                    Xn[q, row] = X[tuple(idx)]
                row += 1
        ref = np.linalg.lstsq(KR, Xn.T, rcond=None)[0].T
        got, flag = solve_normal(mttkrp(X, F, n), gram_hadamard(F, n))
        assert not flag
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


def test_objective_non_increasing(rng):
    Q, R = 8, 4
    X = rng.random((Q, Q, Q))
    F = [rng.standard_normal((Q, R)) for _ in range(3)]
    prev = np.inf
    for _ in range(15):
        for n in range(3):
            Fn, _ = solve_normal(mttkrp(X, F, n), gram_hadamard(F, n))
            F[n] = Fn
            obj = np.linalg.norm(X - _cp(F))
            assert obj <= prev * (1 + 1e-12) + 1e-13
            prev = obj


def test_planted_exact_rank_recovered(rng):
    Q, R = 10, 4
    T = [rng.standard_normal((Q, R)) for _ in range(3)]
    X = _cp(T)
    init = [t + 1e-3 * rng.standard_normal(t.shape) for t in T]
    F, lam, done, flag = cp_als(X, init, 60)
    assert done == 60 and not flag
    assert np.linalg.norm(X - _cp(F, lam)) <= 1e-10 * np.linalg.norm(X)
    # columns are unit 2-norm after the sweep
    for f in F:
        assert np.allclose(np.linalg.norm(f, axis=0), 1.0, atol=1e-14)


def test_rank_one_equals_power_method(rng):
    """R = 1: ALS is the higher-order power method; compare with an
    independent power iteration on the same start."""
    Q = 7
    X = rng.random((Q, Q, Q))
    b0 = rng.standard_normal((Q, 1)); c0 = rng.standard_normal((Q, 1)); a0 = rng.standard_normal((Q, 1))
    F, lam, _, _ = cp_als(X, [a0, b0, c0], 40)
    b = b0[:, 0] / np.linalg.norm(b0); c = c0[:, 0] / np.linalg.norm(c0)
    for _ in range(40):
        a = np.tensordot(np.tensordot(X, c, axes=([2], [0])), b, axes=([1], [0])); a /= np.linalg.norm(a)
        b = np.tensordot(np.tensordot(X, c, axes=([2], [0])), a, axes=([0], [0])); b /= np.linalg.norm(b)
        c = np.tensordot(np.tensordot(X, b, axes=([1], [0])), a, axes=([0], [0]))
        sig = np.linalg.norm(c); c /= sig
    assert abs(lam[0] - sig) <= 1e-12 * sig
    for got, ref in zip(F, (a, b, c)):
        assert np.linalg.norm(np.abs(got[:, 0]) - np.abs(ref)) <= 1e-10


def test_replica_fit_matches_direct_residual(rng):
    Q, R = 9, 3
    X = rng.random((Q, Q, Q))
    init = [rng.standard_normal((Q, R)) for _ in range(3)]
    F, lam, _, _ = cp_als(X, init, 5)
    M3 = mttkrp(X, F, 2)
    direct = 1 - np.linalg.norm(X - _cp(F, lam)) / np.linalg.norm(X)
    assert abs(replica_fit(X, F, lam, M3) - direct) <= 1e-7


def test_tolerance_mode_stops_early(rng):
    Q, R = 10, 3
    T = [rng.standard_normal((Q, R)) for _ in range(3)]
    X = _cp(T)
    init = [t + 1e-4 * rng.standard_normal(t.shape) for t in T]
    _, _, done, _ = cp_als(X, init, 200, tol=1e-10)
    assert 2 <= done < 200


def test_singular_normal_matrix_uses_pseudo_inverse(rng):
    Q, R = 5, 3
    F = [rng.standard_normal((Q, R)) for _ in range(3)]
    F[1][:, 2] = F[1][:, 1]            # duplicated column -> rank-deficient Gram
    F[2][:, 2] = F[2][:, 1]
    M = rng.standard_normal((Q, R))
    G = gram_hadamard(F, 0)
    out, flag = solve_normal(M, G)
    assert flag
    ref = M @ np.linalg.pinv(G, rcond=1e-12, hermitian=True)
    assert np.linalg.norm(out - ref) <= 1e-8 * np.linalg.norm(ref)
