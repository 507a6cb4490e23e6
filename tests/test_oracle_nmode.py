"""Pins of the N-mode oracle (supplement, higher-order extension)."""
import numpy as np

from oracle import OctenOracle, compress_dense, cp_als, fit_dense
from oracle.nmode import (OctenNOracle, compress_dense_n, cp_als_n, fit_dense_n, mttkrp_n)
from oracle.octen_oracle import replica_cols


def _stream(rng, dims, K, R, sigma=0.0):
    fac = [rng.random((d, R)) for d in dims]
    C = rng.random((K, R))
    letters = "abcdefg"[:len(dims)]
    X = np.einsum("kr," + ",".join(l + "r" for l in letters) + "->k" + letters, C, *fac)
    return fac, C, X + sigma * rng.standard_normal(X.shape)


def test_three_modes_is_the_three_mode_oracle(rng):
    """At N = 3 every step equals the (pinned) three-mode oracle's."""
    I, J, R, P, Q, S = 14, 12, 3, 3, 7, 2
    M1 = S + P * (Q - S)
    _, _, X = _stream(rng, (I, J), 20, R, 0.01)
    U = rng.standard_normal((I, M1)); V = rng.standard_normal((J, M1))
    Ws = [rng.standard_normal((t, M1)) for t in (12, 4, 4)]
    init = rng.standard_normal((P, 3, Q, R))
    a = OctenOracle(I, J, R, P, Q, S, U, V)
    b = OctenNOracle((I, J), R, P, Q, S, [U, V])
    k0 = 0
    for bi, W in enumerate(Ws):
        t = W.shape[0]
        Za = a.compress_batch(X[k0:k0 + t], W)
        Zb = b.compress_batch(X[k0:k0 + t], W)
        assert np.allclose(Za, Zb, rtol=1e-13, atol=1e-13)
        a.update_replicas(); b.update_replicas()
        a.cp_als_replicas(15, init=init if bi == 0 else None)
        b.cp_als_replicas(15, init=init if bi == 0 else None)
        assert np.allclose(a.F, b.F, rtol=1e-11, atol=1e-12)
        A, B, C = a.recover_factors()
        (An, Bn), Cn = b.recover_factors()
        for x, y in ((A, An), (B, Bn), (C, Cn)):
            assert np.allclose(x, y, rtol=1e-9, atol=1e-10)
        k0 += t
    assert abs(fit_dense(X, A, B, C)[0] - fit_dense_n(X, [An, Bn], Cn)[0]) <= 1e-10


def test_compression_four_modes_brute_force(rng):
    dims, t, P, Q, S = (3, 4, 2), 3, 2, 3, 1
    M1 = S + P * (Q - S)
    X = rng.standard_normal((t,) + dims)
    Us = [rng.standard_normal((d, M1)) for d in dims]
    W = rng.standard_normal((t, M1))
    Z = compress_dense_n(X, Us, W, P, Q, S)
    for p in range(P):
        c = replica_cols(P, Q, S, p)
        for q1 in range(Q):
            for q2 in range(Q):
                for q3 in range(Q):
                    for qt in range(Q):
                        s = 0.0
                        for k in range(t):
                            for i in range(dims[0]):
                                for j in range(dims[1]):
                                    for l in range(dims[2]):
                                        s += (X[k, i, j, l] * Us[0][i, c[q1]] * Us[1][j, c[q2]] *
                                              Us[2][l, c[q3]] * W[k, c[qt]])
                        assert abs(Z[p, q1, q2, q3, qt] - s) <= 1e-12 * (1 + abs(s))


def test_compression_is_linear_in_the_batch(rng):
    dims, P, Q, S = (5, 4, 6), 3, 4, 2
    M1 = S + P * (Q - S)
    Us = [rng.standard_normal((d, M1)) for d in dims]
    X1 = rng.standard_normal((3,) + dims); X2 = rng.standard_normal((2,) + dims)
    W1 = rng.standard_normal((3, M1)); W2 = rng.standard_normal((2, M1))
    whole = compress_dense_n(np.concatenate([X1, X2]), Us, np.vstack([W1, W2]), P, Q, S)
    parts = compress_dense_n(X1, Us, W1, P, Q, S) + compress_dense_n(X2, Us, W2, P, Q, S)
    assert np.allclose(whole, parts, rtol=1e-12, atol=1e-12)


def test_mttkrp_n_against_loops(rng):
    Q, R = 3, 2
    Y = rng.standard_normal((Q, Q, Q, Q))
    F = [rng.standard_normal((Q, R)) for _ in range(4)]
    for n in range(4):
        M = mttkrp_n(Y, F, n)
        for q in range(Q):
            for r in range(R):
                s = 0.0
                for idx in np.ndindex(Q, Q, Q, Q):
                    if idx[n] != q:
                        continue
                    pr = Y[idx]
                    for m in range(4):
                        if m != n:
                            pr *= F[m][idx[m], r]
                    s += pr
                assert abs(M[q, r] - s) <= 1e-12


def test_als_recovers_planted_four_mode_rank(rng):
    Q, R = 8, 3
    F = [rng.standard_normal((Q, R)) for _ in range(4)]
    Y = np.einsum("ar,br,cr,dr->abcd", *F)
    init = [f + 0.2 * rng.standard_normal(f.shape) for f in F]
    G, lam, fb = cp_als_n(Y, init, 60)
    Yh = np.einsum("r,ar,br,cr,dr->abcd", lam, *G)
    assert not fb and np.linalg.norm(Yh - Y) / np.linalg.norm(Y) < 1e-8


def test_noiseless_four_mode_stream_is_recovered():
    """An exactly rank-R 4-mode stream with determined non-temporal modes
    (M1 >= I_n) and batches no wider than M1 is recovered with fit >= 0.9999
    after every batch.  The first ALS call starts near the planted replica
    factors (U_n[:, cols_p]^T A_n and W[:, cols_p]^T C, perturbed by 1e-3), so
    that the check is on matching and recovery, not on where ALS from a
    random start lands in a fixed number of sweeps."""
    rng = np.random.default_rng(20180705)
    dims, R, P, Q, S = (10, 9, 8), 2, 4, 6, 3
    M1 = S + P * (Q - S)
    fac, Ct, X = _stream(rng, dims, 30, R)
    Us = [rng.standard_normal((d, M1)) for d in dims]
    o = OctenNOracle(dims, R, P, Q, S, Us)
    k0 = 0
    for b, t in enumerate((12, 9, 9)):
        W = rng.standard_normal((t, M1))
        init = None
        if b == 0:
            init = np.empty((P, 4, Q, R))
            for p in range(P):
                c = replica_cols(P, Q, S, p)
                for n in range(3):
                    init[p, n] = Us[n][:, c].T @ fac[n]
                init[p, 3] = W[:, c].T @ Ct[:t]
            init += 1e-3 * rng.standard_normal(init.shape)
        o.compress_batch(X[k0:k0 + t], W)
        o.update_replicas()
        o.cp_als_replicas(300, init=init)
        As, C = o.recover_factors()
        k0 += t
        assert fit_dense_n(X[:k0], As, C)[0] >= 0.9999, b
