"""Pins of the FP64 warm-start reference: finite differences, closed forms of
Adam, special cases of the sketch, and round trips of the column maps."""
import numpy as np
import pytest

from oracle.warmstart import (adam_step, candidate_init, column_signs, judge, mlp_backward,
                              mlp_forward, mlp_param_shapes, mode3_change, mse_loss,
                              replica_fit_of, sketch, warmstart_features, warmstart_targets)


def _params(rng, n_in, n_h, n_out, scale=0.4):
    return [scale * rng.standard_normal(s) for s in mlp_param_shapes(n_in, n_h, n_out)]


def test_gradients_match_central_differences(rng):
    n_in, n_h, n_out, n = 11, 7, 6, 9
    params = _params(rng, n_in, n_h, n_out)
    X = rng.standard_normal((n, n_in))
    T = rng.standard_normal((n, n_out))
    Y, cache = mlp_forward(params, X, n_out)
    # stay away from the rectifier kinks so that differences are smooth
    assert np.min(np.abs(cache[1])) > 1e-3 and np.min(np.abs(cache[3])) > 1e-3
    L, dY = mse_loss(Y, T)
    grads = mlp_backward(params, cache, dY)
    h = 1e-6
    for w, g in zip(params, grads):
        num = np.zeros_like(w)
        for idx in np.ndindex(w.shape):
            old = w[idx]
            w[idx] = old + h
            lp = mse_loss(mlp_forward(params, X, n_out)[0], T)[0]
            w[idx] = old - h
            lm = mse_loss(mlp_forward(params, X, n_out)[0], T)[0]
            w[idx] = old
            num[idx] = (lp - lm) / (2 * h)
        assert np.linalg.norm(num - g) <= 1e-6 * np.linalg.norm(g)


def test_zero_last_layer_is_the_identity_on_the_columns(rng):
    params = _params(rng, 10, 5, 6)
    params[4][:] = 0.0
    params[5][:] = 0.0
    X = rng.standard_normal((4, 10))
    Y, _ = mlp_forward(params, X, 6)
    assert np.array_equal(Y, X[:, :6])


def test_adam_first_step_closed_form(rng):
    w0 = rng.standard_normal(5)
    g = rng.standard_normal(5)
    w = [w0.copy()]
    m, v = [np.zeros(5)], [np.zeros(5)]
    adam_step(w, [g], m, v, 1, lr=0.01, eps=1e-8)
    # bias-corrected moments are g and g^2 after one step
    assert np.allclose(w[0], w0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_adam_minimises_a_quadratic(rng):
    target = rng.standard_normal(4)
    w = [np.zeros(4)]
    m, v = [np.zeros(4)], [np.zeros(4)]
    for step in range(1, 3001):
        adam_step(w, [w[0] - target], m, v, step, lr=0.01)
    assert np.linalg.norm(w[0] - target) < 1e-3


def test_sketch_special_cases(rng):
    P, Q, D = 3, 4, 5
    Z = rng.standard_normal((P, Q, Q, Q))
    G = rng.standard_normal((D, Q ** 3))
    s = sketch(Z, G)
    assert np.allclose(sketch(3.5 * Z, G), s, rtol=1e-13, atol=1e-13)   # scale-free
    assert np.allclose(sketch(-Z, G), -s, rtol=1e-13, atol=1e-13)
    # rows of G that pick single entries give those entries over the norm
    idx = [0, 7, 21, 63, 40]
    E = np.zeros((D, Q ** 3)); E[np.arange(D), idx] = 1.0
    pick = sketch(Z, E)
    for p in range(P):
        z = Z[p].reshape(-1)
        assert np.allclose(pick[p], z[idx] / np.sqrt(np.sum(z * z)), rtol=1e-14)
    assert np.all(sketch(np.zeros_like(Z), G) == 0)


def test_column_signs():
    x = np.array([[1.0, -3.0, 0.0], [-2.0, 3.0, 0.0]])
    # column 0: largest magnitude -2; column 1: tie, the first (-3) wins; zero column: +1
    assert column_signs(x).tolist() == [-1.0, -1.0, 1.0]


def test_features_targets_round_trip_and_sign_invariance(rng):
    P, Q, R, D = 2, 5, 3, 4
    F = rng.standard_normal((P, 3, Q, R))
    F /= np.linalg.norm(F, axis=2, keepdims=True)
    lam = rng.uniform(0.5, 3.0, (P, R))
    sk = rng.standard_normal((P, D))
    Z = rng.standard_normal((P, Q, Q, Q))
    X, signs = warmstart_features(F, lam, sk, Z)
    assert X.shape == (P * R, 4 * Q + D)
    T = warmstart_targets(F, lam, signs)
    # the third block is c + u, the fourth u
    assert np.allclose(T[:, :2 * Q], X[:, :2 * Q], rtol=0, atol=1e-15)
    assert np.allclose(T[:, 2 * Q:], X[:, 2 * Q:3 * Q] - X[:, 3 * Q:4 * Q], rtol=1e-12, atol=1e-12)
    back = candidate_init(T, signs, Q)
    c = np.cbrt(lam)[:, None, None, :]
    assert np.allclose(back, F * c, rtol=1e-14, atol=1e-15)
    # flipping a column in modes 1 and 3 (same rank-one term) leaves the features alone
    G = F.copy()
    G[:, 0, :, 1] *= -1
    G[:, 2, :, 1] *= -1
    X2, _ = warmstart_features(G, lam, sk, Z)
    assert np.allclose(X2, X, rtol=0, atol=1e-14)


def test_mode3_change_is_the_rank_one_least_squares_update(rng):
    """For rank one, c + u is the mode-3 least-squares column of Y + Z when
    c was that of Y (Sec. 2: the mode-3 normal equations with a, b held)."""
    from oracle import mttkrp, solve_normal, gram_hadamard
    Q = 7
    Y = rng.standard_normal((Q, Q, Q))
    Z = rng.standard_normal((Q, Q, Q))
    a = rng.standard_normal((Q, 1)); b = rng.standard_normal((Q, 1))

    def ls_c(T):
        F = [a, b, np.zeros((Q, 1))]
        return solve_normal(mttkrp(T, F, 2), gram_hadamard(F, 2))[0][:, 0]

    c = ls_c(Y)
    assert np.allclose(c + mode3_change(Z, a[:, 0], b[:, 0]), ls_c(Y + Z), rtol=1e-12, atol=1e-12)


def test_replica_fit_matches_gram_identity(rng):
    from oracle import replica_fit
    Q, R = 6, 3
    Y = rng.standard_normal((Q, Q, Q))
    F = [rng.standard_normal((Q, R)) for _ in range(3)]
    lam = np.ones(R)
    M3 = np.einsum("abc,ar,br->cr", Y, F[0], F[1])
    assert abs(replica_fit_of(Y, *F) - replica_fit(Y, F, lam, M3)) < 1e-12


def test_judge_keeps_better_or_equal_candidates(rng):
    P, Q, R = 2, 5, 2
    F = rng.standard_normal((P, 3, Q, R))
    F /= np.linalg.norm(F, axis=2, keepdims=True)
    lam = rng.uniform(1.0, 2.0, (P, R))
    c = np.cbrt(lam)[:, None, None, :]
    exact = F * c
    Y = np.stack([np.einsum("ar,br,cr->abc", *exact[p]) for p in range(P)])
    # replica 0: the plain start itself (a tie keeps the candidate);
    # replica 1: a perturbed start, worse than the exact plain one
    cand = exact.copy()
    cand[1] += 0.3 * rng.standard_normal(cand[1].shape)
    chosen, keep = judge(Y, cand, F, lam)
    assert keep.tolist() == [True, False]
    assert np.allclose(chosen[1], exact[1])
