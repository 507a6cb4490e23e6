"""Pins of factor matching (Sec. 4.2, Eq. 5) and the least-squares update
(Sec. 4.3, Eq. 6, Eq. 7), plus the temporal reading R-C1."""
import math

import numpy as np
import pytest

from oracle import (distribute_lambda, greedy_assign, match_replicas, stack_rhs,
                    weighted_minnorm_lstsq, canonicalize, match_previous, replica_cols,
                    OctenOracle, fit_dense)
from paper_1807_01350_amd import synth


def test_lambda_distribution_keeps_model(rng):
    Q, R = 6, 3
    F = [rng.standard_normal((Q, R)) for _ in range(3)]
    lam = rng.random(R) + 0.1
    G = distribute_lambda(F, lam)
    a = np.einsum("ar,br,cr,r->abc", F[0], F[1], F[2], lam)
    b = np.einsum("ar,br,cr->abc", G[0], G[1], G[2])
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a)) * 10


def test_greedy_assign_basic_and_ties():
    sim = np.array([[0.1, 0.9, 0.2], [0.8, 0.85, 0.3], [0.05, 0.2, 0.7]])
    perm, margin = greedy_assign(sim)
    assert list(perm) == [1, 0, 2]
    assert margin == pytest.approx(0.05)
    # exact tie: smallest column first, then smallest row
    tie = np.array([[0.5, 0.5], [0.5, 0.5]])
    perm, margin = greedy_assign(tie)
    assert list(perm) == [0, 1] and margin == 0.0
    # a permutation always results, even when every row prefers one column
    same = np.array([[0.9, 0.1, 0.1], [0.8, 0.2, 0.1], [0.7, 0.1, 0.3]])
    perm, _ = greedy_assign(same)
    assert sorted(perm) == [0, 1, 2]


def test_planted_permutation_and_scales_recovered(rng):
    """Replica factors built as (compression^T truth) Pi_p D_pn with
    D_p1 D_p2 D_p3 = I and random signs: the permutation is recovered exactly
    and the aligned factors equal the reference's convention to 1e-12."""
    I, J, t, R, P, Q, S = 30, 28, 20, 4, 5, 8, 3
    M1 = S + P * (Q - S)
    A = rng.random((I, R)); B = rng.random((J, R)); C = rng.random((t, R))
    U = rng.standard_normal((I, M1)); V = rng.standard_normal((J, M1)); W = rng.standard_normal((t, M1))
    truth = []
    for p in range(P):
        c = replica_cols(P, Q, S, p)
        truth.append([U[:, c].T @ A, V[:, c].T @ B, W[:, c].T @ C])
    Fs = np.zeros((P, 3, Q, R))
    perms = [np.arange(R)] + [rng.permutation(R) for _ in range(P - 1)]
    Ds = []
    for p in range(P):
        d1 = (rng.random(R) + 0.5) * rng.choice([-1, 1], R)
        d2 = (rng.random(R) + 0.5) * rng.choice([-1, 1], R)
        d3 = 1.0 / (d1 * d2)
        if p == 0:
            d1 = d2 = d3 = np.ones(R)
        Ds.append((d1, d2, d3))
        for n, d in enumerate((d1, d2, d3)):
            # replica column perms[p][r] holds true component r
            Fs[p, n][:, perms[p]] = truth[p][n] * d
    aligned, perm, scale, margins = match_replicas(Fs, S)
    for p in range(P):
        # replica column perms[p][r] must map to reference column r
        inv = np.empty(R, int); inv[perms[p]] = np.arange(R)
        assert np.array_equal(perm[p], inv)
        for n in range(3):
            assert np.linalg.norm(aligned[p, n] - truth[p][n]) <= 1e-12 * np.linalg.norm(truth[p][n])


def _literal_stack(Pt, rhs_list, P, Q, S):
    """Eq. 6 literally: per replica the rows of U_p^T (anchors repeated)."""
    rows, rhs = [], []
    for p in range(P):
        c = replica_cols(P, Q, S, p)
        rows.append(Pt[:, c].T)
        rhs.append(rhs_list[p])
    return np.vstack(rows), np.vstack(rhs)


@pytest.mark.parametrize("n", [25, 60])   # over- and under-determined
def test_dedup_weighted_equals_literal_stack(rng, n):
    P, Q, S, R = 4, 12, 3, 5
    M1 = S + P * (Q - S)
    Pt = rng.standard_normal((n, M1))
    per_rep = [rng.standard_normal((Q, R)) for _ in range(P)]
    Plit, rlit = _literal_stack(Pt, per_rep, P, Q, S)
    ref = np.linalg.pinv(Plit) @ rlit
    ref2 = np.linalg.lstsq(Plit, rlit, rcond=None)[0]
    rhs = stack_rhs(np.stack(per_rep), S)
    got = weighted_minnorm_lstsq(Pt, rhs, P, S)
    assert np.linalg.norm(ref - ref2) <= 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_exact_replica_factors_give_exact_factor(rng):
    I, R, P, Q, S = 40, 5, 5, 12, 3
    M1 = S + P * (Q - S)
    A = rng.random((I, R))
    U = rng.standard_normal((I, M1))
    per_rep = np.stack([U[:, replica_cols(P, Q, S, p)].T @ A for p in range(P)])
    got = weighted_minnorm_lstsq(U, stack_rhs(per_rep, S), P, S)
    assert np.linalg.norm(got - A) <= 1e-12 * np.linalg.norm(A)


def test_canonicalize_keeps_model_and_fixes_sign(rng):
    A = rng.standard_normal((7, 3)); B = rng.standard_normal((6, 3)); C = rng.standard_normal((5, 3))
    Ac, Bc, kappa = canonicalize(A, B)
    x1 = np.einsum("ir,jr,kr->ijk", A, B, C)
    x2 = np.einsum("ir,jr,kr->ijk", Ac, Bc, C * kappa)
    assert np.max(np.abs(x1 - x2)) <= 1e-13
    for M in (Ac, Bc):
        assert np.allclose(np.linalg.norm(M, axis=0), 1.0)
        idx = np.argmax(np.abs(M), axis=0)
        assert np.all(M[idx, np.arange(3)] > 0)
    # canonical form does not depend on the input scaling or sign
    Ac2, Bc2, _ = canonicalize(A * np.array([-2.0, 0.5, 3.0]), B * np.array([1.0, -1.0, 0.25]))
    assert np.allclose(Ac, Ac2, atol=1e-14) and np.allclose(Bc, Bc2, atol=1e-14)


def test_match_previous_recovers_permutation_and_sign(rng):
    A = rng.standard_normal((9, 4)); B = rng.standard_normal((8, 4))
    Ap, Bp, _ = canonicalize(A, B)
    pi = np.array([2, 0, 3, 1])
    sa = np.array([1, -1, 1, -1.0]); sb = np.array([1, 1, -1, -1.0])
    perm, signs, margin = match_previous(Ap[:, pi] * sa, Bp[:, pi] * sb, Ap, Bp)
    assert np.array_equal(perm, pi)
    assert np.array_equal(signs, sa * sb)
    assert margin > 0


def _run_stream(temporal, iters):
    c = synth.C1
    A, B, C, X = synth.dense_stream(c.I, c.J, c.K, c.R, c.sigma, c.config_id, noiseless=True)
    U, V = synth.compression_UV(c.I, c.J, c.P, c.Q, c.S, c.config_id)
    init = synth.als_init(c.P, c.Q, c.R, c.config_id)
    o = OctenOracle(c.I, c.J, c.R, c.P, c.Q, c.S, U, V, temporal=temporal)
    fits = []
    for b, (k0, t) in enumerate(c.schedule()):
        o.compress_batch(X[k0:k0 + t], synth.temporal_W(t, c.M1, c.config_id, b))
        o.update_replicas()
        o.cp_als_replicas(iters, init=init if b == 0 else None)
        Ah, Bh, Ch = o.recover_factors()
        fits.append(fit_dense(X[:o.K], Ah, Bh, Ch)[0])
    return o, fits


@pytest.fixture(scope="module")
def exact_streams():
    return _run_stream("incremental", 3000), _run_stream("full", 3000)


def test_noiseless_low_rank_stream_is_recovered(exact_streams):
    """Exactly low-rank noiseless stream, determined system (M1 >= I, J, K):
    fit >= 0.9999 after every batch."""
    (_, fits), _ = exact_streams
    assert min(fits) >= 0.9999


def test_incremental_and_full_temporal_readings_agree(exact_streams):
    """R-C1 (new rows only, with the carried history subtracted) equals R-C2
    (all rows re-solved) on exact data while K <= M1."""
    (o1, _), (o2, _) = exact_streams
    assert o1.K <= o1.M1
    assert np.linalg.norm(o1.C - o2.C) <= 1e-8 * np.linalg.norm(o2.C)
    assert np.linalg.norm(o1.A - o2.A) <= 1e-8
