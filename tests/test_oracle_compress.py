"""Pins of the oracle's compression and summary update (Sec. 4.1, Eq. 1, Eq. 2)
against brute force, closed forms and special cases."""
import numpy as np
import pytest

from oracle import (compress_dense, compress_coo, compress_coo_entries, coo_segments, sort_coo,
                    update_summaries, replica_cols)
from paper_1807_01350_amd import synth


def _rand_problem(g, I, J, t, P, Q, S):
    M1 = S + P * (Q - S)
    X = g.standard_normal((t, I, J))
    U = g.standard_normal((I, M1))
    V = g.standard_normal((J, M1))
    W = g.standard_normal((t, M1))
    return X, U, V, W


def test_replica_columns_share_first_S():
    P, Q, S = 3, 5, 2
    cols = [replica_cols(P, Q, S, p) for p in range(P)]
    for c in cols:
        assert list(c[:S]) == [0, 1]
        assert len(c) == Q
    private = np.concatenate([c[S:] for c in cols])
    assert sorted(private) == list(range(S, S + P * (Q - S)))
    assert np.array_equal(replica_cols(P, Q, S, 1), synth.replica_columns(P, Q, S, 1))


def test_compress_matches_six_nested_loops(rng):
    I, J, t, P, Q, S = 5, 5, 3, 2, 3, 1
    X, U, V, W = _rand_problem(rng, I, J, t, P, Q, S)
    Z = compress_dense(X, U, V, W, P, Q, S)
    for p in range(P):
        c = replica_cols(P, Q, S, p)
        ref = np.zeros((Q, Q, Q))
        for a in range(Q):
            for b in range(Q):
                for cc in range(Q):
                    s = 0.0
                    for i in range(I):
                        for j in range(J):
                            for k in range(t):
                                s += X[k, i, j] * U[i, c[a]] * V[j, c[b]] * W[k, c[cc]]
                    ref[a, b, cc] = s
        assert np.max(np.abs(Z[p] - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_compress_of_cp_tensor_is_cp_of_compressed_factors(rng):
    """Sec. 4.2 (Kronecker/Khatri-Rao property): compressing [[A,B,C]] gives
    [[U^T A, V^T B, W^T C]]."""
    I, J, t, R, P, Q, S = 9, 7, 6, 3, 3, 4, 2
    A = rng.random((I, R)); B = rng.random((J, R)); C = rng.random((t, R))
    X = np.zeros((t, I, J))
    for r in range(R):
        X += C[:, r][:, None, None] * np.outer(A[:, r], B[:, r])[None]
    _, U, V, W = _rand_problem(rng, I, J, t, P, Q, S)
    Z = compress_dense(X, U, V, W, P, Q, S)
    for p in range(P):
        c = replica_cols(P, Q, S, p)
        a, b, cc = U[:, c].T @ A, V[:, c].T @ B, W[:, c].T @ C
        ref = np.zeros((Q, Q, Q))
        for r in range(R):
            ref += a[:, r][:, None, None] * b[:, r][None, :, None] * cc[:, r][None, None, :]
        assert np.linalg.norm(Z[p] - ref) <= 1e-12 * np.linalg.norm(ref)


def test_identity_compression_reduces_to_mode3_product(rng):
    """With one replica, Q = I = J and identity mode-1/2 matrices, the
    compression is the textbook mode-3 product X x3 W^T."""
    I = J = Q = 6
    t, P, S = 4, 1, 1
    X = rng.standard_normal((t, I, J))
    U = np.eye(I); V = np.eye(J)
    W = rng.standard_normal((t, Q))
    Z = compress_dense(X, U, V, W, P, Q, S)[0]
    ref = np.zeros((I, J, Q))
    for c in range(Q):
        for k in range(t):
            ref[:, :, c] += W[k, c] * X[k]
    assert np.max(np.abs(Z - ref)) <= 1e-13


def test_linearity_identity(rng):
    """Compressing the concatenated [X_old; X_new] with [W_old; W_new] equals
    Y + Z (Eq. 2 with fixed mode-1/2 matrices), to 1e-12 relative."""
    I, J, P, Q, S = 11, 13, 3, 5, 2
    X_old, U, V, W_old = _rand_problem(rng, I, J, 7, P, Q, S)
    X_new = rng.standard_normal((4, I, J))
    W_new = rng.standard_normal((4, W_old.shape[1]))
    Y = compress_dense(X_old, U, V, W_old, P, Q, S)
    Z = compress_dense(X_new, U, V, W_new, P, Q, S)
    full = compress_dense(np.concatenate([X_old, X_new]), U, V, np.vstack([W_old, W_new]), P, Q, S)
    upd = update_summaries(Y, Z)
    assert np.linalg.norm(upd - full) <= 1e-12 * np.linalg.norm(full)


def test_sparse_equals_dense_of_densified(rng):
    I, J, t, P, Q, S = 12, 10, 5, 2, 4, 1
    _, U, V, W = _rand_problem(rng, I, J, t, P, Q, S)
    nnz = 60
    k = rng.integers(0, t, nnz); i = rng.integers(0, I, nnz); j = rng.integers(0, J, nnz)
    v = rng.standard_normal(nnz)
    Xd = np.zeros((t, I, J))
    np.add.at(Xd, (k, i, j), v)      # duplicates add up
    Zs = compress_coo(k, i, j, v, t, U, V, W, P, Q, S)
    Zd = compress_dense(Xd, U, V, W, P, Q, S)
    assert np.linalg.norm(Zs - Zd) <= 1e-12 * np.linalg.norm(Zd)


def test_zero_batch_leaves_summary_unchanged(rng):
    I, J, t, P, Q, S = 6, 5, 3, 2, 3, 1
    X, U, V, W = _rand_problem(rng, I, J, t, P, Q, S)
    Y = compress_dense(X, U, V, W, P, Q, S)
    Z0 = compress_dense(np.zeros_like(X), U, V, W, P, Q, S)
    assert np.all(Z0 == 0)
    assert np.array_equal(update_summaries(Y, Z0), Y)


def _sorted_coo(rng, t, I, J, nnz, empty_slices=()):
    k = rng.integers(0, t, nnz); i = rng.integers(0, I, nnz); j = rng.integers(0, J, nnz)
    keep = ~np.isin(k, list(empty_slices))
    k, i, j = k[keep], i[keep], j[keep]
    order = np.lexsort((j, i, k))
    return k[order], i[order], j[order]


def test_coo_segments_against_loop(rng):
    # brute force: walk the nonzeros once, opening a segment at every change
    # of (k, i); slices 1 and 4 (and the last) have no nonzeros
    t = 7
    k, i, j = _sorted_coo(rng, t, 5, 6, 80, empty_slices=(1, 4, 6))
    seg_start, seg_row, slice_seg = coo_segments(k, i, t)
    starts, rows, first = [], [], {}
    for n in range(len(k)):
        if n == 0 or (k[n], i[n]) != (k[n - 1], i[n - 1]):
            first.setdefault(int(k[n]), len(starts))
            starts.append(n); rows.append(int(i[n]))
    assert seg_start.tolist() == starts + [len(k)]
    assert seg_row.tolist() == rows
    # slice_seg: a slice without nonzeros starts where the next one does
    expect = []
    for x in range(t + 1):
        later = [first[q] for q in first if q >= x]
        expect.append(min(later) if later else len(starts))
    assert slice_seg.tolist() == expect
    assert slice_seg[1] == slice_seg[2] and slice_seg[4] == slice_seg[5]
    assert slice_seg[6] == slice_seg[7] == len(starts)
    # each segment holds one (k, i), and neighbours differ
    for s in range(len(starts)):
        sl = slice(seg_start[s], seg_start[s + 1])
        assert len(set(zip(k[sl].tolist(), i[sl].tolist()))) == 1


def test_coo_segments_empty_batch():
    seg_start, seg_row, slice_seg = coo_segments(np.zeros(0, int), np.zeros(0, int), 3)
    assert seg_start.tolist() == [0] and seg_row.size == 0 and slice_seg.tolist() == [0] * 4


def test_coo_entries_match_full_compression(rng):
    I, J, t, P, Q, S = 9, 8, 6, 3, 4, 2
    _, U, V, W = _rand_problem(rng, I, J, t, P, Q, S)
    k, i, j = _sorted_coo(rng, t, I, J, 70)
    v = rng.standard_normal(k.size)
    Z = compress_coo(k, i, j, v, t, U, V, W, P, Q, S)
    picks = [(0, 0, 0), (1, 3, 2), (2, 1, 3), (2, 0, 1)]
    got = compress_coo_entries(k, i, j, v, t, U, V, W, P, Q, S, picks)
    for (p, a, b), row in zip(picks, got):
        assert np.allclose(row, Z[p, a, b, :], rtol=1e-13, atol=1e-13)


def test_sort_coo_against_python_sort(rng):
    # brute force: Python's stable sort on (k, i, j) tuples; duplicates keep
    # their input order (told apart by their values)
    n = 300
    k = rng.integers(0, 4, n); i = rng.integers(0, 5, n); j = rng.integers(0, 6, n)
    v = np.arange(n, dtype=np.float64)
    ks, is_, js, vs = sort_coo(k, i, j, v)
    want = sorted(range(n), key=lambda e: (k[e], i[e], j[e]))
    assert vs.tolist() == [float(e) for e in want]
    assert ks.tolist() == [int(k[e]) for e in want]
    assert is_.tolist() == [int(i[e]) for e in want] and js.tolist() == [int(j[e]) for e in want]
    # compression does not depend on the order of the nonzeros
    P, Q, S, I, J, t = 2, 4, 1, 5, 6, 4
    M1 = S + P * (Q - S)
    U = rng.standard_normal((I, M1)); V = rng.standard_normal((J, M1)); W = rng.standard_normal((t, M1))
    vv = rng.standard_normal(n)
    a = compress_coo(k, i, j, vv, t, U, V, W, P, Q, S)
    b = compress_coo(*sort_coo(k, i, j, vv), t, U, V, W, P, Q, S)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
