"""FP64 oracle of the N-mode extension (supplement, "Extending to
Higher-Order Tensors"): an N-mode tensor growing in its last (temporal)
mode, with N - 1 fixed compression matrices for the non-temporal modes and
fresh temporal rows per batch.  TEST INFRASTRUCTURE ONLY: imported by tests,
the smoke check and the benchmark's CPU-baseline leg, never by the product
path; it shares no code with the HIP implementation.

Every step is the three-mode oracle's step written for N modes (the three-
mode oracle is this one at N = 3, which a test checks):
  compression   Z_p = X x_1 U1_p^T ... x_{N-1} U(N-1)_p^T x_N W_p^T
  update        Y_p += Z_p
  replica CP    Gauss-Seidel ALS over the N modes (reading R-ALS)
  matching      lambda^(1/N) on each mode, similarity = product over the N
                modes of |cos| between anchor columns, exclusive greedy
                assignment, per-mode least-squares scale (reading R-MATCH)
  recovery      per non-temporal mode the weighted minimum-norm solve of the
                deduplicated stack (R-STACK, R-PINV); canonical columns of
                the N - 1 non-temporal factors; temporal rows by the
                incremental solve with the carried history removed (R-C1,
                the products of the N - 1 modes' scales and |cos| in place of
                the two of three modes)
  fit           1 - ||X - [[A1, ..., A(N-1), C]]|| / ||X|| (reading R-FIT)

Layouts: a batch X is (t, I_1, ..., I_{N-1}) (time first, like the three-mode
oracle's (t, I, J)); a replica summary is (Q,) * N with the temporal index
last; replica factors are (P, N, Q, R), mode N - 1 temporal."""
from __future__ import annotations

import math

import numpy as np

from .octen_oracle import (gram_hadamard, greedy_assign, replica_cols, solve_normal, stack_rhs,
                           weighted_minnorm_lstsq)

__all__ = ["compress_dense_n", "mttkrp_n", "cp_als_n", "match_replicas_n", "canonicalize_n",
           "match_previous_n", "fit_dense_n", "OctenNOracle"]


def compress_dense_n(X, Us, W, P, Q, S):
    """Z_p for every replica (supplement, compressed cubes of an N-mode
    tensor): the non-temporal modes contracted with each replica's columns of
    their compression matrices, then the temporal mode with W_p."""
    X = np.asarray(X, np.float64)
    N = X.ndim
    assert len(Us) == N - 1
    Z = np.empty((P,) + (Q,) * N)
    for p in range(P):
        c = replica_cols(P, Q, S, p)
        T = X
        # contract mode n (axis 1 of the remaining non-temporal axes first):
        # after k steps T is (t, Q, ..., Q, I_{k+1}, ..., I_{N-1})
        for n in range(N - 1):
            T = np.tensordot(T, Us[n][:, c], axes=([1 + n], [0]))   # new axis appended last
            T = np.moveaxis(T, -1, 1 + n)
        # temporal: Z[q_1..q_{N-1}, c] = sum_k T[k, q...] W_p(k, c)
        Z[p] = np.tensordot(T, W[:, c], axes=([0], [0]))
    return Z


def mttkrp_n(Y, F, n):
    """Mode-n unfolding of Y times the Khatri-Rao product of the other
    factors (Sec. 2): M(q, r) = sum over the other indices of Y * prod_m
    F_m(idx_m, r)."""
    N = Y.ndim
    letters = "abcdefgh"[:N]
    ins = [letters] + [letters[m] + "r" for m in range(N) if m != n]
    ops = [Y] + [F[m] for m in range(N) if m != n]
    return np.einsum(",".join(ins) + "->" + letters[n] + "r", *ops)


def cp_als_n(Y, init, iters):
    """Rank-R CP of one N-mode replica by alternating least squares (reading
    R-ALS at N modes): Gauss-Seidel over the modes, F_n = M_n G_n^{-1} with
    G_n the Hadamard product of the other Grams, unit columns after every
    mode update, lambda = norms of the last mode.
    Returns (F list, lam, fallback flag)."""
    F = [np.array(f, dtype=np.float64) for f in init]
    N = len(F)
    R = F[0].shape[1]
    lam = np.ones(R)
    flag = False
    for _ in range(iters):
        for n in range(N):
            M = mttkrp_n(Y, F, n)
            G = np.ones((R, R))
            for m in range(N):
                if m != n:
                    G = G * (F[m].T @ F[m])
            Fn, fb = solve_normal(M, G)
            flag |= fb
            nrm = np.linalg.norm(Fn, axis=0)
            nrm = np.where(nrm > 0, nrm, 1.0)
            F[n] = Fn / nrm
            lam = nrm
    return F, lam, flag


def _abs_cos(a, b):
    na = np.linalg.norm(a, axis=0)
    nb = np.linalg.norm(b, axis=0)
    den = np.outer(na, nb)
    num = np.abs(a.T @ b)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def match_replicas_n(Fs, S):
    """Matching of Sec. 4.2 over N modes (reading R-MATCH): replica 0 is the
    reference; similarity = product over the N modes of |cos| between the
    first S rows (anchors); exclusive greedy pairing; per-mode least-squares
    scale of each anchor column onto the reference's.
    Fs: (P, N, Q, R) after lambda distribution.  Returns (aligned, perm,
    margins)."""
    Fs = np.asarray(Fs, np.float64)
    P, N, Q, R = Fs.shape
    aligned = np.zeros_like(Fs)
    perm = np.zeros((P, R), dtype=np.int64)
    margins = np.full(P, np.inf)
    aligned[0] = Fs[0]
    perm[0] = np.arange(R)
    for p in range(1, P):
        sim = np.ones((R, R))
        for n in range(N):
            sim = sim * _abs_cos(Fs[p, n, :S, :], Fs[0, n, :S, :])
        pr, margins[p] = greedy_assign(sim)
        perm[p] = pr
        for n in range(N):
            a = Fs[p, n, :S, :]
            b = Fs[0, n, :S, :]
            for r in range(R):
                rr = pr[r]
                den = float(a[:, r] @ a[:, r])
                d = float(b[:, rr] @ a[:, r]) / den if den > 0 else 0.0
                aligned[p, n, :, rr] = d * Fs[p, n, :, r]
    return aligned, perm, margins


def canonicalize_n(Fs):
    """Reading R-C1 step 1 for the N - 1 non-temporal factors: unit columns,
    largest-magnitude entry positive (lowest index on a tie).  Returns
    (canonical list, kappa = product over the modes of norm * sign)."""
    out, kappa = [], None
    for M in Fs:
        n = np.linalg.norm(M, axis=0)
        idx = np.argmax(np.abs(M), axis=0)
        s = np.sign(M[idx, np.arange(M.shape[1])])
        s = np.where(s == 0, 1.0, s)
        n = np.where(n > 0, n, 1.0)
        out.append(M / (n * s))
        kappa = n * s if kappa is None else kappa * n * s
    return out, kappa


def match_previous_n(cur, prev):
    """Reading R-C1 step 2 over the N - 1 non-temporal modes: exclusive
    greedy pairing on the product of |cos| with the previous batch's
    canonical factors; sign = product of the cosines' signs."""
    R = cur[0].shape[1]
    sim = np.ones((R, R))
    crosses = []
    for a, b in zip(cur, prev):
        c = a.T @ b
        nn = np.outer(np.linalg.norm(a, axis=0), np.linalg.norm(b, axis=0))
        sim = sim * np.abs(c) / np.where(nn > 0, nn, 1.0)
        crosses.append(c)
    perm, margin = greedy_assign(sim)
    signs = np.ones(R)
    for c in crosses:
        signs = signs * np.array([np.sign(c[r, perm[r]]) for r in range(R)])
    signs = np.where(signs == 0, 1.0, signs)
    return perm, signs, margin


def fit_dense_n(X, As, C, k0=0):
    """Sec. 5.1 fitness (reading R-FIT) of [[A_1, ..., A_{N-1}, C]] on the
    slices X[k] (global index k0 + k).  Returns (fit, sse, norm2)."""
    X = np.asarray(X, np.float64)
    N = X.ndim
    letters = "abcdefg"[:N - 1]
    sse = nx = 0.0
    for k in range(X.shape[0]):
        Xh = np.einsum(",".join(l + "r" for l in letters) + ",r->" + letters,
                       *As, C[k0 + k])
        d = X[k] - Xh
        sse += float(np.sum(d * d))
        nx += float(np.sum(X[k] * X[k]))
    return (1.0 - math.sqrt(sse) / math.sqrt(nx) if nx > 0 else 0.0), sse, nx


class OctenNOracle:
    """Algorithm 1 for an N-mode tensor growing in its last mode (the
    supplement's higher-order version), one method per step; the state is the
    three-mode oracle's with N - 1 non-temporal factors."""

    def __init__(self, dims, R, P, Q, S, Us):
        self.dims = tuple(int(d) for d in dims)     # I_1 .. I_{N-1}
        self.N = len(self.dims) + 1
        self.R, self.P, self.Q, self.S = R, P, Q, S
        self.M1 = S + P * (Q - S)
        self.Us = [np.asarray(u, np.float64) for u in Us]
        assert all(u.shape == (d, self.M1) for u, d in zip(self.Us, self.dims))
        self.Y = np.zeros((P,) + (Q,) * self.N)
        self.Z = self.W = None
        self.t = self.K = 0
        self.F = self.lam = None
        self.prev = None
        self.C = np.zeros((0, R))
        self.H = np.zeros((self.M1, R))
        self.last = {}

    def compress_batch(self, X, W):
        X = np.asarray(X, np.float64)
        assert X.shape[1:] == self.dims
        self.t = X.shape[0]
        self.W = np.asarray(W, np.float64)
        self.Z = compress_dense_n(X, self.Us, self.W, self.P, self.Q, self.S)
        return self.Z

    def update_replicas(self):
        self.Y = self.Y + self.Z
        self.K += self.t
        return self.Y

    def cp_als_replicas(self, iters, init=None):
        if init is None:
            init = self.F
        init = np.asarray(init, np.float64)
        F = np.zeros((self.P, self.N, self.Q, self.R))
        lam = np.zeros((self.P, self.R))
        for p in range(self.P):
            Fp, lp, _ = cp_als_n(self.Y[p], list(init[p]), iters)
            F[p] = np.stack(Fp)
            lam[p] = lp
        self.F, self.lam = F, lam
        return F, lam

    def recover_factors(self):
        P, Q, S, R, N = self.P, self.Q, self.S, self.R, self.N
        root = np.power(self.lam, 1.0 / N)                      # lambda^(1/N), lambda > 0
        Fd = self.F * root[:, None, None, :]
        aligned, perm, margins = match_replicas_n(Fd, S)
        rhs = [stack_rhs(aligned[:, n], S) for n in range(N)]
        raw = [weighted_minnorm_lstsq(self.Us[n], rhs[n], P, S) for n in range(N - 1)]
        cur, kappa = canonicalize_n(raw)
        if self.prev is None:
            tperm, tsign, tmargin = np.arange(R), np.ones(R), np.inf
        else:
            tperm, tsign, tmargin = match_previous_n(cur, self.prev)
        Hcur = self.H[:, tperm] * tsign
        Cold = self.C[:, tperm] * tsign
        Cnew = weighted_minnorm_lstsq(self.W, rhs[N - 1] - Hcur / kappa, P, S) * kappa
        self.C = np.vstack([Cold, Cnew])
        self.H = Hcur + self.W.T @ Cnew
        self.prev = cur
        self.last = dict(aligned=aligned, perm=perm, margins=margins, rhs=rhs, tperm=tperm,
                         tsign=tsign, kappa=kappa)
        return cur, self.C
