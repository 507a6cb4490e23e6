"""Plain, slow, FP64 CPU oracle of the online compressed CP decomposition.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.  It shares no code
with the HIP implementation.

Every function states the passage of the paper it follows.  The paper is
"OCTen: Online Compression-based Tensor Decomposition" (Gujral, Pasricha,
Yang, Papalexakis).  Section numbers: 4.1 "Parallel Compression and
Decomposition", 4.2 "Factor match for identifiability", 4.3 "Update results",
5.1 "Evaluation Measures", 5.4.3 "[Q4] Parameter Sensitivity", Algorithm 1
(supplement).  Equations: Eq. 1 compression triplets with shared columns,
Eq. 2 summary update, Eq. 3/4 uniqueness conditions, Eq. 5 stacked matched
factors, Eq. 6 stacked compression matrices, Eq. 7 the least-squares update,
Eq. 8 the lower bound on p.

Where the paper is silent or ambiguous the reading used is named in the
docstring (R-* tags); all of them are listed with their justification in the
design notes of the repository.

Layouts (shared with the HIP side only through the argument conventions):
  X      [t][I][J]   frontal slices, j fastest
  U      [I][M1]     deduplicated mode-1 compression matrix [G | H_1 .. H_P]
  V      [J][M1]     same for mode 2
  W      [t][M1]     the batch's mode-3 compression rows
  Y, Z   [P][Q][Q][Q]
  F      [P][3][Q][R] replica factors
M1 = S + P*(Q-S); replica p uses columns [0..S) and [S+p(Q-S) .. S+(p+1)(Q-S)).

Parity status: compression, update, MTTKRP/ALS steps, the deduplicated
least-squares recovery, the fit and the identifiability bound are pinned by
brute force, closed forms, invariants and library routines (see tests).
The readings R-ALS (iteration/normalisation details), R-MATCH (exclusive
greedy assignment) and R-C1 (temporal carry) have no worked example in the
paper: parity unpinned against the paper's own numbers; pinned only by
planted and exact-data cases.
"""
from __future__ import annotations

import math
import numpy as np

__all__ = [
    "replica_cols", "compress_dense", "compress_coo", "coo_segments", "sort_coo",
    "compress_coo_entries", "update_summaries",
    "mttkrp", "gram_hadamard", "solve_normal", "cp_als", "replica_fit",
    "distribute_lambda", "greedy_assign", "match_replicas", "stack_rhs",
    "weighted_minnorm_lstsq", "canonicalize", "match_previous",
    "fit_dense", "fit_coo_identity", "identifiability", "p_min_bound",
    "OctenOracle",
]


# ---------------------------------------------------------------------------
# Compression (Sec. 4.1, Eq. 1; Algorithm 1 first step)
# ---------------------------------------------------------------------------

def replica_cols(P: int, Q: int, S: int, p: int) -> np.ndarray:
    """Columns of replica p in the deduplicated compression matrices.  Eq. 1:
    every triplet starts with the shared columns (u, v, w), followed by the
    replica's own columns.  Reading R-SHARED: exactly S shared columns, first."""
    return np.r_[np.arange(S), S + p * (Q - S) + np.arange(Q - S)]


def compress_dense(X, U, V, W, P, Q, S):
    """Z_p = X x1 U_p^T x2 V_p^T x3 W_p^T for every replica p (Sec. 4.1).

    The paper compresses the first mode first, then the second, then the third
    (Sec. 4.1, complexity paragraph); each mode product is one tensordot."""
    X = np.asarray(X, dtype=np.float64)
    t, I, J = X.shape
    Z = np.empty((P, Q, Q, Q))
    for p in range(P):
        c = replica_cols(P, Q, S, p)
        Up, Vp, Wp = U[:, c], V[:, c], W[:, c]
        # mode 1: T1[a, k, j] = sum_i U_p(i, a) X(k, i, j)
        T1 = np.tensordot(Up, X, axes=([0], [1]))            # (Q, t, J)
        # mode 2: T2[a, k, b] = sum_j T1[a, k, j] V_p(j, b)
        T2 = np.tensordot(T1, Vp, axes=([2], [0]))           # (Q, t, Q)
        # mode 3: Z[a, b, c] = sum_k T2[a, k, b] W_p(k, c)
        Z[p] = np.tensordot(T2, Wp, axes=([1], [0]))         # (Q, Q, Q)
    return Z


def compress_coo(k, i, j, v, t, U, V, W, P, Q, S):
    """Same Z_p as `compress_dense` for a tensor given by its nonzeros
    (Sec. 4.1: the summaries of a sparse tensor are dense).  Duplicate
    coordinates add up.  For each slice, the mode-1 product is the sum over
    nonzeros of v * U_p(i, :) placed at column j, then modes 2 and 3 follow."""
    k = np.asarray(k, np.int64); i = np.asarray(i, np.int64); j = np.asarray(j, np.int64)
    v = np.asarray(v, np.float64)
    Z = np.zeros((P, Q, Q, Q))
    for p in range(P):
        c = replica_cols(P, Q, S, p)
        Up, Vp, Wp = U[:, c], V[:, c], W[:, c]
        # mode 2 on the nonzeros: contribution to M_k(a, b) = sum v U(i,a) V(j,b)
        M = np.zeros((t, Q, Q))
        for kk in range(t):
            sel = k == kk
            if not np.any(sel):
                continue
            M[kk] = (Up[i[sel]] * v[sel, None]).T @ Vp[j[sel]]
        Z[p] = np.tensordot(M, Wp, axes=([0], [0]))
    return Z


def sort_coo(k, i, j, v):
    """A COO batch in (k, i, j) order (the sparse input of Sec. 4.1, whose
    segments are runs of equal (k, i)); equal coordinates keep their input
    order (a stable sort, numpy's lexsort)."""
    k = np.asarray(k); i = np.asarray(i); j = np.asarray(j); v = np.asarray(v)
    order = np.lexsort((j, i, k))
    return k[order], i[order], j[order], v[order]


def coo_segments(k, i, t):
    """Bookkeeping of a COO batch sorted by (k, i, j) (Sec. 4.1 sparse input).
    A segment is a maximal run of nonzeros sharing (k, i), numbered in input
    order.  Returns int64 arrays seg_start [nseg + 1] (first nonzero of each
    segment, then nnz), seg_row [nseg] (its i) and slice_seg [t + 1] (number
    of segments of slices before x, for x = 0..t)."""
    k = np.asarray(k, np.int64); i = np.asarray(i, np.int64)
    nnz = k.size
    head = np.ones(nnz, bool)
    if nnz > 1:
        head[1:] = (k[1:] != k[:-1]) | (i[1:] != i[:-1])
    starts = np.flatnonzero(head)
    seg_start = np.append(starts, nnz).astype(np.int64)
    seg_row = i[starts]
    seg_slice = k[starts]
    slice_seg = np.array([np.count_nonzero(seg_slice < x) for x in range(t + 1)], np.int64)
    return seg_start, seg_row, slice_seg


def compress_coo_entries(k, i, j, v, t, U, V, W, P, Q, S, picks):
    """Selected fibres of the compressed batch, one at a time: for each
    (p, a, b) in picks, Z_p[a, b, :] = sum_k m_k W_p(k, :) with
    m_k = sum over the nonzeros of slice k of v U_p(i, a) V_p(j, b)
    (Eq. 1 written entrywise for one mode-1 and one mode-2 index)."""
    k = np.asarray(k, np.int64); i = np.asarray(i, np.int64); j = np.asarray(j, np.int64)
    v = np.asarray(v, np.float64)
    out = []
    for p, a, b in picks:
        c = replica_cols(P, Q, S, p)
        m = np.zeros(t)
        np.add.at(m, k, v * U[i, c[a]] * V[j, c[b]])
        out.append(m @ W[:, c])
    return np.array(out)


def update_summaries(Y, Z):
    """Eq. 2 / Algorithm 1 second step: X_p = Y_p (+) Z_p.  Reading R-UPD: the
    element-wise "W'(k, q)" factor in Eq. 2 is the mode-3 weighting already
    applied inside the compression, so the update is a plain sum."""
    return Y + Z


# ---------------------------------------------------------------------------
# Per-replica CP decomposition (Sec. 4.1 last paragraph; Sec. 2 CP model)
# ---------------------------------------------------------------------------

def mttkrp(X, F, n):
    """Mode-n unfolding times the Khatri-Rao product of the other factors
    (Sec. 2, the unfolded CP model): M_n(q, r) = sum over the other two
    indices of X * F_m(., r) * F_l(., r)."""
    if n == 0:
        return np.einsum("abc,br,cr->ar", X, F[1], F[2])
    if n == 1:
        return np.einsum("abc,ar,cr->br", X, F[0], F[2])
    return np.einsum("abc,ar,br->cr", X, F[0], F[1])


def gram_hadamard(F, n):
    """Element-wise product of the Gram matrices F_m^T F_m of the other modes:
    the normal matrix of the mode-n least-squares problem."""
    R = F[0].shape[1]
    G = np.ones((R, R))
    for m in range(3):
        if m != n:
            G = G * (F[m].T @ F[m])
    return G


def solve_normal(M, G):
    """F = M G^{-1} for symmetric positive definite G (Cholesky); reading
    R-ALS: if G is not positive definite, a pseudo-inverse with cut-off
    1e-12 * largest eigenvalue is used instead."""
    try:
        L = np.linalg.cholesky(G)
        Y = np.linalg.solve(L, M.T)
        return np.linalg.solve(L.T, Y).T, False
    except np.linalg.LinAlgError:
        w, Qv = np.linalg.eigh(G)
        cut = 1e-12 * max(w.max(), 0.0)
        winv = np.where(w > cut, 1.0 / np.where(w > cut, w, 1.0), 0.0)
        return M @ (Qv * winv) @ Qv.T, True


def replica_fit(X, F, lam, M3):
    """Fit of the replica model [[lam; F1, F2, F3]] from Gram identities:
    ||X - Xh||^2 = ||X||^2 - 2 <X, Xh> + ||Xh||^2 with <X, Xh> computed from
    the last MTTKRP (mode 3).  Returns 1 - ||X - Xh|| / ||X||."""
    nx2 = float(np.sum(X * X))
    inner = float(np.sum(lam * np.sum(M3 * F[2], axis=0)))
    G = (F[0].T @ F[0]) * (F[1].T @ F[1]) * (F[2].T @ F[2])
    nh2 = float(lam @ G @ lam)
    res2 = max(nx2 - 2 * inner + nh2, 0.0)
    return 1.0 - math.sqrt(res2) / math.sqrt(nx2) if nx2 > 0 else 0.0


def cp_als(X, init, iters, tol=0.0):
    """Rank-R CP of one replica by alternating least squares (Sec. 4.1:
    each worker decomposes its replica; Algorithm 1 third step).

    Reading R-ALS: Gauss-Seidel over modes 1, 2, 3; each mode solves
    F_n = M_n G_n^{-1}; after every mode update the columns are scaled to unit
    2-norm and lambda holds the norms of the last updated mode.  With tol = 0
    exactly `iters` sweeps run; with tol > 0 the loop stops after the first
    sweep whose replica-fit change is below tol.
    Returns (F list of 3 (Q x R) arrays, lam (R,), sweeps done, fallback flag)."""
    F = [np.array(init[0], dtype=np.float64), np.array(init[1], dtype=np.float64),
         np.array(init[2], dtype=np.float64)]
    R = F[0].shape[1]
    lam = np.ones(R)
    done, fit_old, flag = 0, None, False
    for _ in range(iters):
        M = None
        for n in range(3):
            M = mttkrp(X, F, n)
            G = gram_hadamard(F, n)
            Fn, fb = solve_normal(M, G)
            flag |= fb
            nrm = np.linalg.norm(Fn, axis=0)
            nrm = np.where(nrm > 0, nrm, 1.0)
            F[n] = Fn / nrm
            lam = nrm
        done += 1
        if tol > 0:
            fit = replica_fit(X, F, lam, M)
            if fit_old is not None and abs(fit - fit_old) < tol:
                break
            fit_old = fit
    return F, lam, done, flag


# ---------------------------------------------------------------------------
# Factor match (Sec. 4.2, Eq. 5; Algorithm 1 matching loop)
# ---------------------------------------------------------------------------

def distribute_lambda(F, lam):
    """Eq. 5 and the text before it: each replica factor carries lambda^(1/N),
    here N = 3, so that [[F1, F2, F3]] reproduces the replica model."""
    s = np.cbrt(lam)
    return [f * s for f in F]


def greedy_assign(sim):
    """Reading R-MATCH: exclusive greedy assignment on a similarity matrix
    sim[r, r'] (row r of the replica, column r' of the reference).  Repeatedly
    take the largest entry among unassigned rows and columns; scanning r'
    ascending then r ascending and keeping only strictly larger values breaks
    ties towards the smallest r', then the smallest r.
    Returns (perm with perm[r] = r', margin).  The margin is the smallest gap,
    over the selection rounds, between the chosen entry and the best other
    free entry in its row or its column (its competitors); a margin of zero
    means the choice was decided by the tie-break."""
    R = sim.shape[0]
    perm = -np.ones(R, dtype=np.int64)
    row_free = np.ones(R, bool)
    col_free = np.ones(R, bool)
    margin = np.inf
    for _ in range(R):
        best, br, bc = -np.inf, -1, -1
        for c in range(R):
            if not col_free[c]:
                continue
            for r in range(R):
                if not row_free[r]:
                    continue
                if sim[r, c] > best:
                    best, br, bc = sim[r, c], r, c
        rival = -np.inf
        for c in range(R):
            if col_free[c] and c != bc:
                rival = max(rival, sim[br, c])
        for r in range(R):
            if row_free[r] and r != br:
                rival = max(rival, sim[r, bc])
        if np.isfinite(rival):
            margin = min(margin, best - rival)
        perm[br] = bc
        row_free[br] = False
        col_free[bc] = False
    return perm, margin


def _abs_cos(a, b):
    """|cos| between the columns of a (S x R) and b (S x R): out[r, r']."""
    na = np.linalg.norm(a, axis=0)
    nb = np.linalg.norm(b, axis=0)
    den = np.outer(na, nb)
    num = np.abs(a.T @ b)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def match_replicas(Fs, S):
    """Sec. 4.2 and Algorithm 1: align every replica's factors to one reference
    through the shared anchor rows.

    Fs: (P, 3, Q, R) replica factors after lambda distribution.  The anchor
    block of replica p, mode n is its first S rows (they come from the shared
    compression columns).  Reading R-MATCH: the reference is replica 0 (the
    single reference of Fig. 1); the similarity is the product over modes of
    |cos| between anchor columns (any per-column normalisation, l1, l2 or max,
    drops out of |cos|); columns are paired by exclusive greedy assignment; the
    scale (sign included) of each mode is the least-squares fit of the anchor
    column onto the reference's.
    Returns (aligned (P, 3, Q, R), perm (P, R), scale (P, 3, R), margins (P,))."""
    Fs = np.asarray(Fs, dtype=np.float64)
    P, _, Q, R = Fs.shape
    aligned = np.zeros_like(Fs)
    perm = np.zeros((P, R), dtype=np.int64)
    scale = np.ones((P, 3, R))
    margins = np.full(P, np.inf)
    aligned[0] = Fs[0]
    perm[0] = np.arange(R)
    for p in range(1, P):
        sim = np.ones((R, R))
        for n in range(3):
            sim = sim * _abs_cos(Fs[p, n, :S, :], Fs[0, n, :S, :])
        pr, margins[p] = greedy_assign(sim)
        perm[p] = pr
        for n in range(3):
            a = Fs[p, n, :S, :]
            b = Fs[0, n, :S, :]
            for r in range(R):
                rr = pr[r]
                den = float(a[:, r] @ a[:, r])
                d = float(b[:, rr] @ a[:, r]) / den if den > 0 else 0.0
                scale[p, n, r] = d
                aligned[p, n, :, rr] = d * Fs[p, n, :, r]
    return aligned, perm, scale, margins


# ---------------------------------------------------------------------------
# Stacking and least-squares recovery (Sec. 4.3, Eq. 6 and Eq. 7)
# ---------------------------------------------------------------------------

def stack_rhs(aligned_mode, S):
    """Deduplicated right-hand side for one mode (Eq. 5 stack with the shared
    rows merged): [mean over p of the anchor rows; replica 0 private rows; ...;
    replica P-1 private rows] -> (M1 x R).  Together with the sqrt(P) row
    weights of `weighted_minnorm_lstsq` this has the same least-squares
    solutions as the literal stack of Eq. 5/6 (the anchor equations repeat P
    times there)."""
    A = np.asarray(aligned_mode, dtype=np.float64)   # (P, Q, R)
    return np.vstack([A[:, :S, :].mean(axis=0)] + [A[p, S:, :] for p in range(A.shape[0])])


def weighted_minnorm_lstsq(Pt, rhs, P, S):
    """Eq. 7 with the inverse read as the Moore-Penrose pseudo-inverse (reading
    R-PINV): the minimum-norm minimiser of || w * (Pt^T x - rhs) || where Pt is
    the deduplicated compression matrix (n x M1, the caller's layout, so the
    stacked system matrix of Eq. 6 is Pt^T) and w = sqrt(P) on the S shared
    rows, 1 elsewhere.  Solved by numpy.linalg.lstsq (SVD based)."""
    Pt = np.asarray(Pt, dtype=np.float64)
    M1 = Pt.shape[1]
    w = np.ones(M1)
    w[:S] = math.sqrt(P)
    x, *_ = np.linalg.lstsq(w[:, None] * Pt.T, w[:, None] * rhs, rcond=None)
    return x


def canonicalize(A, B):
    """Reading R-C1, step 1: scale the columns of A and B to unit 2-norm and
    make the entry of largest magnitude of each column positive (the lowest
    index wins a tie).  Returns (Ac, Bc, kappa) with A = Ac * na * sa and
    kappa = na * sa * nb * sb, so that [[A, B, C]] = [[Ac, Bc, C * kappa]]."""
    def one(M):
        n = np.linalg.norm(M, axis=0)
        idx = np.argmax(np.abs(M), axis=0)
        s = np.sign(M[idx, np.arange(M.shape[1])])
        s = np.where(s == 0, 1.0, s)
        n = np.where(n > 0, n, 1.0)
        return M / (n * s), n * s
    Ac, ka = one(A)
    Bc, kb = one(B)
    return Ac, Bc, ka * kb


def match_previous(Ac, Bc, Ap, Bp):
    """Reading R-C1, step 2: pair the current canonical columns with the
    previous batch's by exclusive greedy assignment on |cos_A| * |cos_B| and
    record the sign s_r = sign(cos_A) * sign(cos_B) of each pair.
    Returns (perm, signs, margin) with perm[r] = previous column of r."""
    ca = Ac.T @ Ap
    cb = Bc.T @ Bp
    na = np.outer(np.linalg.norm(Ac, axis=0), np.linalg.norm(Ap, axis=0))
    nb = np.outer(np.linalg.norm(Bc, axis=0), np.linalg.norm(Bp, axis=0))
    sim = np.abs(ca) / np.where(na > 0, na, 1.0) * np.abs(cb) / np.where(nb > 0, nb, 1.0)
    perm, margin = greedy_assign(sim)
    R = Ac.shape[1]
    signs = np.array([np.sign(ca[r, perm[r]]) * np.sign(cb[r, perm[r]]) for r in range(R)])
    signs = np.where(signs == 0, 1.0, signs)
    return perm, signs, margin


# ---------------------------------------------------------------------------
# Fit (Sec. 5.1) and identifiability (Eq. 3, Eq. 4, Eq. 8)
# ---------------------------------------------------------------------------

def fit_dense(X, A, B, C, k0=0):
    """Sec. 5.1 fitness as a fraction: 1 - ||X - [[A,B,C]]||_F / ||X||_F over
    the given slices X[k] (global slice index k0 + k).
    Returns (fit, sse, norm2)."""
    X = np.asarray(X, dtype=np.float64)
    sse = 0.0
    nx = 0.0
    for k in range(X.shape[0]):
        Xh = (A * C[k0 + k]) @ B.T
        d = X[k] - Xh
        sse += float(np.sum(d * d))
        nx += float(np.sum(X[k] * X[k]))
    fit = 1.0 - math.sqrt(sse) / math.sqrt(nx) if nx > 0 else 0.0
    return fit, sse, nx


def fit_coo_identity(k, i, j, v, A, B, C):
    """Sec. 5.1 fitness for a sparse tensor through
    ||X - Xh||^2 = ||X||^2 - 2 <X, Xh> + 1^T (A^T A * B^T B * C^T C) 1,
    where C holds every slice the nonzeros index.  Returns (fit, sse, norm2)."""
    v = np.asarray(v, np.float64)
    nx = float(v @ v)
    xh = np.einsum("nr,nr,nr->n", A[np.asarray(i)], B[np.asarray(j)], C[np.asarray(k)])
    inner = float(v @ xh)
    G = (A.T @ A) * (B.T @ B) * (C.T @ C)
    nh = float(G.sum())
    sse = max(nx - 2 * inner + nh, 0.0)
    fit = 1.0 - math.sqrt(sse) / math.sqrt(nx) if nx > 0 else 0.0
    return fit, sse, nx


def p_min_bound(I, J, K, Q, shared):
    """Eq. 8 as printed: p >= max((I - shared)/(Q - shared), J/Q, K/Q)."""
    return max((I - shared) / (Q - shared), J / Q, K / Q)


def identifiability(I, J, K, t, R, P, Q, S):
    """Verdicts on the conditions of Sec. 4.2 and Sec. 5.4.3 (all host side).

    bit 0: Eq. 8 holds (P >= ceil of the printed bound)
    bit 1: M1 >= I  (mode-1 least squares determined)
    bit 2: M1 >= J  (mode-2 determined)
    bit 3: M1 >= t  (temporal rows of the batch determined)
    bit 4: Eq. 4 with generic Kruskal ranks min(dim, R):
           sum_n min(Q, k_n) >= 2R + 2
    Returns (bits, p_min)."""
    M1 = S + P * (Q - S)
    pmin = p_min_bound(I, J, K, Q, S)
    bits = 0
    if P >= math.ceil(pmin - 1e-12):
        bits |= 1
    if M1 >= I:
        bits |= 2
    if M1 >= J:
        bits |= 4
    if M1 >= t:
        bits |= 8
    kr = min(Q, min(I, R)) + min(Q, min(J, R)) + min(Q, min(K, R))
    if kr >= 2 * R + 2:
        bits |= 16
    return bits, pmin


# ---------------------------------------------------------------------------
# The whole update, one call per step (Algorithm 1)
# ---------------------------------------------------------------------------

class OctenOracle:
    """Algorithm 1 for a 3-mode tensor growing in mode 3, one method per step.

    State kept between batches, as in Sec. 4.1 (only the summaries, the
    compression matrices and the previous factors are stored): Y, the replica
    factors, the canonical A and B of the previous batch, C, and the temporal
    carry H = W_old^T C_old in deduplicated layout (M1 x R, reading R-C1).
    temporal = "incremental" (R-C1, default) or "full" (R-C2: all K rows of C
    re-solved each batch from the whole W history)."""

    def __init__(self, I, J, R, P, Q, S, U, V, temporal="incremental"):
        self.I, self.J, self.R, self.P, self.Q, self.S = I, J, R, P, Q, S
        self.M1 = S + P * (Q - S)
        self.U = np.asarray(U, np.float64)
        self.V = np.asarray(V, np.float64)
        assert self.U.shape == (I, self.M1) and self.V.shape == (J, self.M1)
        self.Y = np.zeros((P, Q, Q, Q))
        self.Z = None
        self.W = None
        self.W_hist = []
        self.t = 0
        self.K = 0
        self.F = None            # (P, 3, Q, R) replica factors, unit columns
        self.lam = None          # (P, R)
        self.iters_done = None
        self.A = self.B = None   # canonical factors of the last recovery
        self.C = np.zeros((0, R))
        self.H = np.zeros((self.M1, R))
        self.temporal = temporal
        self.last = {}

    # Algorithm 1, first step
    def compress_batch(self, X, W):
        X = np.asarray(X, np.float64)
        self.t = X.shape[0]
        self.W = np.asarray(W, np.float64)
        assert self.W.shape == (self.t, self.M1)
        self.Z = compress_dense(X, self.U, self.V, self.W, self.P, self.Q, self.S)
        return self.Z

    def compress_batch_coo(self, k, i, j, v, t, W):
        self.t = int(t)
        self.W = np.asarray(W, np.float64)
        self.Z = compress_coo(k, i, j, v, t, self.U, self.V, self.W, self.P, self.Q, self.S)
        return self.Z

    # Algorithm 1, second step
    def update_replicas(self):
        self.Y = update_summaries(self.Y, self.Z)
        self.W_hist.append(self.W)
        self.K += self.t
        return self.Y

    # Algorithm 1, third step
    def cp_als_replicas(self, iters, tol=0.0, init=None):
        if init is None:
            assert self.F is not None, "first batch needs an explicit init"
            init = self.F
        init = np.asarray(init, np.float64)
        F = np.zeros((self.P, 3, self.Q, self.R))
        lam = np.zeros((self.P, self.R))
        done = np.zeros(self.P, np.int64)
        for p in range(self.P):
            Fp, lp, d, _ = cp_als(self.Y[p], init[p], iters, tol)
            F[p] = np.stack(Fp)
            lam[p] = lp
            done[p] = d
        self.F, self.lam, self.iters_done = F, lam, done
        return F, lam, done

    # Algorithm 1, matching loop and final solve
    def recover_factors(self):
        P, Q, S, R = self.P, self.Q, self.S, self.R
        Fd = np.stack([np.stack(distribute_lambda(list(self.F[p]), self.lam[p])) for p in range(P)])
        aligned, perm, scale, margins = match_replicas(Fd, S)
        rhs = [stack_rhs(aligned[:, n], S) for n in range(3)]
        A_raw = weighted_minnorm_lstsq(self.U, rhs[0], P, S)
        B_raw = weighted_minnorm_lstsq(self.V, rhs[1], P, S)
        Ac, Bc, kappa = canonicalize(A_raw, B_raw)
        if self.temporal == "full":
            Wfull = np.vstack(self.W_hist)
            C_raw = weighted_minnorm_lstsq(Wfull, rhs[2], P, S)
            C = C_raw * kappa
            self.C = C
            tperm, tsign, tmargin = np.arange(R), np.ones(R), np.inf
        else:
            if self.A is None:
                tperm, tsign, tmargin = np.arange(R), np.ones(R), np.inf
            else:
                tperm, tsign, tmargin = match_previous(Ac, Bc, self.A, self.B)
            Hcur = self.H[:, tperm] * tsign
            Cold = self.C[:, tperm] * tsign
            H_ref = Hcur / kappa
            Cnew_raw = weighted_minnorm_lstsq(self.W, rhs[2] - H_ref, P, S)
            Cnew = Cnew_raw * kappa
            self.C = np.vstack([Cold, Cnew])
            self.H = Hcur + self.W.T @ Cnew
        self.A, self.B = Ac, Bc
        self.last = dict(aligned=aligned, perm=perm, scale=scale, margins=margins,
                         rhs=rhs, A_raw=A_raw, B_raw=B_raw, kappa=kappa,
                         tperm=tperm, tsign=tsign, tmargin=tmargin, Fd=Fd)
        return self.A, self.B, self.C
