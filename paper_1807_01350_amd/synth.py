"""Seeded synthetic inputs for the online CP workloads.

This module is shared by the oracle side and the HIP side: it draws random
numbers and lays them out, and holds none of the method's arithmetic (no
compression, no ALS, no matching, no recovery, no fit).

The workload model follows the paper's synthetic protocol (Sec. 5.3,
"Experimental Setup", and the dataset table there): factor matrices of known
rank R with uniformly distributed entries, a tensor built from them, plus
Gaussian noise, streamed along the third (time) mode in batches of frontal
slices.  The random compression matrices (Sec. 4.1, Eq. 1) and the ALS
starting point are random draws of the method itself; they are produced here
and passed to both implementations as inputs.

Seeds: ``numpy.random.Generator(PCG64(seed))`` with
``seed = 180701350 + 1000 * config_id + purpose`` and purpose
0 = factors, 1 = noise, 2 = compression matrices, 3 = ALS init, 4 = MLP,
5 = sparse coordinates.  Per-batch draws use ``SeedSequence([seed, batch])``.
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED_BASE = 180701350

PURPOSE_FACTORS = 0
PURPOSE_NOISE = 1
PURPOSE_COMPRESSION = 2
PURPOSE_ALS_INIT = 3
PURPOSE_MLP = 4
PURPOSE_COORDS = 5


def seed_of(config_id: int, purpose: int) -> int:
    return SEED_BASE + 1000 * int(config_id) + int(purpose)


def rng(config_id: int, purpose: int, sub: int | None = None) -> np.random.Generator:
    s = seed_of(config_id, purpose)
    if sub is None:
        return np.random.Generator(np.random.PCG64(s))
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([s, int(sub)])))


@dataclasses.dataclass(frozen=True)
class StreamConfig:
    """One streamed workload: sizes, replica layout and batch schedule."""
    name: str
    config_id: int
    I: int
    J: int
    R: int
    P: int
    Q: int
    S: int
    t0: int                 # slices in the initial batch (summary of X_old)
    batches: tuple          # depths of the update batches
    sigma: float = 0.01     # noise standard deviation
    iters: int = 50         # fixed ALS iterations
    x_dtype: str = "f64"    # element type of the streamed slices
    nnz_per_slice: int = 0  # sparse streams: coordinate draws per slice
    zipf_a: float = 0.0     # sparse streams: Zipf exponent of modes 1 and 2

    @property
    def M1(self) -> int:
        """Distinct compression columns per mode: S shared + P*(Q-S) private."""
        return self.S + self.P * (self.Q - self.S)

    @property
    def K(self) -> int:
        return self.t0 + int(sum(self.batches))

    def schedule(self):
        """List of (k0, t): first slice index and depth of every batch."""
        out, k = [(0, self.t0)], self.t0
        for t in self.batches:
            out.append((k, int(t)))
            k += int(t)
        return out


# The dense 50^3 case: 30 initial slices then two batches of 10, P=4 replicas of
# 20^3, 3 shared anchor rows, 50 ALS iterations, FP64.
C1 = StreamConfig("dense50_f64", 1, I=50, J=50, R=5, P=4, Q=20, S=3, t0=30,
                  batches=(10, 10), x_dtype="f64")
# The dense 1000^3 case: 500 initial slices then ten batches of 50, P=12
# replicas of 60^3, 3 shared anchor rows, 50 ALS iterations, FP32 slices.
C2 = StreamConfig("dense1000_f32", 2, I=1000, J=1000, R=10, P=12, Q=60, S=3,
                  t0=500, batches=(50,) * 10, x_dtype="f32")
# The sparse 10^5 x 10^5 stream: 2000 slices of 10^5 Zipf(1.2)-distributed
# coordinate draws each (density about 1e-5), rank 20; 200 initial slices then
# batches of 100; P=16 replicas of 80^3 with 3 shared anchor rows.
C3 = StreamConfig("sparse1e5_f32", 3, I=100_000, J=100_000, R=20, P=16, Q=80, S=3,
                  t0=200, batches=(100,) * 18, x_dtype="f32", nnz_per_slice=100_000,
                  zipf_a=1.2)


def replica_columns(P: int, Q: int, S: int, p: int) -> np.ndarray:
    """Column indices of replica p inside the deduplicated compression matrix:
    the S shared columns first, then replica p's Q-S private columns."""
    return np.r_[np.arange(S), S + p * (Q - S) + np.arange(Q - S)].astype(np.int64)


def cp_factors(I: int, J: int, K: int, R: int, config_id: int):
    """Ground-truth factors with U[0,1] entries (Sec. 5.3)."""
    g = rng(config_id, PURPOSE_FACTORS)
    A = g.random((I, R))
    B = g.random((J, R))
    C = g.random((K, R))
    return A, B, C


def dense_stream(I: int, J: int, K: int, R: int, sigma: float, config_id: int,
                 dtype=np.float64, noiseless: bool = False):
    """X[k][i][j] = sum_r A(i,r) B(j,r) C(k,r) + sigma * N(0,1); returns
    (A, B, C, X) with X in `dtype`, slice-major (j fastest)."""
    A, B, C = cp_factors(I, J, K, R, config_id)
    X = np.einsum("ir,jr,kr->kij", A, B, C)
    if not noiseless and sigma > 0:
        X += sigma * rng(config_id, PURPOSE_NOISE).standard_normal(X.shape)
    return A, B, C, np.ascontiguousarray(X.astype(dtype))


def to_bf16_grid(x):
    """Nearest value with 8 significant bits (the bfloat16 grid), ties to
    even, returned as float64.  Used to draw compression matrices whose
    entries the bfloat16 matrix cores take without rounding."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def compression_UV(I: int, J: int, P: int, Q: int, S: int, config_id: int):
    """Fixed mode-1/mode-2 compression matrices in deduplicated layout
    U = [G | H_1 | ... | H_P] (I x M1), same for V: N(0,1) draws rounded to
    the bfloat16 grid (8 significant bits).  The method needs only that
    compression and recovery use the same random matrices; on this grid every
    arithmetic form of the compression takes them exactly."""
    M1 = S + P * (Q - S)
    g = rng(config_id, PURPOSE_COMPRESSION)
    U = to_bf16_grid(g.standard_normal((I, M1)))
    V = to_bf16_grid(g.standard_normal((J, M1)))
    return np.ascontiguousarray(U), np.ascontiguousarray(V)


def temporal_W(t: int, M1: int, config_id: int, batch: int):
    """Fresh mode-3 compression rows for one batch: W (t x M1), N(0,1)."""
    g = rng(config_id, PURPOSE_COMPRESSION, sub=1000 + batch)
    return np.ascontiguousarray(g.standard_normal((t, M1)))


def als_init(P: int, Q: int, R: int, config_id: int):
    """Seeded N(0,1) starting factors for the first batch: (P, 3, Q, R)."""
    g = rng(config_id, PURPOSE_ALS_INIT)
    return np.ascontiguousarray(g.standard_normal((P, 3, Q, R)))


def zipf_indices(g: np.random.Generator, n: int, size: int, a: float):
    """Truncated Zipf(a) over [0, n) followed by a fixed random relabelling."""
    ranks = np.arange(1, n + 1, dtype=np.float64)
    w = ranks ** (-a)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    r = np.searchsorted(cdf, g.random(size), side="right")
    r = np.minimum(r, n - 1)
    relabel = g.permutation(n)
    return relabel[r]


def coo_stream(I: int, J: int, K: int, R: int, nnz_per_slice: int, sigma: float,
               config_id: int, zipf_a: float = 1.2):
    """Sparse COO stream: modes 1 and 2 truncated Zipf(a) with a fixed random
    relabelling, mode 3 uniform (nnz_per_slice draws per slice), de-duplicated
    and sorted by (k, i, j).  Values are a rank-R CP model with U[0,1] factors
    evaluated at the coordinates plus sigma * N(0,1).

    Returns (A, B, C, k, i, j, v) with int32 coordinates and float32 values."""
    A, B, C = cp_factors(I, J, K, R, config_id)
    g = rng(config_id, PURPOSE_COORDS)
    gi = np.random.Generator(np.random.PCG64(g.integers(1 << 62)))
    gj = np.random.Generator(np.random.PCG64(g.integers(1 << 62)))
    relabel_i = gi.permutation(I)
    relabel_j = gj.permutation(J)
    wi = np.arange(1, I + 1, dtype=np.float64) ** (-zipf_a)
    wj = np.arange(1, J + 1, dtype=np.float64) ** (-zipf_a)
    cdf_i = np.cumsum(wi); cdf_i /= cdf_i[-1]
    cdf_j = np.cumsum(wj); cdf_j /= cdf_j[-1]
    ks, is_, js = [], [], []
    for k in range(K):
        ii = relabel_i[np.minimum(np.searchsorted(cdf_i, g.random(nnz_per_slice), side="right"), I - 1)]
        jj = relabel_j[np.minimum(np.searchsorted(cdf_j, g.random(nnz_per_slice), side="right"), J - 1)]
        key = np.unique(ii.astype(np.int64) * J + jj)
        ks.append(np.full(key.size, k, np.int64))
        is_.append(key // J)
        js.append(key % J)
    k = np.concatenate(ks).astype(np.int32)
    i = np.concatenate(is_).astype(np.int32)
    j = np.concatenate(js).astype(np.int32)
    vals = np.einsum("nr,nr,nr->n", A[i], B[j], C[k])
    vals += sigma * rng(config_id, PURPOSE_NOISE).standard_normal(vals.shape)
    return A, B, C, k, i, j, vals.astype(np.float32)


def mlp_params(n_in: int, n_hidden: int, n_out: int, config_id: int, last_scale: float = 0.0):
    """Starting parameters of the warm-start network, FP32, in the layout
    W1 [H][In], b1, W2 [H][H], b2, W3 [Out][H], b3: He-normal hidden weights,
    zero biases, last layer N(0, last_scale^2 / H) (0: the network starts as
    the identity on the previous columns)."""
    g = rng(config_id, PURPOSE_MLP)
    W1 = g.standard_normal((n_hidden, n_in)) * np.sqrt(2.0 / n_in)
    W2 = g.standard_normal((n_hidden, n_hidden)) * np.sqrt(2.0 / n_hidden)
    W3 = g.standard_normal((n_out, n_hidden)) * (last_scale / np.sqrt(n_hidden))
    parts = [W1, np.zeros(n_hidden), W2, np.zeros(n_hidden), W3, np.zeros(n_out)]
    return np.concatenate([x.reshape(-1) for x in parts]).astype(np.float32)


def sketch_matrix(D: int, Q: int, config_id: int):
    """Fixed Gaussian sketch of a replica summary: D x Q^3, N(0, 1/D), FP32."""
    g = rng(config_id, PURPOSE_MLP, sub=77)
    return (g.standard_normal((D, Q ** 3)) / np.sqrt(D)).astype(np.float32)


# ---------------------------------------------------------------- N modes ---

def nmode_factors(dims, K: int, R: int, config_id: int):
    """Ground-truth factors of an N-mode stream (N = len(dims) + 1): one
    U[0,1] matrix per non-temporal mode and the temporal C (K x R)."""
    g = rng(config_id, PURPOSE_FACTORS, sub=len(dims))
    fac = [g.random((int(d), R)) for d in dims]
    C = g.random((K, R))
    return fac, C


def nmode_slices(fac, C, k0: int, t: int, sigma: float, config_id: int, batch: int):
    """Slices k0 .. k0+t-1 of the N-mode stream: the rank-R model of the
    factors plus sigma * N(0,1) (a draw per batch), shape (t, I_1, ...,
    I_{N-1}), the last mode fastest, float64."""
    letters = "abcdefg"[:len(fac)]
    X = np.einsum("kr," + ",".join(l + "r" for l in letters) + "->k" + letters,
                  C[k0:k0 + t], *fac)
    if sigma > 0:
        X += sigma * rng(config_id, PURPOSE_NOISE, sub=batch).standard_normal(X.shape)
    return np.ascontiguousarray(X)


def compression_Us(dims, P: int, Q: int, S: int, config_id: int):
    """Fixed compression matrices of the non-temporal modes, deduplicated
    layout (I_n x M1), N(0,1) rounded to the bfloat16 grid as for three modes."""
    M1 = S + P * (Q - S)
    g = rng(config_id, PURPOSE_COMPRESSION, sub=len(dims))
    return [np.ascontiguousarray(to_bf16_grid(g.standard_normal((int(d), M1)))) for d in dims]


def nmode_als_init(P: int, N: int, Q: int, R: int, config_id: int):
    """Seeded N(0,1) starting factors of the first batch: (P, N, Q, R)."""
    g = rng(config_id, PURPOSE_ALS_INIT, sub=N)
    return np.ascontiguousarray(g.standard_normal((P, N, Q, R)))
