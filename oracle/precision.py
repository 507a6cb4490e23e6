"""Emulation of narrow input types for checking the matrix-core forms of the
compression (test infrastructure only).

round_bf16: round-to-nearest-even of float32 values to bfloat16 (8
significant bits), returned as float64.  Values given in float64 are first rounded to
float32, as the HIP path does when it packs its operands.

compress_dense_bf16_emulated: the multi-mode product of Sec. 4.1 (Eq. 1) with
every input rounded to bfloat16 and the intermediate X_k V rounded to
bfloat16 once more, exactly where the bfloat16 matrix-core path rounds it;
all sums are exact FP64.  The contraction order follows that path (mode 2,
then mode 1, then mode 3), because the intermediate rounding depends on it.
"""
import numpy as np

from .octen_oracle import replica_cols


def round_bf16(x):
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((b >> 16) & 1)
    r = ((b + bias) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def compress_dense_bf16_emulated(X, U, V, W, P, Q, S):
    Xb = round_bf16(np.asarray(X, np.float32))
    Ub = round_bf16(U)
    Vb = round_bf16(V)
    t = Xb.shape[0]
    Z = np.empty((P, Q, Q, Q))
    for p in range(P):
        c = replica_cols(P, Q, S, p)
        # mode 2 first: T2[k, i, b] = sum_j X(k, i, j) V_p(j, b), rounded
        T2 = round_bf16(np.tensordot(Xb, Vb[:, c], axes=([2], [0])).astype(np.float32))
        # mode 1: M[k, a, b] = sum_i U_p(i, a) T2[k, i, b]
        M = np.einsum("ia,kib->kab", Ub[:, c], T2)
        # mode 3 with the unrounded W
        Z[p] = np.tensordot(M, W[:, c], axes=([0], [0]))
    return Z
