"""Narrow-type forms of the compression of Sec. 4.1 (Eq. 1), for checking the
matrix-core kernels.  TEST INFRASTRUCTURE ONLY: imported by tests, never by
the product path; it shares no code with the HIP implementation.

What a narrow form computes is defined here as the compression of its
rounded inputs with exact sums:

  f32     X as given (float32 values), U, V rounded to float32;
  bf16    X, U, V rounded to bfloat16 (8 significant bits, nearest, ties to
          even);
  bf16x2  X replaced by hi + lo with hi = bf16(x), lo = bf16(x - hi): a
          two-term bfloat16 expansion holding 16 significant bits of x;
          U, V rounded to bfloat16.

`compress_rounded` evaluates that definition in FP64 through the plain
oracle (mode 1, then 2, then 3), so nothing in it follows a kernel's order.

`error_bound` states how far a kernel may lie from the definition, entrywise,
for the arithmetic these forms prescribe: the mode-2 product
T = x_hat V accumulated in float32, T carried into the mode-1 product either
in float32 (f32), rounded once to bfloat16 (bf16) or as a two-term bfloat16
expansion (bf16x2), the mode-1 product accumulated in float32, the mode-3
product in float64 and the result stored in float32.  Products of bfloat16
values are exact in float32, so only the additions and the carry of T round.
Sums use the probabilistic bound of Higham and Mary ("A new approach to
probabilistic rounding error analysis", SIAM J. Sci. Comput. 41(5), 2019,
Thm. 3.1): a sum of n terms computed with unit roundoff u is off by at most
gamma_n(lam) * sum |terms|, gamma_n(lam) = exp(lam sqrt(n) u + n u^2/(1-u)) - 1,
except with probability at most 2 n exp(-lam^2 (1-u)^2 / 2).
"""
import math

import numpy as np

from .octen_oracle import compress_dense, replica_cols

U_BF16 = 2.0 ** -8    # unit roundoff of bfloat16 (8 significant bits)
U_F32 = 2.0 ** -24    # unit roundoff of float32 (24 significant bits)

FORMS = ("f32", "bf16", "bf16x2")


def round_bf16(x):
    """Round-to-nearest-even to bfloat16 of the float32 value of x (values
    given in float64 are first rounded to float32), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((b >> 16) & 1)
    r = ((b + bias) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def split_bf16(x):
    """Two-term bfloat16 expansion of float32 values: (hi, lo) with
    hi = bf16(x) and lo = bf16(x - hi); x - hi is exact in float32."""
    f = np.asarray(x, dtype=np.float32)
    hi = round_bf16(f)
    lo = round_bf16(f - hi.astype(np.float32))
    return hi, lo


def rounded_inputs(form, X, U, V):
    """The inputs a form computes with (float64 arrays holding exactly the
    rounded values)."""
    X = np.asarray(X, np.float32)
    if form == "f32":
        return (X.astype(np.float64), np.asarray(U, np.float32).astype(np.float64),
                np.asarray(V, np.float32).astype(np.float64))
    if form == "bf16":
        return round_bf16(X), round_bf16(U), round_bf16(V)
    if form == "bf16x2":
        hi, lo = split_bf16(X)
        return hi + lo, round_bf16(U), round_bf16(V)
    raise ValueError(form)


def compress_rounded(form, X, U, V, W, P, Q, S):
    """The definition of a narrow form: the FP64 compression of the rounded
    inputs (W stays FP64: the mode-3 product is FP64 in every form)."""
    Xr, Ur, Vr = rounded_inputs(form, X, U, V)
    return compress_dense(Xr, Ur, Vr, W, P, Q, S)


def gamma(n, lam, u):
    """Probabilistic error constant of a sum of n terms (Higham and Mary,
    Thm. 3.1)."""
    return math.expm1(lam * math.sqrt(n) * u + n * u * u / (1.0 - u))


def error_bound(form, X, U, V, W, P, Q, S, lam=8.0):
    """Entrywise bound (P, Q, Q, Q) on |Z_kernel - compress_rounded(form)|
    for the arithmetic described in the module docstring."""
    Xr, Ur, Vr = rounded_inputs(form, X, U, V)
    t, I, J = Xr.shape
    terms = 2 if form == "bf16x2" else 1           # products per (i, j) in the mode-2 sum
    g1 = gamma(terms * J, lam, U_F32)               # mode-2 sum in float32
    g2 = gamma(terms * I, lam, U_F32)               # mode-1 sum in float32
    carry = {"f32": 0.0, "bf16": U_BF16, "bf16x2": U_BF16 * U_BF16}[form]
    if form == "bf16x2":
        hi, lo = split_bf16(np.asarray(X, np.float32))
        Xabs = np.abs(hi) + np.abs(lo)
    else:
        Xabs = np.abs(Xr)
    Z = compress_dense(Xr, Ur, Vr, W, P, Q, S)
    out = np.empty((P, Q, Q, Q))
    for p in range(P):
        c = replica_cols(P, Q, S, p)
        Ua, Va, Wa = np.abs(Ur[:, c]), np.abs(Vr[:, c]), np.abs(W[:, c])
        T = np.tensordot(Xr, Vr[:, c], axes=([2], [0]))          # (t, I, Q) exact
        S1 = np.tensordot(Xabs, Va, axes=([2], [0]))            # sum |x| |V|
        # error of the carried T: float32 accumulation of the mode-2 sum,
        # then the carry into the mode-1 product
        eT = g1 * S1 + carry * (np.abs(T) + g1 * S1)
        # mode-1 sum in float32 over the carried T
        Tc = np.abs(T) + eT
        eM = np.einsum("ia,kib->kab", Ua, eT + g2 * Tc)        # (t, Q, Q)
        out[p] = np.tensordot(eM, Wa, axes=([0], [0])) + U_F32 * np.abs(Z[p]) * 1.0001
    return out
