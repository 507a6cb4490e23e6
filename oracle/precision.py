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

from .octen_oracle import compress_dense, gram_hadamard, replica_cols, replica_fit, solve_normal

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


# ---------------------------------------------------------------------------
# Two-term bfloat16 form of the replica ALS contractions (Sec. 4.1, the
# per-replica CP-ALS; the MTTKRP of Sec. 2's unfolded model)
# ---------------------------------------------------------------------------

def two_term_product(X, B):
    """X (n x k) times B (k x m) with both operands taken as two-term
    bfloat16 expansions of their float32 values, x = hi + lo, and each scalar
    product as hi_x hi_b + lo_x hi_b + hi_x lo_b (the lo_x lo_b term dropped).
    Every such product of bfloat16 values is exact; the sums here are FP64."""
    xh, xl = split_bf16(np.asarray(X, np.float32))
    bh, bl = split_bf16(np.asarray(B, np.float32))
    return xh @ bh + xl @ bh + xh @ bl


def _two_term_abs(X, B):
    """Sums of the absolute values of the terms two_term_product adds."""
    xh, xl = split_bf16(np.asarray(X, np.float32))
    bh, bl = split_bf16(np.asarray(B, np.float32))
    return np.abs(xh) @ np.abs(bh) + np.abs(xl) @ np.abs(bh) + np.abs(xh) @ np.abs(bl)


def als_two_term_bound(tr, Q, lam=8.0):
    """Normwise relative bound on how far one sweep of the two-term ALS run
    with float32 sums may lie from cp_als_two_term (exact sums), from the
    trace of that sweep.  T sums 3 Q terms and M3 3 Q^2 terms in float32
    (Higham-Mary constant gamma); to first order, a solve F = M G^-1 turns
    relative errors dM, dG into kappa(G) (dM + dG), the column normalisation
    at most doubles it, a Gram matrix carries twice its factor's error and an
    MTTKRP the sum of its operands' errors:
      dA = 2 k1 eT,  dB = 2 k2 (eT + 3 dA),  dC = 2 k3 (e3 + 3 dA + 3 dB).
    Returns max(dA, dB, dC)."""
    eT = gamma(3 * Q, lam, U_F32) * np.linalg.norm(tr["T_abs"]) / np.linalg.norm(tr["T"])
    e3 = gamma(3 * Q * Q, lam, U_F32) * np.linalg.norm(tr["M3_abs"]) / np.linalg.norm(tr["M3"])
    k1, k2, k3 = (np.linalg.cond(G) for G in tr["G"])
    dA = 2 * k1 * eT
    dB = 2 * k2 * (eT + 3 * dA)
    dC = 2 * k3 * (e3 + 3 * dA + 3 * dB)
    return max(dA, dB, dC)


def cp_als_two_term(Y, init, iters, tol=0.0, trace=None):
    """Replica CP-ALS (Gauss-Seidel over modes 1, 2, 3, columns normalised
    after every mode, lambda from the last mode; the plain oracle's cp_als)
    in which the two contractions with the slab are taken in the two-term
    form:
      T(a, b, r) = sum_c Y(a, b, c) C(c, r)          (serves modes 1 and 2,
                                                       C being fixed for both)
      M1(a, r) = sum_b T(a, b, r) B(b, r),  M2(b, r) = sum_a T(a, b, r) A(a, r)
      W(ab, r) = float32(A(a, r) B(b, r)),  M3(c, r) = sum_ab Y(a, b, c) W(ab, r)
    with T and M3 by two_term_product; everything else (M1, M2, the Grams, the
    R x R solves, the norms) in FP64.  Y is the float32 replica summary
    (Q, Q, Q).  Returns (F, lam, sweeps, fallback flag) like cp_als.

    trace: None or a list that receives, per sweep, a dict with the three
    normal matrices ("G": [G1, G2, G3]) and, for T and M3, the value and the
    sum of the absolute values of its terms ("T", "T_abs", "M3", "M3_abs"),
    for error bounds."""
    Y = np.asarray(Y, np.float32)
    Q = Y.shape[0]
    Yab = Y.reshape(Q * Q, Q)                 # row a Q + b, column c
    F = [np.array(f, dtype=np.float64) for f in init]
    R = F[0].shape[1]
    lam = np.ones(R)
    done, fit_old, flag = 0, None, False
    Yd = Y.astype(np.float64)

    Gs = []

    def update(n, M):
        nonlocal lam, flag
        G = gram_hadamard(F, n)
        Gs.append(G)
        Fn, fb = solve_normal(M, G)
        flag |= fb
        nrm = np.linalg.norm(Fn, axis=0)
        nrm = np.where(nrm > 0, nrm, 1.0)
        F[n] = Fn / nrm
        lam = nrm

    for _ in range(iters):
        Gs.clear()
        Cf = F[2]
        T = two_term_product(Yab, Cf).reshape(Q, Q, R)
        update(0, np.einsum("abr,br->ar", T, F[1]))
        update(1, np.einsum("abr,ar->br", T, F[0]))
        W = (F[0][:, None, :] * F[1][None, :, :]).astype(np.float32).reshape(Q * Q, R)
        M3 = two_term_product(Yab.T, W)
        update(2, M3)
        done += 1
        if trace is not None:
            trace.append({"G": list(Gs), "T": T.reshape(Q * Q, R),
                          "T_abs": _two_term_abs(Yab, Cf), "M3": M3,
                          "M3_abs": _two_term_abs(Yab.T, W)})
        if tol > 0:
            fit = replica_fit(Yd, F, lam, M3)
            if fit_old is not None and abs(fit - fit_old) < tol:
                break
            fit_old = fit
    return F, lam, done, flag
