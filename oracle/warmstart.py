"""Learned warm start for the replica ALS: FP64 reference (test infrastructure
only; the product path never imports it).

The paper warm-starts each replica's ALS from its previous factors (Sec. 4.1,
Algorithm 1 third step).  The learned form predicts a better starting point
column by column:

  features of column r of replica p (length 4Q + D):
      [ s_a a_r ; s_b b_r ; s_a s_b (c_r + u_r) ; s_a s_b u_r ; sketch_p ]
  where a_r, b_r, c_r are the previous unit columns times lambda_r^(1/3)
  (the lambda distribution of Sec. 4.2), s_a and s_b make the entry of
  largest magnitude of a_r and of b_r positive (ties: the first such entry),
  u_r = (Z_p x1 a_r x2 b_r) / (||a_r||^2 ||b_r||^2) is the change of the
  mode-3 least-squares column that the new compressed batch Z_p causes when
  a_r, b_r are held and the other columns are ignored (exact for rank one),
  and sketch_p = G vec(Z_p) / ||Z_p|| is a fixed Gaussian projection of the
  new batch (D rows of G);
  network: residual MLP  y = x[:3Q] + W3 relu(W2 relu(W1 x + b1) + b2) + b3,
  so an untrained network (W3 = 0, b3 = 0) proposes [a; b; c + u];
  target: the columns after ALS on the updated summary, lambda^(1/3)-scaled
  and with the same s_a, s_b applied;
  candidate init: y with the signs undone; kept for a replica only if its
  replica fit (Sec. 5.1 on the summary) is at least that of the plain warm
  start, else the plain warm start is used.

Training minimises the mean squared error with Adam.  Every function here is
plain FP64 NumPy written from these definitions.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "mlp_param_shapes", "mlp_forward", "mlp_backward", "mse_loss", "adam_step",
    "sketch", "column_signs", "mode3_change", "warmstart_features", "warmstart_targets",
    "candidate_init", "replica_fit_of", "judge",
]


def mlp_param_shapes(n_in, n_hidden, n_out):
    """(W1, b1, W2, b2, W3, b3) with W stored as [out][in]."""
    return [(n_hidden, n_in), (n_hidden,), (n_hidden, n_hidden), (n_hidden,),
            (n_out, n_hidden), (n_out,)]


def _ident(x):
    return x


def mlp_forward(params, X, n_out, rnd=None):
    """Y = X[:, :n_out] + W3 relu(W2 relu(W1 X + b1) + b2) + b3, row-wise.
    Returns Y and the activations needed by the backward pass.  rnd, if
    given, is applied to both operands of every matrix product (a network
    whose products take narrower operands, e.g. bfloat16, with exact sums);
    biases, rectifiers and the residual stay exact."""
    r = rnd or _ident
    W1, b1, W2, b2, W3, b3 = params
    X = np.asarray(X, np.float64)
    Z1 = r(X) @ r(W1).T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = r(H1) @ r(W2).T + b2
    H2 = np.maximum(Z2, 0.0)
    Y = X[:, :n_out] + r(H2) @ r(W3).T + b3
    return Y, (X, Z1, H1, Z2, H2)


def mse_loss(Y, T):
    """L = mean over all entries of (Y - T)^2 and dL/dY."""
    D = Y - T
    n = D.size
    return float(np.sum(D * D) / n), 2.0 * D / n


def mlp_backward(params, cache, dY, rnd=None):
    """Gradients of a scalar loss with dL/dY given, by the chain rule through
    the three affine maps and the two rectifiers (relu'(0) = 0).  The
    residual path adds dY to dL/dX but X is an input, so it is not returned.
    rnd as in mlp_forward: applied to both operands of every product."""
    r = rnd or _ident
    W1, b1, W2, b2, W3, b3 = params
    X, Z1, H1, Z2, H2 = cache
    gW3 = r(dY).T @ r(H2)
    gb3 = dY.sum(0)
    dH2 = r(dY) @ r(W3)
    dZ2 = dH2 * (Z2 > 0)
    gW2 = r(dZ2).T @ r(H1)
    gb2 = dZ2.sum(0)
    dH1 = r(dZ2) @ r(W2)
    dZ1 = dH1 * (Z1 > 0)
    gW1 = r(dZ1).T @ r(X)
    gb1 = dZ1.sum(0)
    return [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) of every array, in place;
    step counts from 1."""
    c1 = 1.0 - beta1 ** step
    c2 = 1.0 - beta2 ** step
    for w, g, mm, vv in zip(params, grads, m, v):
        mm *= beta1
        mm += (1.0 - beta1) * g
        vv *= beta2
        vv += (1.0 - beta2) * g * g
        w -= lr * (mm / c1) / (np.sqrt(vv / c2) + eps)


def sketch(Z, G):
    """G vec(Z_p) / ||Z_p|| for every replica p; Z: [P][Q][Q][Q], G: [D][Q^3].
    A zero summary gives a zero sketch."""
    Z = np.asarray(Z, np.float64)
    P = Z.shape[0]
    out = np.zeros((P, G.shape[0]))
    for p in range(P):
        z = Z[p].reshape(-1)
        nz = np.linalg.norm(z)
        if nz > 0:
            out[p] = G @ (z / nz)
    return out


def column_signs(x):
    """+1 or -1 per column: the sign of the entry of largest magnitude (first
    one on ties; +1 for a zero column)."""
    idx = np.argmax(np.abs(x), axis=0)
    s = np.sign(x[idx, np.arange(x.shape[1])])
    s[s == 0] = 1.0
    return s


def _scaled(F, lam):
    """Columns of the three modes times lambda^(1/3): F [3][Q][R]."""
    c = np.cbrt(np.asarray(lam, np.float64))
    return [F[n] * c for n in range(3)]


def mode3_change(Z, a, b):
    """u = (Z x1 a x2 b) / (||a||^2 ||b||^2) for one column pair, Z [Q][Q][Q]."""
    return np.einsum("abc,a,b->c", Z, a, b) / (np.dot(a, a) * np.dot(b, b))


def warmstart_features(F, lam, sk, Z):
    """Features of every column of every replica: rows ordered (p, r).
    F: [P][3][Q][R] unit columns, lam: [P][R], sk: [P][D], Z: [P][Q][Q][Q].
    Returns X [P*R][4Q + D] and the signs [P][R][2] (s_a, s_b)."""
    P, _, Q, R = F.shape
    D = sk.shape[1]
    X = np.zeros((P * R, 4 * Q + D))
    signs = np.zeros((P, R, 2))
    for p in range(P):
        a, b, c = _scaled(F[p], lam[p])
        sa, sb = column_signs(a), column_signs(b)
        signs[p, :, 0], signs[p, :, 1] = sa, sb
        for r in range(R):
            u = mode3_change(np.asarray(Z[p], np.float64), a[:, r], b[:, r])
            s3 = sa[r] * sb[r]
            X[p * R + r] = np.concatenate([sa[r] * a[:, r], sb[r] * b[:, r],
                                           s3 * (c[:, r] + u), s3 * u, sk[p]])
    return X, signs


def warmstart_targets(F, lam, signs):
    """Targets [P*R][3Q] from the factors after ALS, with the feature signs."""
    P, _, Q, R = F.shape
    T = np.zeros((P * R, 3 * Q))
    for p in range(P):
        a, b, c = _scaled(F[p], lam[p])
        for r in range(R):
            sa, sb = signs[p, r]
            T[p * R + r] = np.concatenate([sa * a[:, r], sb * b[:, r], sa * sb * c[:, r]])
    return T


def candidate_init(Y, signs, Q):
    """Network outputs [P*R][3Q] back to factors [P][3][Q][R] (signs undone)."""
    P, R, _ = signs.shape
    out = np.zeros((P, 3, Q, R))
    for p in range(P):
        for r in range(R):
            sa, sb = signs[p, r]
            y = Y[p * R + r]
            out[p, 0, :, r] = sa * y[:Q]
            out[p, 1, :, r] = sb * y[Q:2 * Q]
            out[p, 2, :, r] = sa * sb * y[2 * Q:]
    return out


def replica_fit_of(Y, A, B, C):
    """Sec. 5.1 fit of the model [[A, B, C]] to one summary Y [Q][Q][Q],
    written out entrywise (no Gram identity)."""
    Xh = np.einsum("ar,br,cr->abc", A, B, C)
    ny = np.linalg.norm(Y)
    return 1.0 - np.linalg.norm(Y - Xh) / ny if ny > 0 else 0.0


def judge(Ysum, cand, F, lam):
    """Per replica: use the candidate if its fit is at least that of the plain
    warm start (previous columns times lambda^(1/3)).  Returns the chosen
    starting factors [P][3][Q][R] and a bool array (True = learned kept)."""
    P = Ysum.shape[0]
    chosen = np.zeros_like(cand)
    keep = np.zeros(P, bool)
    for p in range(P):
        a, b, c = _scaled(F[p], lam[p])
        f_plain = replica_fit_of(Ysum[p], a, b, c)
        f_cand = replica_fit_of(Ysum[p], *cand[p])
        keep[p] = f_cand >= f_plain
        chosen[p] = cand[p] if keep[p] else np.stack([a, b, c])
    return chosen, keep
