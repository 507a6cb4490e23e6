"""Python binding of libocten (ctypes).  Argument marshalling only: every step
of the update runs in the HIP library; torch supplies device memory and the
stream.  The functions carry the C names; `Octen` wraps a handle.

Importing this module loads the built library and fails loudly if it is
missing: there is no fallback implementation.  torch is imported first so
that the library binds to the HIP runtime torch has loaded: a process must
hold one HIP runtime, or device memory from one is unknown to the other.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (must precede the library load, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libocten.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libocten.so is not built ({LIB_PATH}); run `python -m paper_1807_01350_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

OCTEN_ABI_VERSION = 1
OCTEN_OK, OCTEN_ERR_ARG, OCTEN_ERR_STATE, OCTEN_ERR_HIP, OCTEN_ERR_NOMEM, OCTEN_ERR_NUMERIC, \
    OCTEN_ERR_UNSUPPORTED = range(7)
OCTEN_F64, OCTEN_F32, OCTEN_BF16, OCTEN_BF16X2 = 0, 1, 2, 4
OCTEN_INIT_GIVEN, OCTEN_INIT_PREV, OCTEN_INIT_LEARNED = 0, 1, 2
(OCTEN_STATE_Y, OCTEN_STATE_Z, OCTEN_STATE_FACTORS, OCTEN_STATE_LAMBDA, OCTEN_STATE_PERM,
 OCTEN_STATE_ALIGNED, OCTEN_STATE_RHS, OCTEN_STATE_H, OCTEN_STATE_TPERM, OCTEN_STATE_ITERS,
 OCTEN_STATE_MARGIN, OCTEN_STATE_FLAGS, OCTEN_STATE_COO_SIZES, OCTEN_STATE_COO_SEG_START,
 OCTEN_STATE_COO_SEG_ROW, OCTEN_STATE_COO_SLICE_SEG, OCTEN_STATE_WARM_KEEP,
 OCTEN_STATE_WARM_FITS) = range(18)
OCTEN_FLAG_REFERENCE_PATH = 0x2
OCTEN_FLAG_TIMING = 0x4
OCTEN_FLAG_ALS_ONE_WG = 0x8
OCTEN_FLAG_ALS_DEVICE_SYNC = 0x10
OCTEN_FLAG_ALS_FEW_WG = 0x20
(OCTEN_STAGE_COMPRESS_MAIN, OCTEN_STAGE_COMPRESS_MODE3, OCTEN_STAGE_UPDATE, OCTEN_STAGE_ALS,
 OCTEN_STAGE_RECOVER, OCTEN_STAGE_COO_INDEX) = range(6)

DTYPES = {"f64": OCTEN_F64, "f32": OCTEN_F32, "bf16": OCTEN_BF16, "bf16x2": OCTEN_BF16X2}


class octen_batch_desc(ctypes.Structure):
    _fields_ = [
        ("X", ctypes.c_void_p),
        ("t", ctypes.c_int64),
        ("W", ctypes.c_void_p),
        ("slice_scale", ctypes.c_void_p),
    ]


class octen_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("R", ctypes.c_int32),
        ("P", ctypes.c_int32),
        ("Q", ctypes.c_int32),
        ("S", ctypes.c_int32),
        ("x_dtype", ctypes.c_int32),
        ("compress_dtype", ctypes.c_int32),
        ("als_dtype", ctypes.c_int32),
        ("I", ctypes.c_int64),
        ("J", ctypes.c_int64),
        ("flags", ctypes.c_uint64),
    ]


OCTEN_NM_MAX_MODES = 6


class octen_nm_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("N", ctypes.c_int32),
        ("R", ctypes.c_int32),
        ("P", ctypes.c_int32),
        ("Q", ctypes.c_int32),
        ("S", ctypes.c_int32),
        ("dims", ctypes.c_int64 * (OCTEN_NM_MAX_MODES - 1)),
    ]


_vp = ctypes.c_void_p
_i32, _i64, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_SIGS = {
    "octen_init": ([ctypes.POINTER(octen_config), _vp, _vp, _vp, ctypes.POINTER(_vp)], _i32),
    "octen_compress_batch": ([_vp, _vp, _i64, _vp, _vp], _i32),
    "octen_compress_batch_async": ([_vp, _vp, _i64, _vp, _vp], _i32),
    "octen_compress_batch_coo": ([_vp, _i64, _vp, _vp, _vp, _vp, _i64, _vp], _i32),
    "octen_update_replicas": ([_vp], _i32),
    "octen_health": ([_vp, _vp], _i32),
    "octen_fit_noalloc": ([_vp, _i32, _i64, _i64, _i64, _i32, _i64, _vp, _vp, _vp, _vp, _vp], _i32),
    "octen_cp_als_replicas": ([_vp, _i32, _f64, _i32, _vp, _vp], _i32),
    "octen_recover_factors": ([_vp, _vp, _vp, _vp, _i64, _vp], _i32),
    "octen_fit": ([_vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp], _i32),
    "octen_fit_coo": ([_vp, _i64, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _i64, _vp], _i32),
    "octen_get_state": ([_vp, _i32, _vp, ctypes.c_size_t], _i32),
    "octen_check_identifiable": ([ctypes.POINTER(octen_config), _i64, _i64, _vp, _vp], _i32),
    "octen_stage_times": ([_vp, _i32, _vp, _i32, _vp], _i32),
    "octen_destroy": ([_vp], _i32),
    "octen_status_str": ([_i32], ctypes.c_char_p),
    "octen_last_error": ([_vp], ctypes.c_char_p),
    "octen_abi_version": ([], _i32),
    "octen_mlp_param_count": ([_i32, _i32, _i32], _i64),
    "octen_mlp_create": ([_i32, _i32, _i32, _vp, _vp, ctypes.POINTER(_vp)], _i32),
    "octen_mlp_destroy": ([_vp], _i32),
    "octen_mlp_last_error": ([_vp], ctypes.c_char_p),
    "octen_mlp_forward": ([_vp, _vp, _i64, _vp], _i32),
    "octen_mlp_gradients": ([_vp, _vp, _vp, _i64, _vp, _vp], _i32),
    "octen_mlp_adam": ([_vp, _vp, ctypes.c_float], _i32),
    "octen_mlp_train_step": ([_vp, _vp, _vp, _i64, ctypes.c_float, _vp], _i32),
    "octen_mlp_get_params": ([_vp, _vp], _i32),
    "octen_mlp_last_activations": ([_vp, _i64, _vp, _vp], _i32),
    "octen_autotune": ([_vp, _vp, _i64, _vp], _i32),
    "octen_compress_variant": ([_vp, _i32], _i32),
    "octen_autotune_als": ([_vp, _i32, _vp], _i32),
    "octen_group_create": ([_vp, _i32, ctypes.POINTER(_vp)], _i32),
    "octen_group_step": ([_vp, _vp, _i32, _f64, _i32, _vp], _i32),
    "octen_group_recover": ([_vp, _vp, _vp, _vp, _vp], _i32),
    "octen_group_als_launches": ([_vp, _vp], _i32),
    "octen_group_destroy": ([_vp], _i32),
    "octen_group_last_error": ([_vp], ctypes.c_char_p),
    "octen_warmstart_set": ([_vp, _vp, _vp, _i32], _i32),
    "octen_warmstart_features": ([_vp, _vp], _i32),
    "octen_warmstart_targets": ([_vp, _vp], _i32),
    "octen_nm_init": ([ctypes.POINTER(octen_nm_config), _vp, _vp, ctypes.POINTER(_vp)], _i32),
    "octen_nm_compress_batch": ([_vp, _vp, _i64, _vp], _i32),
    "octen_nm_update_replicas": ([_vp], _i32),
    "octen_nm_cp_als_replicas": ([_vp, _i32, _i32, _vp], _i32),
    "octen_nm_recover_factors": ([_vp, _vp, _vp, _i64, _vp], _i32),
    "octen_nm_fit": ([_vp, _vp, _i64, _i64, _vp, _vp, _vp], _i32),
    "octen_nm_get_state": ([_vp, _i32, _vp, ctypes.c_size_t], _i32),
    "octen_nm_destroy": ([_vp], _i32),
    "octen_nm_last_error": ([_vp], ctypes.c_char_p),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


class OctenError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        msg = f"{where}: {_lib.octen_status_str(status).decode()}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


def _ptr(x):
    """Device/host address of a torch tensor, or an int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def make_config(I, J, R, P, Q, S, x_dtype="f64", compress_dtype="f64", als_dtype="f64", flags=0):
    c = octen_config()
    c.abi_version = OCTEN_ABI_VERSION
    c.I, c.J, c.R, c.P, c.Q, c.S = int(I), int(J), int(R), int(P), int(Q), int(S)
    c.x_dtype = DTYPES[x_dtype]
    c.compress_dtype = DTYPES[compress_dtype]
    c.als_dtype = DTYPES[als_dtype]
    c.flags = int(flags)
    return c


# ---------------------------------------------------------------------------
# Functions with the C names (status codes returned as ints).
# ---------------------------------------------------------------------------

def octen_abi_version():
    return _lib.octen_abi_version()


def octen_init(cfg, U, V, stream=None):
    h = _vp()
    st = _lib.octen_init(ctypes.byref(cfg), _ptr(U), _ptr(V), stream, ctypes.byref(h))
    return st, h


def octen_compress_batch(h, X, t, W, slice_scale=None):
    return _lib.octen_compress_batch(h, _ptr(X), int(t), _ptr(W), _ptr(slice_scale))


def octen_compress_batch_async(h, X, t, W, slice_scale=None):
    return _lib.octen_compress_batch_async(h, _ptr(X), int(t), _ptr(W), _ptr(slice_scale))


def octen_compress_batch_coo(h, nnz, k, i, j, v, t, W):
    return _lib.octen_compress_batch_coo(h, int(nnz), _ptr(k), _ptr(i), _ptr(j), _ptr(v), int(t),
                                         _ptr(W))


def octen_update_replicas(h):
    return _lib.octen_update_replicas(h)


OCTEN_HEALTH_NONFINITE_BATCH, OCTEN_HEALTH_ALS_FAILED = 0x1, 0x2


def octen_fit_noalloc(X, t, I, J, R, k0, A, B, C, stream=None, acc=(0.0, 0.0)):
    """Dense fitness terms without a handle and without device allocation
    (X: float32 or float64 torch tensor [t][I][J]); returns (status,
    (sse, sum X^2)) with the terms added to acc."""
    out = (ctypes.c_double * 2)(*acc)
    xd = OCTEN_F64 if getattr(X, "dtype", None) == torch.float64 else OCTEN_F32
    st = _lib.octen_fit_noalloc(_ptr(X), xd, int(t), int(I), int(J), int(R), int(k0), _ptr(A),
                                _ptr(B), _ptr(C), stream, ctypes.cast(out, _vp))
    return st, (out[0], out[1])


def octen_health(h):
    bits = ctypes.c_int32(0)
    st = _lib.octen_health(h, ctypes.cast(ctypes.byref(bits), _vp))
    return st, bits.value


def octen_cp_als_replicas(h, max_iters, tol, init_mode, init=None, iters_done=None):
    return _lib.octen_cp_als_replicas(h, int(max_iters), float(tol), int(init_mode), _ptr(init),
                                      iters_done)


def octen_recover_factors(h, A, B, C, c_capacity, K_out=None):
    return _lib.octen_recover_factors(h, _ptr(A), _ptr(B), _ptr(C), int(c_capacity), K_out)


def octen_fit(h, X, t, k0, A, B, C, out):
    return _lib.octen_fit(h, _ptr(X), int(t), int(k0), _ptr(A), _ptr(B), _ptr(C), out)


def octen_fit_coo(h, nnz, k, i, j, v, k0, A, B, C, kc, out):
    return _lib.octen_fit_coo(h, int(nnz), _ptr(k), _ptr(i), _ptr(j), _ptr(v), int(k0), _ptr(A),
                              _ptr(B), _ptr(C), int(kc), out)


def octen_get_state(h, what, dst, nbytes):
    return _lib.octen_get_state(h, int(what), _ptr(dst), int(nbytes))


def octen_check_identifiable(cfg, K, t):
    bits = ctypes.c_int32(0)
    pmin = ctypes.c_double(0.0)
    st = _lib.octen_check_identifiable(ctypes.byref(cfg), int(K), int(t),
                                       ctypes.cast(ctypes.byref(bits), _vp),
                                       ctypes.cast(ctypes.byref(pmin), _vp))
    return st, bits.value, pmin.value


OCTEN_TIMING_RING = 256


def octen_stage_times(h, stage, n=OCTEN_TIMING_RING):
    buf = (ctypes.c_double * n)()
    cnt = ctypes.c_int32(0)
    st = _lib.octen_stage_times(h, int(stage), ctypes.cast(buf, _vp), int(n),
                                ctypes.cast(ctypes.byref(cnt), _vp))
    return st, list(buf[:cnt.value])


def octen_destroy(h):
    return _lib.octen_destroy(h)


def octen_status_str(st):
    return _lib.octen_status_str(int(st)).decode()


def octen_last_error(h):
    return _lib.octen_last_error(h).decode()


def octen_mlp_param_count(n_in, n_hidden, n_out):
    return int(_lib.octen_mlp_param_count(int(n_in), int(n_hidden), int(n_out)))


def octen_mlp_create(n_in, n_hidden, n_out, params, stream=None):
    m = _vp()
    st = _lib.octen_mlp_create(int(n_in), int(n_hidden), int(n_out), _ptr(params), stream,
                               ctypes.byref(m))
    return st, m


def octen_mlp_destroy(m):
    return _lib.octen_mlp_destroy(m)


def octen_mlp_last_error(m):
    return _lib.octen_mlp_last_error(m).decode()


def octen_mlp_forward(m, X, n, Y):
    return _lib.octen_mlp_forward(m, _ptr(X), int(n), _ptr(Y))


def octen_mlp_gradients(m, X, T, n, grads, loss_host=None):
    return _lib.octen_mlp_gradients(m, _ptr(X), _ptr(T), int(n), _ptr(grads), loss_host)


def octen_mlp_adam(m, grads, lr):
    return _lib.octen_mlp_adam(m, _ptr(grads), float(lr))


def octen_mlp_train_step(m, X, T, n, lr, loss_host=None):
    return _lib.octen_mlp_train_step(m, _ptr(X), _ptr(T), int(n), float(lr), loss_host)


def octen_mlp_last_activations(m, n, H1, H2):
    return _lib.octen_mlp_last_activations(m, int(n), _ptr(H1), _ptr(H2))


def octen_mlp_get_params(m, dst):
    return _lib.octen_mlp_get_params(m, _ptr(dst))


def octen_autotune(h, X, t, choice=None):
    return _lib.octen_autotune(h, _ptr(X), int(t), choice)


def octen_compress_variant(h, variant):
    return _lib.octen_compress_variant(h, int(variant))


def octen_autotune_als(h, sweeps, choice=None):
    return _lib.octen_autotune_als(h, int(sweeps), choice)


def octen_group_create(handles):
    arr = (_vp * len(handles))(*[h.value if isinstance(h, _vp) else h for h in handles])
    g = _vp()
    st = _lib.octen_group_create(ctypes.cast(arr, _vp), len(handles), ctypes.byref(g))
    return st, g


def octen_group_step(g, descs, max_iters, tol, init_mode=OCTEN_INIT_PREV, replayed=None):
    arr = (octen_batch_desc * len(descs))(*descs)
    return _lib.octen_group_step(g, ctypes.cast(arr, _vp), int(max_iters), float(tol),
                                 int(init_mode), replayed)


def octen_group_recover(g, As, Bs, Cs, caps):
    n = len(As)
    return _lib.octen_group_recover(g, _ptr_array(As), _ptr_array(Bs), _ptr_array(Cs),
                                    ctypes.cast((ctypes.c_int64 * n)(*caps), _vp))


def octen_group_als_launches(g, out):
    return _lib.octen_group_als_launches(g, out)


def octen_group_destroy(g):
    return _lib.octen_group_destroy(g)


def octen_group_last_error(g):
    return _lib.octen_group_last_error(g).decode()


class Group:
    """One update step of many handles as one captured HIP graph."""

    def __init__(self, engines):
        self.engines = list(engines)
        st, g = octen_group_create([e.h for e in self.engines])
        if st != OCTEN_OK:
            raise OctenError(st, "octen_group_create")
        self.g = g

    def step(self, batches, max_iters, tol=0.0, learned=False):
        """batches: list of (X, W) device tensors (same objects each round
        for replay).  Returns True when the captured graph was replayed."""
        descs = [octen_batch_desc(X.data_ptr(), X.shape[0], W.data_ptr(), None)
                 for X, W in batches]
        rep = ctypes.c_int32(0)
        st = octen_group_step(self.g, descs, max_iters, tol,
                              OCTEN_INIT_LEARNED if learned else OCTEN_INIT_PREV,
                              ctypes.cast(ctypes.byref(rep), _vp))
        if st != OCTEN_OK:
            raise OctenError(st, "octen_group_step", octen_group_last_error(self.g))
        for e, (X, _) in zip(self.engines, batches):
            e._pend += int(X.shape[0])
        return bool(rep.value)

    def recover(self, outs):
        """Recovery of every handle after a step, the handles concurrently:
        outs is a list of (A, B, C) device tensors, one per handle.  On an
        error the handles before the one the message names have recovered;
        the host row counts are then left as they were for all."""
        st = octen_group_recover(self.g, [A for A, _, _ in outs], [B for _, B, _ in outs],
                                 [C for _, _, C in outs], [C.shape[0] for _, _, C in outs])
        if st != OCTEN_OK:
            raise OctenError(st, "octen_group_recover", octen_group_last_error(self.g))
        for e in self.engines:
            e.K += e._pend
            e._pend = 0

    def als_launches(self):
        """Cooperative ALS launches in the graph of the latest captured step."""
        n = ctypes.c_int32(0)
        st = octen_group_als_launches(self.g, ctypes.cast(ctypes.byref(n), _vp))
        if st != OCTEN_OK:
            raise OctenError(st, "octen_group_als_launches", octen_group_last_error(self.g))
        return int(n.value)

    def close(self):
        if getattr(self, "g", None):
            octen_group_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def octen_warmstart_set(h, m, G, D):
    return _lib.octen_warmstart_set(h, m, _ptr(G), int(D))


def octen_warmstart_features(h, X):
    return _lib.octen_warmstart_features(h, _ptr(X))


def octen_warmstart_targets(h, T):
    return _lib.octen_warmstart_targets(h, _ptr(T))


class Mlp:
    """The warm-start network: n_in -> n_hidden -> n_hidden -> n_out with a
    residual on the first n_out inputs.  params: torch float32 device tensor
    in the layout of octen_mlp_param_count."""

    def __init__(self, n_in, n_hidden, n_out, params, stream=None):
        import torch
        self.torch = torch
        self.n_in, self.n_hidden, self.n_out = int(n_in), int(n_hidden), int(n_out)
        self.nparam = octen_mlp_param_count(n_in, n_hidden, n_out)
        if params.numel() != self.nparam or params.dtype != torch.float32:
            raise ValueError(f"params must be {self.nparam} float32 values")
        if stream is None:
            stream = torch.cuda.current_stream()
        st, m = octen_mlp_create(n_in, n_hidden, n_out, params, stream.cuda_stream)
        if st != OCTEN_OK:
            raise OctenError(st, "octen_mlp_create")
        self.m = m

    def _check(self, st, where):
        if st != OCTEN_OK:
            raise OctenError(st, where, octen_mlp_last_error(self.m))

    def close(self):
        if getattr(self, "m", None):
            octen_mlp_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, X):
        Y = self.torch.empty((X.shape[0], self.n_out), dtype=self.torch.float32, device=X.device)
        self._check(octen_mlp_forward(self.m, X, X.shape[0], Y), "octen_mlp_forward")
        return Y

    def gradients(self, X, T):
        g = self.torch.empty(self.nparam, dtype=self.torch.float32, device=X.device)
        loss = ctypes.c_double(0.0)
        self._check(octen_mlp_gradients(self.m, X, T, X.shape[0], g,
                                        ctypes.cast(ctypes.byref(loss), _vp)),
                    "octen_mlp_gradients")
        return g, loss.value

    def adam(self, grads, lr):
        self._check(octen_mlp_adam(self.m, grads, lr), "octen_mlp_adam")

    def train_step(self, X, T, lr, want_loss=True):
        loss = ctypes.c_double(0.0)
        self._check(octen_mlp_train_step(self.m, X, T, X.shape[0], lr,
                                         ctypes.cast(ctypes.byref(loss), _vp) if want_loss else None),
                    "octen_mlp_train_step")
        return loss.value if want_loss else None

    def last_activations(self, n):
        H1 = self.torch.empty((n, self.n_hidden), dtype=self.torch.float32, device="cuda")
        H2 = self.torch.empty_like(H1)
        self._check(octen_mlp_last_activations(self.m, n, H1, H2), "octen_mlp_last_activations")
        return H1, H2

    def params(self):
        out = self.torch.empty(self.nparam, dtype=self.torch.float32, device="cuda")
        self._check(octen_mlp_get_params(self.m, out), "octen_mlp_get_params")
        return out


# ---------------------------------------------------------------------------
# Handle wrapper raising on errors; tensors come from torch (device memory).
# ---------------------------------------------------------------------------

class Octen:
    """One online CP stream on one GPU.  U, V: torch float64 device tensors
    [I][M1] and [J][M1]."""

    def __init__(self, I, J, R, P, Q, S, U, V, x_dtype="f64", compress_dtype="f64",
                 als_dtype="f64", flags=0, stream=None):
        import torch
        self.torch = torch
        self.cfg = make_config(I, J, R, P, Q, S, x_dtype, compress_dtype, als_dtype, flags)
        self.I, self.J, self.R, self.P, self.Q, self.S = int(I), int(J), int(R), int(P), int(Q), int(S)
        self.M1 = self.S + self.P * (self.Q - self.S)
        self.acc_dtype = torch.float64 if compress_dtype == "f64" else torch.float32
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        st, h = octen_init(self.cfg, U, V, stream.cuda_stream)
        if st != OCTEN_OK:
            raise OctenError(st, "octen_init")
        self.h = h
        self.K = 0
        self._tz = 0
        self._pend = 0

    def _check(self, st, where):
        if st != OCTEN_OK:
            raise OctenError(st, where, octen_last_error(self.h))

    def close(self):
        if getattr(self, "h", None):
            octen_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def compress_batch(self, X, W, slice_scale=None):
        self._check(octen_compress_batch(self.h, X, X.shape[0], W, slice_scale), "octen_compress_batch")
        self._tz = int(X.shape[0])

    def compress_batch_async(self, X, W, slice_scale=None):
        """Compression of the next batch on the handle's second stream,
        overlapping the ALS and recovery enqueued after it (call after
        update_replicas of the previous batch)."""
        self._check(octen_compress_batch_async(self.h, X, X.shape[0], W, slice_scale),
                    "octen_compress_batch_async")
        self._tz = int(X.shape[0])

    def compress_batch_coo(self, k, i, j, v, t, W):
        self._check(octen_compress_batch_coo(self.h, v.numel(), k, i, j, v, t, W),
                    "octen_compress_batch_coo")
        self._tz = int(t)

    def update_replicas(self):
        self._check(octen_update_replicas(self.h), "octen_update_replicas")
        self._pend += self._tz
        self._tz = 0

    def health(self):
        """(status, bits) of octen_health: waits, reports and clears the
        conditions recorded on the device since the last report."""
        return octen_health(self.h)

    def cp_als_replicas(self, iters, tol=0.0, init=None, want_iters=False, learned=False):
        mode = OCTEN_INIT_GIVEN if init is not None else (
            OCTEN_INIT_LEARNED if learned else OCTEN_INIT_PREV)
        buf = (ctypes.c_int32 * self.P)() if want_iters else None
        self._check(octen_cp_als_replicas(self.h, iters, tol, mode, init,
                                          ctypes.cast(buf, _vp) if buf is not None else None),
                    "octen_cp_als_replicas")
        return np.array(buf[:], dtype=np.int32) if buf is not None else None

    def recover_factors(self, A, B, C):
        K = ctypes.c_int64(0)
        st = octen_recover_factors(self.h, A, B, C, C.shape[0], ctypes.cast(ctypes.byref(K), _vp))
        if st in (OCTEN_OK, OCTEN_ERR_NUMERIC):   # the factors were written either way
            self.K = K.value
            self._pend = 0
        self._check(st, "octen_recover_factors")
        return self.K

    def recover_factors_async(self, A, B, C):
        """Same without waiting for the stream (K tracked on the host)."""
        self._check(octen_recover_factors(self.h, A, B, C, C.shape[0], None), "octen_recover_factors")
        self.K += self._pend
        self._pend = 0
        return self.K

    def fit_terms(self, X, k0, A, B, C, acc=None):
        out = (ctypes.c_double * 2)(*(acc if acc is not None else (0.0, 0.0)))
        self._check(octen_fit(self.h, X, X.shape[0], k0, A, B, C, ctypes.cast(out, _vp)), "octen_fit")
        return out[0], out[1]

    def fit_coo_terms(self, k, i, j, v, k0, A, B, C, kc, acc=None):
        """(sum v^2, sum v * Xh, Gram term) for the given nonzeros; the first
        two are added to acc, the third is over the rows [0, kc) of C."""
        a = acc if acc is not None else (0.0, 0.0, 0.0)
        out = (ctypes.c_double * 3)(*a)
        self._check(octen_fit_coo(self.h, v.numel(), k, i, j, v, k0, A, B, C, kc,
                                  ctypes.cast(out, _vp)), "octen_fit_coo")
        return out[0], out[1], out[2]

    def autotune(self, X):
        ch = ctypes.c_int32(0)
        self._check(octen_autotune(self.h, X, X.shape[0], ctypes.cast(ctypes.byref(ch), _vp)),
                    "octen_autotune")
        return ch.value

    def compress_variant(self, variant):
        self._check(octen_compress_variant(self.h, int(variant)), "octen_compress_variant")

    def autotune_als(self, sweeps=10):
        ch = ctypes.c_int32(0)
        self._check(octen_autotune_als(self.h, sweeps, ctypes.cast(ctypes.byref(ch), _vp)),
                    "octen_autotune_als")
        return ch.value

    def warmstart_set(self, mlp, G, D):
        self._check(octen_warmstart_set(self.h, mlp.m if mlp is not None else None, G, D),
                    "octen_warmstart_set")
        self._ws_D = int(D)

    def warmstart_features(self):
        torch = self.torch
        X = torch.empty((self.P * self.R, 4 * self.Q + self._ws_D), dtype=torch.float32,
                        device="cuda")
        self._check(octen_warmstart_features(self.h, X), "octen_warmstart_features")
        return X

    def warmstart_targets(self):
        torch = self.torch
        T = torch.empty((self.P * self.R, 3 * self.Q), dtype=torch.float32, device="cuda")
        self._check(octen_warmstart_targets(self.h, T), "octen_warmstart_targets")
        return T

    def coo_segments(self):
        """Bookkeeping of the last sparse batch: (seg_start, seg_row, slice_seg)
        as int32 device tensors."""
        torch = self.torch
        sizes = self.state(OCTEN_STATE_COO_SIZES).cpu()
        nseg, t = int(sizes[0]), int(sizes[1])
        out = []
        for what, n in ((OCTEN_STATE_COO_SEG_START, nseg + 1), (OCTEN_STATE_COO_SEG_ROW, nseg),
                        (OCTEN_STATE_COO_SLICE_SEG, t + 1)):
            buf = torch.empty((max(n, 1),), dtype=torch.int32, device="cuda")
            self._check(octen_get_state(self.h, what, buf, buf.numel() * 4), "octen_get_state")
            out.append(buf[:n])
        return tuple(out)

    def stage_ms(self, stage, n=OCTEN_TIMING_RING):
        """Durations (ms) of the last n runs of a stage, oldest first."""
        st, ms = octen_stage_times(self.h, stage, n)
        self._check(st, "octen_stage_times")
        return ms

    def state(self, what):
        torch = self.torch
        P, Q, R, M1 = self.P, self.Q, self.R, self.M1
        dev = "cuda"
        shapes = {
            OCTEN_STATE_Y: ((P, Q, Q, Q), self.acc_dtype),
            OCTEN_STATE_Z: ((P, Q, Q, Q), self.acc_dtype),
            OCTEN_STATE_FACTORS: ((P, 3, Q, R), torch.float64),
            OCTEN_STATE_LAMBDA: ((P, R), torch.float64),
            OCTEN_STATE_PERM: ((P, R), torch.int32),
            OCTEN_STATE_ALIGNED: ((P, 3, Q, R), torch.float64),
            OCTEN_STATE_RHS: ((3, M1, R), torch.float64),
            OCTEN_STATE_H: ((M1, R), torch.float64),
            OCTEN_STATE_TPERM: ((R,), torch.int32),
            OCTEN_STATE_ITERS: ((P,), torch.int32),
            OCTEN_STATE_MARGIN: ((P,), torch.float64),
            OCTEN_STATE_FLAGS: ((P,), torch.int32),
            OCTEN_STATE_COO_SIZES: ((2,), torch.int32),
            OCTEN_STATE_WARM_KEEP: ((P,), torch.int32),
            OCTEN_STATE_WARM_FITS: ((P, 2), torch.float64),
        }
        shape, dt = shapes[what]
        out = torch.empty(shape, dtype=dt, device=dev)
        self._check(octen_get_state(self.h, what, out, out.numel() * out.element_size()),
                    "octen_get_state")
        return out


# ------------------------------------------------------------------ N-mode ---

def make_nm_config(dims, R, P, Q, S):
    cfg = octen_nm_config()
    cfg.abi_version = OCTEN_ABI_VERSION
    cfg.N = len(dims) + 1
    cfg.R, cfg.P, cfg.Q, cfg.S = int(R), int(P), int(Q), int(S)
    for n, d in enumerate(dims[:OCTEN_NM_MAX_MODES - 1]):
        cfg.dims[n] = int(d)
    return cfg


def _ptr_array(tensors):
    """Host array of device pointers (None stays NULL)."""
    arr = (_vp * max(len(tensors), 1))(*[_ptr(x) for x in tensors])
    return arr


def octen_nm_init(cfg, Us, stream=None):
    h = _vp()
    arr = _ptr_array(Us) if Us is not None else None
    st = _lib.octen_nm_init(ctypes.byref(cfg), ctypes.cast(arr, _vp) if arr is not None else None,
                            stream, ctypes.byref(h))
    return st, h


def octen_nm_compress_batch(h, X, t, W):
    return _lib.octen_nm_compress_batch(h, _ptr(X), int(t), _ptr(W))


def octen_nm_update_replicas(h):
    return _lib.octen_nm_update_replicas(h)


def octen_nm_cp_als_replicas(h, iters, init_mode, init=None):
    return _lib.octen_nm_cp_als_replicas(h, int(iters), int(init_mode), _ptr(init))


def octen_nm_recover_factors(h, As, C, c_capacity, K_out=None):
    arr = _ptr_array(As)
    return _lib.octen_nm_recover_factors(h, ctypes.cast(arr, _vp), _ptr(C), int(c_capacity), K_out)


def octen_nm_fit(h, X, t, k0, As, C, out):
    arr = _ptr_array(As)
    return _lib.octen_nm_fit(h, _ptr(X), int(t), int(k0), ctypes.cast(arr, _vp), _ptr(C), out)


def octen_nm_get_state(h, what, dst, nbytes):
    return _lib.octen_nm_get_state(h, int(what), _ptr(dst), int(nbytes))


def octen_nm_destroy(h):
    return _lib.octen_nm_destroy(h)


def octen_nm_last_error(h):
    return _lib.octen_nm_last_error(h).decode()


class OctenN:
    """One online CP stream of an N-mode tensor growing in its last mode
    (N = len(dims) + 1).  Us: N - 1 torch float64 device tensors [I_n][M1]."""

    def __init__(self, dims, R, P, Q, S, Us, stream=None):
        import torch
        self.torch = torch
        self.dims = tuple(int(d) for d in dims)
        self.N = len(self.dims) + 1
        self.R, self.P, self.Q, self.S = int(R), int(P), int(Q), int(S)
        self.M1 = self.S + self.P * (self.Q - self.S)
        self.cfg = make_nm_config(self.dims, R, P, Q, S)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        st, h = octen_nm_init(self.cfg, list(Us), stream.cuda_stream)
        if st != OCTEN_OK:
            raise OctenError(st, "octen_nm_init")
        self.h = h
        self.K = 0

    def _check(self, st, where):
        if st != OCTEN_OK:
            raise OctenError(st, where, octen_nm_last_error(self.h))

    def close(self):
        if getattr(self, "h", None):
            octen_nm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def compress_batch(self, X, W):
        self._check(octen_nm_compress_batch(self.h, X, X.shape[0], W), "octen_nm_compress_batch")

    def update_replicas(self):
        self._check(octen_nm_update_replicas(self.h), "octen_nm_update_replicas")

    def cp_als_replicas(self, iters, init=None):
        mode = OCTEN_INIT_GIVEN if init is not None else OCTEN_INIT_PREV
        self._check(octen_nm_cp_als_replicas(self.h, iters, mode, init), "octen_nm_cp_als_replicas")

    def recover_factors(self, As, C):
        K = ctypes.c_int64(0)
        st = octen_nm_recover_factors(self.h, As, C, C.shape[0], ctypes.cast(ctypes.byref(K), _vp))
        if st in (OCTEN_OK, OCTEN_ERR_NUMERIC):
            self.K = K.value
        self._check(st, "octen_nm_recover_factors")
        return self.K

    def recover_factors_async(self, As, C, t):
        """Same without waiting for the stream (t: slices since the last
        recovery, K tracked on the host)."""
        self._check(octen_nm_recover_factors(self.h, As, C, C.shape[0], None),
                    "octen_nm_recover_factors")
        self.K += int(t)
        return self.K

    def fit_terms(self, X, k0, As, C, acc=None):
        out = (ctypes.c_double * 2)(*(acc if acc is not None else (0.0, 0.0)))
        self._check(octen_nm_fit(self.h, X, X.shape[0], k0, As, C, ctypes.cast(out, _vp)),
                    "octen_nm_fit")
        return out[0], out[1]

    def state(self, what):
        torch = self.torch
        P, Q, R, M1, N = self.P, self.Q, self.R, self.M1, self.N
        shapes = {
            OCTEN_STATE_Y: ((P,) + (Q,) * N, torch.float64),
            OCTEN_STATE_Z: ((P,) + (Q,) * N, torch.float64),
            OCTEN_STATE_FACTORS: ((P, N, Q, R), torch.float64),
            OCTEN_STATE_ALIGNED: ((P, N, Q, R), torch.float64),
            OCTEN_STATE_LAMBDA: ((P, R), torch.float64),
            OCTEN_STATE_PERM: ((P, R), torch.int32),
            OCTEN_STATE_RHS: ((N, M1, R), torch.float64),
            OCTEN_STATE_H: ((M1, R), torch.float64),
            OCTEN_STATE_TPERM: ((R,), torch.int32),
            OCTEN_STATE_MARGIN: ((P,), torch.float64),
            OCTEN_STATE_FLAGS: ((P,), torch.int32),
        }
        shape, dt = shapes[what]
        out = torch.empty(shape, dtype=dt, device="cuda")
        self._check(octen_nm_get_state(self.h, what, out, out.numel() * out.element_size()),
                    "octen_nm_get_state")
        return out
