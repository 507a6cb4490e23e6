"""Shared drivers for parity tests: run one synthetic stream through the
oracle and through the HIP library (via the C ABI) on the same inputs."""
import dataclasses
import sys

import numpy as np

from paper_1807_01350_amd import synth


def rel(a, b):
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@dataclasses.dataclass
class Case:
    name: str
    I: int
    J: int
    R: int
    P: int
    Q: int
    S: int
    batches: tuple          # depths, first one is the initial summary
    iters: int = 50
    sigma: float = 0.01
    config_id: int = 1
    noiseless: bool = False

    @property
    def M1(self):
        return self.S + self.P * (self.Q - self.S)

    @property
    def K(self):
        return int(sum(self.batches))


def make_inputs(c: Case, x_dtype=np.float64):
    A, B, C, X = synth.dense_stream(c.I, c.J, c.K, c.R, c.sigma, c.config_id,
                                    dtype=x_dtype, noiseless=c.noiseless)
    U, V = synth.compression_UV(c.I, c.J, c.P, c.Q, c.S, c.config_id)
    Ws = [synth.temporal_W(t, c.M1, c.config_id, b) for b, t in enumerate(c.batches)]
    init = synth.als_init(c.P, c.Q, c.R, c.config_id)
    return X, U, V, Ws, init


def run_oracle(c: Case, X, U, V, Ws, init, tol=0.0):
    from oracle import OctenOracle, fit_dense
    o = OctenOracle(c.I, c.J, c.R, c.P, c.Q, c.S, U, V)
    out = []
    k0 = 0
    for b, t in enumerate(c.batches):
        o.compress_batch(X[k0:k0 + t], Ws[b])
        Z = o.Z.copy()
        o.update_replicas()
        o.cp_als_replicas(c.iters, tol=tol, init=init if b == 0 else None)
        A, B, C = o.recover_factors()
        fit = fit_dense(X[:o.K], A, B, C)[0]
        out.append(dict(Z=Z, Y=o.Y.copy(), F=o.F.copy(), lam=o.lam.copy(), iters=o.iters_done.copy(),
                        perm=o.last["perm"].copy(), margins=o.last["margins"].copy(),
                        aligned=o.last["aligned"].copy(), rhs=np.stack(o.last["rhs"]),
                        A=A.copy(), B=B.copy(), C=C.copy(), fit=fit, tperm=o.last["tperm"].copy(),
                        H=o.H.copy(), K=o.K))
        k0 += t
    return out


def run_gpu(c: Case, X, U, V, Ws, init, compress_dtype="f64", x_dtype="f64", tol=0.0, flags=0,
            log=None, als_dtype="f64"):
    import torch
    from paper_1807_01350_amd import octen as oc
    dev = "cuda"
    tX = torch.from_numpy(np.ascontiguousarray(X)).to(dev)
    tU = torch.from_numpy(U).to(dev)
    tV = torch.from_numpy(V).to(dev)
    tinit = torch.from_numpy(init).to(dev)
    eng = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, tU, tV, x_dtype=x_dtype,
                   compress_dtype=compress_dtype, als_dtype=als_dtype, flags=flags)
    A = torch.empty((c.I, c.R), dtype=torch.float64, device=dev)
    B = torch.empty((c.J, c.R), dtype=torch.float64, device=dev)
    C = torch.empty((c.K, c.R), dtype=torch.float64, device=dev)
    out = []
    k0 = 0
    for b, t in enumerate(c.batches):
        if log:
            print(f"[{c.name}] gpu batch {b} k0={k0} t={t}", file=sys.stderr, flush=True)
        tW = torch.from_numpy(Ws[b]).to(dev)
        eng.compress_batch(tX[k0:k0 + t], tW)
        Z = eng.state(oc.OCTEN_STATE_Z).cpu().numpy()
        eng.update_replicas()
        iters = eng.cp_als_replicas(c.iters, tol=tol, init=tinit if b == 0 else None, want_iters=True)
        K = eng.recover_factors(A, B, C)
        sse, nx = eng.fit_terms(tX[:K], 0, A, B, C)
        torch.cuda.synchronize()
        out.append(dict(Z=Z, Y=eng.state(oc.OCTEN_STATE_Y).cpu().numpy(),
                        F=eng.state(oc.OCTEN_STATE_FACTORS).cpu().numpy(),
                        lam=eng.state(oc.OCTEN_STATE_LAMBDA).cpu().numpy(), iters=iters,
                        perm=eng.state(oc.OCTEN_STATE_PERM).cpu().numpy(),
                        margins=eng.state(oc.OCTEN_STATE_MARGIN).cpu().numpy(),
                        aligned=eng.state(oc.OCTEN_STATE_ALIGNED).cpu().numpy(),
                        rhs=eng.state(oc.OCTEN_STATE_RHS).cpu().numpy(),
                        A=A.cpu().numpy().copy(), B=B.cpu().numpy().copy(),
                        C=C[:K].cpu().numpy().copy(), fit=1 - np.sqrt(sse / nx),
                        tperm=eng.state(oc.OCTEN_STATE_TPERM).cpu().numpy(),
                        H=eng.state(oc.OCTEN_STATE_H).cpu().numpy(),
                        flags=eng.state(oc.OCTEN_STATE_FLAGS).cpu().numpy(), K=K))
        k0 += t
    eng.close()
    return out
