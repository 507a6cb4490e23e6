"""Benchmark of the online compressed CP update on one MI355X.

Default workload: the dense 1000 x 1000 stream with rank-10 ground truth
(U[0,1] factors, Gaussian noise sigma = 0.01), streamed along mode 3: 500
initial slices, then batches of 50; P = 12 replicas of 60^3 with S = 3 shared
anchor rows, 50 ALS sweeps per batch, FP64 solves and recovery.  One step =
one batch through compress -> update -> ALS -> recover (the whole update).

--workload sparse: the 10^5 x 10^5 COO stream (10^5 truncated-Zipf(1.2)
coordinate draws per slice in modes 1 and 2, rank 20), 200 initial slices then
batches of 100; P = 16 replicas of 80^3, S = 3.

Synthetic data are generated on the GPU from a seeded generator (no dataset
exists for these workloads).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--form bf16|f32]
                  [--workload dense|dense50|long|sweep|sparse|batched|forms|nmode]

--workload nmode: the four-mode stream of the higher-order extension
(100 x 100 x 100 x K, rank 5; P = 10 replicas of 16^4), FP64.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "new slices/sec & compression HBM GB/s (% peak) at fit within 1e-3 of FP64 oracle"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3, "f64": 78.6}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--form", choices=("bf16x2", "bf16", "f32"), default="bf16x2")
    ap.add_argument("--als-form", choices=("f64", "bf16x2"), default="bf16x2",
                    help="arithmetic of the ALS slab contractions (bf16x2: two-term "
                         "bfloat16 operands, float32 sums; needs a narrow --form)")
    ap.add_argument("--als-one-wg", action="store_true",
                    help="batched workload: every stream's ALS as one workgroup per replica "
                         "inside its graph branch (all streams concurrently) instead of "
                         "cooperative launches after the join")
    ap.add_argument("--als-wg", choices=("few", "spread"), default="few",
                    help="batched workload: workgroups per replica of the cooperative ALS, the "
                         "fewest whose slab fits in LDS (few: more streams share a launch) or "
                         "enough to spread about 2e5 FMAs per workgroup and sweep")
    ap.add_argument("--als-device-sync", action="store_true",
                    help="dense stream: agent-scope release and acquire at every ALS replica "
                         "barrier, also when a replica's workgroups share one XCD")
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--batch", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fit", action="store_true")
    ap.add_argument("--no-gate", action="store_true",
                    help="dense stream: skip the fit gate against the FP64 oracle")
    ap.add_argument("--overlap", action="store_true",
                    help="dense stream: a second pass that overlaps the next batch's "
                         "compression with the current batch's ALS and recovery")
    ap.add_argument("--workload", choices=("dense", "dense50", "long", "sweep", "sparse",
                                           "batched", "forms", "nmode", "copy"),
                    default="dense")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--tols", default="1e-4,1e-5,1e-6",
                    help="forms workload: the replica-fit stopping tolerances, all reported")
    ap.add_argument("--train-streams", type=int, default=6)
    ap.add_argument("--streams", type=int, default=64)
    ap.add_argument("--long-I", type=int, default=100)
    ap.add_argument("--long-K", type=int, default=100_000)
    ap.add_argument("--sweep-seeds", type=int, default=5)
    return ap.parse_args()


def gen_stream(torch, I, J, K, R, sigma, seed, dev):
    """X[k] = A diag(C[k]) B^T + sigma N(0,1), f32 on the device (seeded)."""
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    A = torch.rand((I, R), generator=g, device=dev, dtype=torch.float64)
    B = torch.rand((J, R), generator=g, device=dev, dtype=torch.float64)
    C = torch.rand((K, R), generator=g, device=dev, dtype=torch.float64)
    Bt = B.t().contiguous()
    X = torch.empty((K, I, J), dtype=torch.float32, device=dev)
    ch = 25
    for k0 in range(0, K, ch):
        k1 = min(K, k0 + ch)
        blk = torch.matmul(A.unsqueeze(0) * C[k0:k1].unsqueeze(1), Bt)
        blk += sigma * torch.randn(blk.shape, generator=g, device=dev, dtype=torch.float64)
        X[k0:k1] = blk.float()
    return X


def traffic_from_profile(form, source="compress_mfma.hip", profile=None):
    """HBM bytes per launch of a kernel (by default the compression kernel of
    the given form) from the committed rocprofv3 counter summary, if it was
    taken on the current source of that kernel (one file, or several hashed
    in the order given)."""
    import hashlib
    srcs = (source,) if isinstance(source, str) else tuple(source)
    prof = os.path.join(ROOT, "profiles",
                        profile or f"compress_pipe_{form}_dense1000_counters.md")
    if not os.path.exists(prof):
        return None
    blob = b"".join(open(os.path.join(ROOT, "paper_1807_01350_amd", "csrc", f), "rb").read()
                    for f in srcs)
    h = hashlib.sha256(blob).hexdigest()[:16]
    txt = open(prof).read()
    m = re.search(r"source_sha256_16:\s*([0-9a-f]{16})", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != h:
        return None
    return float(b.group(1))


def cores_used():
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    threads = cores
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        if info:
            threads = max(int(x.get("num_threads", 1)) for x in info)
    except Exception:
        pass
    return int(threads)


def gen_coo_batches(torch, c, schedule, seed, dev):
    """Seeded on-device COO stream: per slice nnz_per_slice distinct (i, j),
    each coordinate a truncated Zipf(a) draw over its mode then a fixed
    random relabelling (drawn until a slice holds that many distinct pairs,
    then a uniform random subset of that size kept); sorted by (k, i, j); values = rank-R CP model with
    U[0,1] factors at the coordinates + sigma N(0,1).  Returns the factors and
    a list of (k, i, j, v) per batch (k relative to the batch)."""
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    f64 = torch.float64
    A = torch.rand((c.I, c.R), generator=g, device=dev, dtype=f64)
    B = torch.rand((c.J, c.R), generator=g, device=dev, dtype=f64)
    C = torch.rand((c.K, c.R), generator=g, device=dev, dtype=f64)

    def zipf_sampler(n):
        w = torch.arange(1, n + 1, device=dev, dtype=f64) ** (-c.zipf_a)
        cdf = torch.cumsum(w, 0)
        cdf /= cdf[-1].clone()
        relabel = torch.randperm(n, generator=g, device=dev)
        return lambda m: relabel[torch.searchsorted(
            cdf, torch.rand(m, generator=g, device=dev, dtype=f64), right=True).clamp_(max=n - 1)]

    draw_i, draw_j = zipf_sampler(c.I), zipf_sampler(c.J)
    out = []
    IJ = c.I * c.J
    for k0, t in schedule:
        per = c.nnz_per_slice
        # draw until every slice holds at least nnz_per_slice distinct
        # coordinates, then keep a uniformly random nnz_per_slice of them
        key = torch.empty(0, dtype=torch.int64, device=dev)
        need = torch.full((t,), per, dtype=torch.int64, device=dev)
        while True:
            extra = (2 * need).clamp_(min=0)
            kk = torch.repeat_interleave(torch.arange(t, device=dev, dtype=torch.int64), extra)
            if kk.numel() == 0:
                break
            key = torch.unique(torch.cat([key, (kk * c.I + draw_i(kk.numel())) * c.J +
                                          draw_j(kk.numel())]))
            have = torch.bincount(key // IJ, minlength=t)
            need = (per - have).clamp_(min=0)
            if int(need.sum()) == 0:
                break
        sl = key // IJ
        pri = torch.rand(key.numel(), generator=g, device=dev, dtype=f64)
        order = torch.argsort(sl.double() + pri)
        sl_o = sl[order]
        first = torch.zeros(t + 1, dtype=torch.int64, device=dev)
        first[1:] = torch.cumsum(torch.bincount(sl_o, minlength=t), 0)
        rank = torch.arange(key.numel(), device=dev) - first[sl_o]
        key = torch.sort(key[order][rank < per]).values
        del sl, pri, order, sl_o, rank
        k = key // (c.I * c.J)
        rem = key - k * (c.I * c.J)
        i = rem // c.J
        j = rem - i * c.J
        v = torch.empty(key.numel(), dtype=torch.float32, device=dev)
        for q0 in range(0, key.numel(), 1 << 22):
            q1 = min(key.numel(), q0 + (1 << 22))
            val = (A[i[q0:q1]] * B[j[q0:q1]] * C[k0 + k[q0:q1]]).sum(1)
            val += c.sigma * torch.randn(val.shape, generator=g, device=dev, dtype=f64)
            v[q0:q1] = val.float()
        out.append((k.int(), i.int(), j.int(), v))
        del key, kk, rem
    return A, B, C, out


def cpu_baseline_sparse(c, U, V, W, init, iters, batch_slices, batch):
    """The oracle, untuned, on a bounded sample of one timed sparse batch
    (device tensors k, i, j, v): compression of its first 2 slices, 5 ALS
    sweeps on all replicas, one recovery; scaled to a whole batch
    (compression x t/2, ALS x iters/5)."""
    import oracle
    ns, sweeps = 2, 5
    kd, id_, jd, vd = batch
    sel = kd < ns
    k, i, j, v = (x[sel].cpu().numpy() for x in (kd, id_, jd, vd))
    o = oracle.OctenOracle(c.I, c.J, c.R, c.P, c.Q, c.S, U, V)
    t0 = time.perf_counter()
    o.compress_batch_coo(k, i, j, v, ns, W[:ns])
    t_c = time.perf_counter() - t0
    o.update_replicas()
    t0 = time.perf_counter()
    o.cp_als_replicas(sweeps, init=init)
    t_a = time.perf_counter() - t0
    t0 = time.perf_counter()
    o.recover_factors()
    t_r = time.perf_counter() - t0
    est = t_c * batch_slices / ns + t_a * iters / sweeps + t_r
    return {"value": batch_slices / est, "unit": "slices/s", "cores": cores_used(),
            "kind": "oracle",
            "sample": f"FP64 oracle on {ns} slices ({v.size} nonzeros) of the sparse stream: "
                      f"compression {t_c:.2f} s, {sweeps} ALS sweeps on all {c.P} replicas "
                      f"{t_a:.2f} s, recovery {t_r:.2f} s; scaled to a batch of "
                      f"{batch_slices} slices and {iters} sweeps = {est:.1f} s"}


def run_sparse(args):
    import torch
    from paper_1807_01350_amd import octen as oc
    from paper_1807_01350_amd import synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    c = synth.C3
    t = 100 if args.batch == 50 else args.batch
    nsteps = args.warmup + args.steps
    sched = [(0, c.t0)] + [(c.t0 + t * b, t) for b in range(nsteps)]
    Kuse = c.t0 + t * nsteps
    assert Kuse <= c.K, "more slices than the stream holds"
    print(f"[bench] generating {len(sched)} sparse batches", file=sys.stderr, flush=True)
    Af, Bf, Cf, batches = gen_coo_batches(torch, c, sched, synth.seed_of(c.config_id, 5), dev)
    U, V = synth.compression_UV(c.I, c.J, c.P, c.Q, c.S, c.config_id)
    Ws = [synth.temporal_W(tt, c.M1, c.config_id, b) for b, (_, tt) in enumerate(sched)]
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    init = synth.als_init(c.P, c.Q, c.R, c.config_id)
    tinit = torch.from_numpy(init).to(dev)
    print("[bench] init", file=sys.stderr, flush=True)
    eng = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, torch.from_numpy(U).to(dev),
                   torch.from_numpy(V).to(dev), x_dtype="f32", compress_dtype=args.form,
                   flags=oc.OCTEN_FLAG_TIMING)
    A = torch.empty((c.I, c.R), dtype=torch.float64, device=dev)
    B = torch.empty((c.J, c.R), dtype=torch.float64, device=dev)
    C = torch.empty((Kuse, c.R), dtype=torch.float64, device=dev)

    def step(b):
        k, i, j, v = batches[b]
        eng.compress_batch_coo(k, i, j, v, sched[b][1], tW[b])
        eng.update_replicas()
        eng.cp_als_replicas(args.iters, init=tinit if b == 0 else None)
        eng.recover_factors_async(A, B, C)

    for b in range(0, args.warmup + 1):
        step(b)
    torch.cuda.synchronize()
    print("[bench] timed steps", file=sys.stderr, flush=True)
    t_start = time.perf_counter()
    for b in range(args.warmup + 1, nsteps + 1):
        step(b)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = 1e3 * elapsed / args.steps
    value = t * args.steps / elapsed

    def last(stage):
        vv = eng.stage_ms(stage, args.steps)
        return float(np.mean(vv)) if vv else None

    st = {
        "coo_index": last(oc.OCTEN_STAGE_COO_INDEX),
        "compress_main": last(oc.OCTEN_STAGE_COMPRESS_MAIN),
        "compress_mode3": last(oc.OCTEN_STAGE_COMPRESS_MODE3),
        "update": last(oc.OCTEN_STAGE_UPDATE),
        "als": last(oc.OCTEN_STAGE_ALS),
        "recover": last(oc.OCTEN_STAGE_RECOVER),
    }
    # algorithmic bytes of one launch of the gather + MFMA kernel, averaged
    # over the timed batches: (j, v) per nonzero, (start, row) per segment,
    # the distinct rows of U and V (M1 f32 each), the t x P x Q^2 output
    byts, flops, nnz_avg = [], [], []
    for b in range(args.warmup + 1, nsteps + 1):
        k, i, j, v = batches[b]
        nnz = v.numel()
        nseg = int(torch.unique(k.long() * c.I + i.long()).numel())
        di = int(torch.unique(i).numel())
        dj = int(torch.unique(j).numel())
        byts.append(nnz * 8 + nseg * 8 + (di + dj) * c.M1 * 4 + t * c.P * c.Q * c.Q * 4)
        flops.append(2.0 * nnz * c.M1 + 2.0 * nseg * c.P * c.Q * c.Q)
        nnz_avg.append(nnz)
    bytes_launch = float(np.mean(byts))
    kms = st["compress_main"]
    gbs = bytes_launch / (kms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            # both forms gather in FP32 through the same kernel
            "traffic": traffic_from_profile(None, "sparse.hip",
                                            "coo_compress_f32_sparse1e5_counters.md"),
            "kernel": "coo_compress (gather of V rows per (k, i) segment + MFMA U^T R)",
            "algorithmic_bytes_per_launch": bytes_launch,
            "algorithmic_flops_per_launch": float(np.mean(flops)),
            "nnz_per_batch": float(np.mean(nnz_avg))}

    fit = None
    if not args.no_fit:
        acc = (0.0, 0.0, 0.0)
        for b, (k0, tt) in enumerate(sched):
            k, i, j, v = batches[b]
            acc = eng.fit_coo_terms(k, i, j, v, k0, A, B, C, Kuse, acc=acc)
        nx, inner, gram = acc
        fit = 1.0 - float(np.sqrt(max(nx - 2 * inner + gram, 0.0) / nx))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_sparse(c, U, V, Ws[args.warmup + 1], init, args.iters, t,
                                  batches[args.warmup + 1])

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "slices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded on-device generator; truncated Zipf(1.2) coordinates, "
                "rank-20 U[0,1] CP values + N(0, 0.01^2))",
        "config": {"workload": f"sparse1e5_coo: I=J=100000, R=20, {c.nnz_per_slice} coordinate "
                               f"draws per slice, {c.t0} initial slices then batches of {t}; "
                               f"P=16, Q=80, S=3; {args.iters} ALS sweeps; f32 gathers with "
                               f"f32 MFMA accumulation, f64 solves",
                   "I": c.I, "J": c.J, "R": c.R, "P": c.P, "Q": c.Q, "S": c.S, "batch": t,
                   "initial_slices": c.t0, "als_iters": args.iters, "compress_dtype": args.form},
        "compression_gbs": round(gbs, 1),
        "compression_hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
        "stage_ms": {kk: (round(vv, 4) if vv is not None else None) for kk, vv in st.items()},
        "fit": fit,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    eng.close()
    print(json.dumps(out))


def batched_shapes(n, seed):
    """Per stream (I, J, t, R, P, Q): I, J ~ U{200..4000}, t ~ U{10..200},
    R ~ U{5..30}, P ~ U{4..16}, Q ~ U{20..80}; R is drawn again while R > Q."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        I, J = (int(x) for x in g.integers(200, 4001, 2))
        t = int(g.integers(10, 201))
        P = int(g.integers(4, 17))
        Q = int(g.integers(20, 81))
        R = int(g.integers(5, 31))
        while R > Q:
            R = int(g.integers(5, 31))
        out.append((I, J, t, R, P, Q))
    return out


def run_batched(args):
    """Many independent dense FP32 streams of uneven sizes: one initial batch
    per stream through its own calls (autotuned compression), then rounds in
    which all streams' compress + update + ALS run as one captured HIP graph,
    followed by the recovery of all streams (octen_group_recover: each on a
    stream of its own, concurrently).  Each round's slices are generated on the
    device before the round and are not timed."""
    import torch
    from paper_1807_01350_amd import octen as oc
    from paper_1807_01350_amd import synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    S, sigma = 3, 0.01
    rounds = args.warmup + args.steps
    shapes = batched_shapes(args.streams, synth.seed_of(4, 0))
    g = torch.Generator(device=dev)
    g.manual_seed(synth.seed_of(4, 1))
    f64 = torch.float64
    streams = []
    # the oracle's sample: the two streams of least oracle work per round
    # (its ALS, einsum contractions, dominates: P Q^3 R per sweep; its
    # compression is BLAS)
    def _work(sh):
        I, J, t, R, P, Q = sh
        return P * Q ** 3 * R * args.iters + I * J * t * (S + P * (Q - S)) / 50
    sample = set(sorted(range(len(shapes)), key=lambda q: _work(shapes[q]))[:2])
    print(f"[bench] {len(shapes)} streams: creating handles", file=sys.stderr, flush=True)
    for q, (I, J, t, R, P, Q) in enumerate(shapes):
        M1 = S + P * (Q - S)
        A = torch.rand((I, R), generator=g, device=dev, dtype=f64)
        B = torch.rand((J, R), generator=g, device=dev, dtype=f64)
        C = torch.rand(((rounds + 1) * t, R), generator=g, device=dev, dtype=f64)
        # N(0,1) compression matrices on the bfloat16 grid (as synth draws them)
        U = torch.randn((I, M1), generator=g, device=dev, dtype=f64).float().bfloat16().double()
        V = torch.randn((J, M1), generator=g, device=dev, dtype=f64).float().bfloat16().double()
        eng = oc.Octen(I, J, R, P, Q, S, U, V, x_dtype="f32", compress_dtype=args.form,
                       flags=(oc.OCTEN_FLAG_ALS_ONE_WG if args.als_one_wg else 0)
                       | (oc.OCTEN_FLAG_ALS_FEW_WG if args.als_wg == "few" else 0))
        X = torch.empty((t, I, J), dtype=torch.float32, device=dev)
        W = torch.empty((t, M1), dtype=f64, device=dev)
        init = torch.randn((P, 3, Q, R), generator=g, device=dev, dtype=f64)
        outs = (torch.empty((I, R), dtype=f64, device=dev), torch.empty((J, R), dtype=f64, device=dev),
                torch.empty(((rounds + 1) * t, R), dtype=f64, device=dev))
        streams.append(dict(shape=(I, J, t, R, P, Q), A=A, B=B, C=C, eng=eng, X=X, W=W,
                            init=init, outs=outs, M1=M1, UV=(U, V) if q in sample else None))
        del U, V

    def fill(st, r):
        I, J, t, R, P, Q = st["shape"]
        Bt = st["B"].t().contiguous()
        for k0 in range(0, t, 8):
            k1 = min(t, k0 + 8)
            blk = torch.matmul(st["A"].unsqueeze(0) * st["C"][r * t + k0:r * t + k1].unsqueeze(1), Bt)
            blk += sigma * torch.randn(blk.shape, generator=g, device=dev, dtype=f64)
            st["X"][k0:k1] = blk.float()
        st["W"].normal_(generator=g)

    print("[bench] initial batches and autotuning", file=sys.stderr, flush=True)
    choices = []
    for st in streams:
        fill(st, 0)
        e = st["eng"]
        choices.append(e.autotune(st["X"]))
        e.compress_batch(st["X"], st["W"])
        e.update_replicas()
        e.cp_als_replicas(args.iters, init=st["init"])
        e.recover_factors_async(*st["outs"])
    torch.cuda.synchronize()
    group = oc.Group([st["eng"] for st in streams])
    batches = [(st["X"], st["W"]) for st in streams]
    times, replays = [], []
    slices = sum(st["shape"][2] for st in streams)
    for r in range(1, rounds + 1):
        for st in streams:
            fill(st, r)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        replays.append(group.step(batches, args.iters))
        group.recover([st["outs"] for st in streams])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        print(f"[bench] round {r}: {times[-1] * 1e3:.1f} ms, replayed {replays[-1]}",
              file=sys.stderr, flush=True)
    timed = times[args.warmup:]
    elapsed = float(sum(timed))
    value = slices * len(timed) / elapsed
    xbytes = sum(4.0 * I * J * t for (I, J, t, R, P, Q) in (st["shape"] for st in streams))
    gbs = xbytes / (elapsed / len(timed)) / 1e9
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "slices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / len(timed), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.form,
        "data": "synthetic (seeded on-device generator per stream; U[0,1] CP models + N(0, 0.01^2))",
        "config": {"workload": f"batched{len(streams)}: {len(streams)} dense FP32 streams, I,J in "
                               f"[200,4000], t in [10,200], R in [5,30], P in [4,16], Q in [20,80], "
                               f"S=3; one step = one round of all streams (compress + update + "
                               f"{args.iters} ALS sweeps in one captured graph, then the recovery of "
                               f"all streams, each on a stream of its own)",
                   "streams": len(streams), "slices_per_round": slices,
                   "x_bytes_per_round": xbytes, "als_iters": args.iters,
                   "compress_dtype": args.form,
                   "als": "one workgroup per replica in each stream's branch" if args.als_one_wg
                          else ("cooperative after the join, streams of the same ALS kernel "
                                "sharing launches; workgroups per replica: "
                                + ("fewest fitting the slab in LDS" if args.als_wg == "few"
                                   else "about 2e5 FMAs each per sweep")),
                   "als_launches": group.als_launches()},
        "round_ms": [round(1e3 * x, 3) for x in times],
        "replayed": replays,
        "x_stream_gbs": round(gbs, 1),
        "autotune_choices": choices,
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole round (X bytes streamed / round time)"},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        # the oracle on a sample: the two cheapest streams, an initial batch
        # (untimed) then one update round (timed: compress, update, ALS,
        # recover), on batches drawn the same way as the timed rounds
        import oracle
        tot_s, tot_n, desc = 0.0, 0, []
        for q in sorted(sample):
            st = streams[q]
            I, J, t, R, P, Q = st["shape"]
            U, V = (x.cpu().numpy() for x in st["UV"])
            o = oracle.OctenOracle(I, J, R, P, Q, S, U, V)
            fill(st, 0)
            o.compress_batch(st["X"].double().cpu().numpy(), st["W"].cpu().numpy())
            o.update_replicas()
            o.cp_als_replicas(args.iters, init=st["init"].cpu().numpy())
            o.recover_factors()
            fill(st, 1)
            Xh, Wh = st["X"].double().cpu().numpy(), st["W"].cpu().numpy()
            t1 = time.perf_counter()
            o.compress_batch(Xh, Wh)
            o.update_replicas()
            o.cp_als_replicas(args.iters)
            o.recover_factors()
            tot_s += time.perf_counter() - t1
            tot_n += t
            desc.append(f"I={I} J={J} t={t} R={R} P={P} Q={Q}")
        out["cpu_baseline"] = {"value": round(tot_n / tot_s, 3), "unit": "slices/s",
                               "cores": cores_used(), "kind": "oracle",
                               "sample": f"one update round of the two streams of least oracle work ("
                                         f"{'; '.join(desc)}) through the FP64 oracle, "
                                         f"{tot_s:.2f} s; the device rounds stream all "
                                         f"{len(streams)}"}
    group.close()
    for st in streams:
        st["eng"].close()
    print(json.dumps(out))


def run_forms(args):
    """The dense 1000 x 1000 stream in two forms with the same ALS stopping
    rule (replica fit change below tol, at most --iters sweeps), for every
    tol in --tols: the plain FP32 form (FP32 compression, ALS from the
    previous factors, one call per step) and the two-term BF16 + graph +
    learned-warm-start form (the step captured once as a HIP graph and
    replayed, ALS from the judged network start); then fixed budgets of 5,
    10 and 20 sweeps from the plain and from the network start (FP32
    compression in both).  The network (4Q + 32 -> 256 -> 256 -> 3Q) is first
    trained, untimed, on pairs from other streams of the same shape."""
    import torch
    from paper_1807_01350_amd import octen as oc
    from paper_1807_01350_amd import synth
    from paper_1807_01350_amd import warmstart as ws

    dev = "cuda:0"
    torch.cuda.set_device(0)
    c = synth.C2
    t = args.batch
    D = 32
    G = torch.from_numpy(synth.sketch_matrix(D, c.Q, 900)).to(dev)
    n_in, n_out = 4 * c.Q + D, 3 * c.Q
    t_train0, n_train_b = 200, 8
    feats, targs = [], []
    for sid in range(args.train_streams):
        cid = 200 + sid
        Xs = gen_stream(torch, c.I, c.J, t_train0 + n_train_b * t, c.R, c.sigma,
                        synth.seed_of(cid, 1), dev)
        U, V = synth.compression_UV(c.I, c.J, c.P, c.Q, c.S, cid)
        e = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, torch.from_numpy(U).to(dev),
                     torch.from_numpy(V).to(dev), x_dtype="f32", compress_dtype="f32")
        e.warmstart_set(None, G, D)
        bs = [Xs[:t_train0]] + [Xs[t_train0 + b * t:t_train0 + (b + 1) * t] for b in range(n_train_b)]
        Ws = [torch.from_numpy(synth.temporal_W(x.shape[0], c.M1, cid, b)).to(dev)
              for b, x in enumerate(bs)]
        init = torch.from_numpy(synth.als_init(c.P, c.Q, c.R, cid)).to(dev)
        f, tt = ws.collect_pairs(e, bs, Ws, init, tol=1e-8, max_iters=300)
        feats += f
        targs += tt
        e.close()
        del Xs
        print(f"[bench] training stream {sid}: {sum(x.shape[0] for x in f)} pairs", file=sys.stderr,
              flush=True)
    Xtr, Ttr = torch.cat(feats), torch.cat(targs)
    net = oc.Mlp(n_in, 256, n_out, torch.from_numpy(synth.mlp_params(n_in, 256, n_out, 901)).to(dev))
    loss0 = ws.evaluate_loss(net, Xtr, Ttr)
    ws.train(net, Xtr, Ttr, 1500, batch=512, lr=1e-3, lr_final=1e-4)
    loss1 = ws.evaluate_loss(net, Xtr, Ttr)
    print(f"[bench] network trained on {Xtr.shape[0]} pairs: loss {loss0:.4g} -> {loss1:.4g}",
          file=sys.stderr, flush=True)

    nsteps = args.warmup + args.steps
    K = c.t0 + t * nsteps
    X = gen_stream(torch, c.I, c.J, K, c.R, c.sigma, synth.seed_of(c.config_id, 1), dev)
    U, V = synth.compression_UV(c.I, c.J, c.P, c.Q, c.S, c.config_id)
    Ws = [torch.from_numpy(synth.temporal_W(c.t0 if b == 0 else t, c.M1, c.config_id, b)).to(dev)
          for b in range(nsteps + 1)]
    init = torch.from_numpy(synth.als_init(c.P, c.Q, c.R, c.config_id)).to(dev)

    def run_stream(form, max_iters, tol, learned, graph):
        """The measured stream through one form; per-batch wall time (timed
        batches only), sweeps per replica, share of replicas whose network
        start was kept, and the fit over the whole stream."""
        bf = form == "bf16x2"
        e = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, torch.from_numpy(U).to(dev),
                     torch.from_numpy(V).to(dev), x_dtype="f32", compress_dtype=form)
        A = torch.empty((c.I, c.R), dtype=torch.float64, device=dev)
        B = torch.empty((c.J, c.R), dtype=torch.float64, device=dev)
        C = torch.empty((K, c.R), dtype=torch.float64, device=dev)
        e.compress_batch(X[:c.t0], Ws[0])
        e.update_replicas()
        e.cp_als_replicas(args.iters, init=init)
        e.recover_factors_async(A, B, C)
        if learned:
            e.warmstart_set(net, G, D)
        group = None
        if graph:
            group = oc.Group([e])
            xb = torch.empty((t, c.I, c.J), dtype=torch.float32, device=dev)
            wb = torch.empty((t, c.M1), dtype=torch.float64, device=dev)
        times, sweeps, kept = [], [], []
        k0 = c.t0
        for b in range(1, nsteps + 1):
            if graph:
                xb.copy_(X[k0:k0 + t])
                wb.copy_(Ws[b])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if graph:
                group.step([(xb, wb)], max_iters, tol, learned=learned)
            else:
                e.compress_batch(X[k0:k0 + t], Ws[b])
                e.update_replicas()
                e.cp_als_replicas(max_iters, tol=tol, learned=learned)
            e.recover_factors_async(A, B, C)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            sweeps.append(float(e.state(oc.OCTEN_STATE_ITERS).float().mean()))
            if learned:
                kept.append(float(e.state(oc.OCTEN_STATE_WARM_KEEP).float().mean()))
            k0 += t
        timed = times[args.warmup:]
        sse = nx = 0.0
        for q0 in range(0, K, 100):
            sse, nx = e.fit_terms(X[q0:min(K, q0 + 100)], q0, A, B, C, acc=(sse, nx))
        if group is not None:
            group.close()
        e.close()
        return {"slices_per_s": round(t * len(timed) / sum(timed), 2),
                "ms_per_step": round(1e3 * sum(timed) / len(timed), 4),
                "mean_sweeps_per_replica": round(float(np.mean(sweeps[args.warmup:])), 2),
                "network_start_kept": (round(float(np.mean(kept)), 3) if kept else None),
                "fallback_rate": (round(1.0 - float(np.mean(kept)), 3) if kept else None),
                "fit": 1.0 - float(np.sqrt(sse / nx))}

    tols = [float(x) for x in args.tols.split(",")]
    per_tol = {}
    for tol in tols:
        a = run_stream("f32", args.iters, tol, learned=False, graph=False)
        b = run_stream("bf16x2", args.iters, tol, learned=True, graph=True)
        per_tol[f"{tol:g}"] = {"fp32_plain": a, "bf16x2_graph_learned": b,
                               "speedup_vs_fp32_plain": round(b["slices_per_s"] / a["slices_per_s"], 3),
                               "fit_difference": b["fit"] - a["fit"]}
        print(f"[bench] tol {tol:g}: {per_tol[f'{tol:g}']}", file=sys.stderr, flush=True)
    # fixed sweep budgets from the plain and from the judged network start
    # (same FP32 compression, so only the start differs)
    budgets = {}
    for nb in (5, 10, 20):
        pl = run_stream("f32", nb, 0.0, learned=False, graph=False)
        ln = run_stream("f32", nb, 0.0, learned=True, graph=False)
        budgets[str(nb)] = {"fit_plain_start": pl["fit"], "fit_learned_start": ln["fit"],
                            "network_start_kept": ln["network_start_kept"]}
        print(f"[bench] budget {nb}: {budgets[str(nb)]}", file=sys.stderr, flush=True)
    net.close()
    head = per_tol[f"{tols[-1]:g}"]
    out = {
        "metric": METRIC, "value": head["bf16x2_graph_learned"]["slices_per_s"], "unit": "slices/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["bf16x2_graph_learned"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16x2",
        "data": "synthetic (seeded on-device generator; rank-10 U[0,1] CP model + N(0, 0.01^2))",
        "config": {"workload": f"dense1000_f32 forms: {c.t0} initial slices then batches of {t}; "
                               f"P=12, Q=60, S=3; ALS until the replica fit changes by less than "
                               f"tol (at most {args.iters} sweeps) in both forms, every tol in "
                               f"{args.tols}; value = the last tol",
                   "tols": tols, "als_max_iters": args.iters,
                   "train_pairs": int(Xtr.shape[0]), "train_loss": [loss0, loss1]},
        "per_tol": per_tol,
        "fixed_budgets": budgets,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def oracle_gate(X, c, t0, t, nb, U, V, Ws, init, iters):
    """The FP64 oracle over the first nb + 1 batches of the stream (t0
    initial slices, then nb batches of t), each downloaded from the device:
    the fit of Sec. 5.1 over all slices seen after every batch, and the wall
    time of the nb update batches (compress, update, ALS, recover; the fit is
    not timed)."""
    import oracle
    o = oracle.OctenOracle(c.I, c.J, c.R, c.P, c.Q, c.S, U, V)
    host = []
    fits, dt = [], 0.0
    k0 = 0
    for b in range(nb + 1):
        tt = t0 if b == 0 else t
        xb = X[k0:k0 + tt].cpu().numpy()
        host.append(xb)
        t_start = time.perf_counter()
        o.compress_batch(xb.astype(np.float64), Ws[b])
        o.update_replicas()
        o.cp_als_replicas(iters, init=init if b == 0 else None)
        A, B, C = o.recover_factors()
        if b > 0:
            dt += time.perf_counter() - t_start
        k0 += tt
        sse = nx = 0.0
        q = 0
        for xs in host:
            _, s1, n1 = oracle.fit_dense(xs, A, B, C, k0=q)
            sse += s1
            nx += n1
            q += xs.shape[0]
        fits.append(1.0 - float(np.sqrt(sse / nx)))
        print(f"[bench] oracle batch {b}: fit {fits[-1]:.6f}", file=sys.stderr, flush=True)
    return fits, dt


def run_dense(args):
    """The dense 1000 x 1000 stream: the fit gate over exactly its 500
    initial slices and ten batches of 50 (GPU and FP64 oracle on the same
    slices, fit after every batch), then warmup and timed batches continuing
    the same stream."""
    import torch
    from paper_1807_01350_amd import octen as oc
    from paper_1807_01350_amd import synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    c = synth.C2
    t = args.batch
    ngate = len(c.batches) if not args.no_gate else 0
    nsteps = args.warmup + args.steps
    nbatch = ngate + nsteps + (args.steps if args.overlap else 0)
    K = c.t0 + t * nbatch
    print(f"[bench] generating {K} slices", file=sys.stderr, flush=True)
    X = gen_stream(torch, c.I, c.J, K, c.R, c.sigma, synth.seed_of(c.config_id, 1), dev)
    U, V = synth.compression_UV(c.I, c.J, c.P, c.Q, c.S, c.config_id)
    Ws = [synth.temporal_W(c.t0 if b == 0 else t, c.M1, c.config_id, b) for b in range(nbatch + 1)]
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    init = synth.als_init(c.P, c.Q, c.R, c.config_id)
    tinit = torch.from_numpy(init).to(dev)
    eng = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, torch.from_numpy(U).to(dev),
                   torch.from_numpy(V).to(dev), x_dtype="f32", compress_dtype=args.form,
                   als_dtype=args.als_form,
                   flags=oc.OCTEN_FLAG_TIMING | (oc.OCTEN_FLAG_ALS_DEVICE_SYNC
                                                 if args.als_device_sync else 0))
    A = torch.empty((c.I, c.R), dtype=torch.float64, device=dev)
    B = torch.empty((c.J, c.R), dtype=torch.float64, device=dev)
    C = torch.empty((K, c.R), dtype=torch.float64, device=dev)

    def step(b, k0, tt):
        eng.compress_batch(X[k0:k0 + tt], tW[b])
        eng.update_replicas()
        eng.cp_als_replicas(args.iters, init=tinit if b == 0 else None)
        eng.recover_factors_async(A, B, C)

    def gpu_fit():
        sse = nx = 0.0
        for q0 in range(0, eng.K, 100):
            q1 = min(eng.K, q0 + 100)
            sse, nx = eng.fit_terms(X[q0:q1], q0, A, B, C, acc=(sse, nx))
        return 1.0 - float(np.sqrt(sse / nx))

    # initial summary (untimed), tuning of the compression kernel and of the
    # ALS launch shape on it (untimed)
    step(0, 0, c.t0)
    tuned = {"compress": eng.autotune(X[c.t0:c.t0 + t]), "als": eng.autotune_als(20)}
    k0 = c.t0
    gate = None
    if ngate:
        # the fit gate: the stream's own ten batches, the fit after each
        fits_gpu = [gpu_fit()]
        for b in range(1, ngate + 1):
            step(b, k0, t)
            k0 += t
            fits_gpu.append(gpu_fit())
            print(f"[bench] gate batch {b}: gpu fit {fits_gpu[-1]:.6f}", file=sys.stderr, flush=True)
        fits_or, t_or = oracle_gate(X, c, c.t0, t, ngate, U, V, Ws, init, args.iters)
        d = [abs(a - b) for a, b in zip(fits_gpu, fits_or)]
        gate = {"stream": f"{c.t0} initial slices then {ngate} batches of {t} (K = {k0})",
                "form": args.form, "als_form": args.als_form,
                "fit_gpu": [round(x, 6) for x in fits_gpu],
                "fit_oracle": [round(x, 6) for x in fits_or],
                "max_abs_dfit": max(d), "bar": 1e-3, "pass": bool(max(d) <= 1e-3),
                "oracle_update_s": t_or}
    torch.cuda.synchronize()
    b0 = ngate + 1
    for b in range(b0, b0 + args.warmup):
        step(b, k0, t)
        k0 += t
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for b in range(b0 + args.warmup, b0 + nsteps):
        step(b, k0, t)
        k0 += t
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = 1e3 * elapsed / args.steps
    value = t * args.steps / elapsed

    def last(stage):
        v = eng.stage_ms(stage, args.steps)
        return float(np.mean(v)) if v else None

    st = {
        "compress_main": last(oc.OCTEN_STAGE_COMPRESS_MAIN),
        "compress_mode3": last(oc.OCTEN_STAGE_COMPRESS_MODE3),
        "update": last(oc.OCTEN_STAGE_UPDATE),
        "als": last(oc.OCTEN_STAGE_ALS),
        "recover": last(oc.OCTEN_STAGE_RECOVER),
    }
    # algorithmic bytes / flops of one launch of the compression kernel
    # (modes 1, 2): X once, the U and V images once; the flops of the plain
    # product (the two-term form runs twice as many matrix-core products)
    esz = 4 if args.form == "f32" else 2
    bytes_launch = t * c.I * c.J * 4 + (c.I + c.J) * c.M1 * esz
    flops_launch = 2.0 * t * c.I * c.J * c.M1 + 2.0 * t * c.I * c.P * c.Q * c.Q
    mfma_flops = flops_launch * (2 if args.form == "bf16x2" else 1)
    kms = st["compress_main"]
    gbs = bytes_launch / (kms * 1e-3) / 1e9
    tflops = mfma_flops / (kms * 1e-3) / 1e12
    traffic = traffic_from_profile(args.form)
    mpk = "bf16" if args.form != "f32" else "f32"
    # the binding roof of the compression kernel: MFMA when the form's matrix
    # work at peak takes longer than its bytes at the HBM peak
    t_mfma = mfma_flops / (MFMA_PEAK_TFLOPS[mpk] * 1e12)
    t_hbm = bytes_launch / (HBM_PEAK_GBS * 1e9)
    if t_mfma > t_hbm:
        croof = {"bound": "mfma", "achieved": round(tflops, 2), "peak": MFMA_PEAK_TFLOPS[mpk],
                 "unit": "TFLOP/s", "frac": round(tflops / MFMA_PEAK_TFLOPS[mpk], 4),
                 "traffic": traffic}
    else:
        croof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic}
    kname = {0: "compress_pipe", 1: "compress_fused (16-byte loads)", 2: "compress_fused",
             3: "compress_pipe2"}.get(tuned["compress"] % 10, "compress")
    if args.form == "bf16x2":
        kname = "compress_pipe2 two-term"
    croof["kernel"] = f"{kname} (modes 1 and 2 of the batch compression)"
    croof["algorithmic_bytes_per_launch"] = bytes_launch
    croof["algorithmic_flops_per_launch"] = flops_launch
    croof["mfma_flops_per_launch"] = mfma_flops
    croof["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
    croof["mfma_frac"] = round(tflops / MFMA_PEAK_TFLOPS[mpk], 4)
    croof["time_at_peaks_us"] = {"mfma": round(t_mfma * 1e6, 1), "hbm": round(t_hbm * 1e6, 1)}

    # the dominant kernel of the step: the cooperative replica ALS, one launch
    # of args.iters sweeps over all replicas; algorithmic flops of the two slab
    # contractions per sweep and replica 4 Q^3 R (the R x R work is smaller by
    # a factor Q^2 / R); the two-term form runs three BF16 products per product
    als_ms = st["als"]
    als_flops = 4.0 * c.Q ** 3 * c.R * c.P * args.iters
    als_tf = als_flops / (als_ms * 1e-3) / 1e12
    if args.als_form == "bf16x2":
        als_exec, als_pk = 3.0 * als_flops, "bf16"
    else:
        als_exec, als_pk = als_flops, "f64"
    als_xtf = als_exec / (als_ms * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": round(als_xtf, 3), "peak": MFMA_PEAK_TFLOPS[als_pk],
            "unit": "TFLOP/s", "frac": round(als_xtf / MFMA_PEAK_TFLOPS[als_pk], 5),
            "traffic": traffic_from_profile(args.als_form,
                                            source=("als_coop_body.h", "als_coop_kernel_body.inc"),
                                            profile=f"als_coop_{args.als_form}_dense1000_counters.md"),
            "kernel": f"als_coop_kernel ({args.als_form} slab contractions, FP64 solves; "
                      f"{args.iters} sweeps of all {c.P} replicas per launch)",
            "algorithmic_flops_per_launch": als_flops, "mfma_flops_per_launch": als_exec,
            "algorithmic_tflops": round(als_tf, 3),
            "frac_of_fp64_mfma_peak": round(als_tf / MFMA_PEAK_TFLOPS["f64"], 4),
            "note": "latency-bound: a sweep is a chain of small phases, three one-wavefront "
                    "R x R inverses and two replica barriers"}

    overlap = None
    if args.overlap:
        # after the timed steps (whose stage times and roofline are taken
        # above): as many further batches of the stream with the next batch's
        # compression on the handle's second stream, overlapping the current
        # batch's ALS and recovery; every batch still goes through compress,
        # update, ALS and recovery
        b1 = b0 + nsteps
        torch.cuda.synchronize()
        t_ov = time.perf_counter()
        eng.compress_batch_async(X[k0:k0 + t], tW[b1])
        for b in range(b1, b1 + args.steps):
            eng.update_replicas()
            if b + 1 < b1 + args.steps:
                eng.compress_batch_async(X[k0 + t:k0 + 2 * t], tW[b + 1])
            eng.cp_als_replicas(args.iters)
            eng.recover_factors_async(A, B, C)
            k0 += t
        torch.cuda.synchronize()
        el_ov = time.perf_counter() - t_ov
        overlap = {"value": round(t * args.steps / el_ov, 3), "unit": "slices/s",
                   "ms_per_step": round(1e3 * el_ov / args.steps, 4), "steps": args.steps,
                   "what": "next batch's compression on a second stream during the current "
                           "batch's ALS and recovery (octen_compress_batch_async)"}

    fit = None
    if not args.no_fit:
        fit = gpu_fit()

    cpu = None
    if gate is not None and not args.no_cpu_baseline:
        cpu = {"value": ngate * t / gate["oracle_update_s"], "unit": "slices/s",
               "cores": cores_used(), "kind": "oracle",
               "sample": f"the {ngate} update batches of {t} slices of the gate run through the "
                         f"FP64 oracle (compress, update, {args.iters} ALS sweeps on all {c.P} "
                         f"replicas, recover), {gate['oracle_update_s']:.1f} s in total"}

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "slices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.form,
        "data": "synthetic (seeded on-device generator; rank-10 U[0,1] CP model + N(0, 0.01^2))",
        "config": {"workload": f"dense1000_f32: I=J=1000, R=10, {c.t0} initial slices then "
                               f"batches of {t}; P=12, Q=60, S=3; {args.iters} ALS sweeps; "
                               f"{args.form} compression, {args.als_form} ALS contractions, f64 "
                               f"solves; timed batches continue the stream after its ten gate "
                               f"batches",
                   "I": c.I, "J": c.J, "R": c.R, "P": c.P, "Q": c.Q, "S": c.S, "batch": t,
                   "initial_slices": c.t0, "als_iters": args.iters, "compress_dtype": args.form,
                   "als_dtype": args.als_form},
        "fit_gate": gate,
        "fit_oracle": gate["fit_oracle"][-1] if gate else None,
        "abs_dfit": gate["max_abs_dfit"] if gate else None,
        "compression_gbs": round(gbs, 1),
        "compression_hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
        "stage_ms": {k: (round(v, 4) if v is not None else None) for k, v in st.items()},
        "autotuned": tuned,
        "fit": fit,
        "roofline": roof,
        "roofline_compression": croof,
        "cpu_baseline": cpu,
        "overlapped": overlap,
    }
    eng.close()
    print(json.dumps(out))


def run_dense50(args):
    """The dense 50 x 50 FP64 stream (rank 5, 30 initial slices then batches of
    10; P = 4 replicas of 20^3, S = 3, 50 sweeps).  Fit gate over exactly its
    50 slices (GPU and FP64 oracle after every batch), then timed batches of
    10 continuing the same stream; the oracle is timed on the same batches
    (about 10 s of them).  Latency-bound: absolute microseconds per batch."""
    import torch
    import oracle
    from paper_1807_01350_amd import octen as oc
    from paper_1807_01350_amd import synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    c = synth.C1
    t = 10
    nsteps = args.warmup + args.steps
    ngate = len(c.batches)
    K = c.t0 + t * (ngate + nsteps)
    _, _, _, Xh = synth.dense_stream(c.I, c.J, K, c.R, c.sigma, c.config_id, dtype=np.float64)
    X = torch.from_numpy(Xh).to(dev)
    U, V = synth.compression_UV(c.I, c.J, c.P, c.Q, c.S, c.config_id)
    nb = ngate + nsteps
    Ws = [synth.temporal_W(c.t0 if b == 0 else t, c.M1, c.config_id, b) for b in range(nb + 1)]
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    init = synth.als_init(c.P, c.Q, c.R, c.config_id)
    eng = oc.Octen(c.I, c.J, c.R, c.P, c.Q, c.S, torch.from_numpy(U).to(dev),
                   torch.from_numpy(V).to(dev), x_dtype="f64", compress_dtype="f64",
                   flags=oc.OCTEN_FLAG_TIMING)
    A = torch.empty((c.I, c.R), dtype=torch.float64, device=dev)
    B = torch.empty((c.J, c.R), dtype=torch.float64, device=dev)
    C = torch.empty((K, c.R), dtype=torch.float64, device=dev)
    tinit = torch.from_numpy(init).to(dev)

    def step(b, k0, tt):
        eng.compress_batch(X[k0:k0 + tt], tW[b])
        eng.update_replicas()
        eng.cp_als_replicas(args.iters, init=tinit if b == 0 else None)
        eng.recover_factors_async(A, B, C)

    o = oracle.OctenOracle(c.I, c.J, c.R, c.P, c.Q, c.S, U, V)
    fits_gpu, fits_or, k0 = [], [], 0
    for b in range(ngate + 1):
        tt = c.t0 if b == 0 else t
        step(b, k0, tt)
        o.compress_batch(Xh[k0:k0 + tt], Ws[b])
        o.update_replicas()
        o.cp_als_replicas(args.iters, init=init if b == 0 else None)
        Ao, Bo, Co = o.recover_factors()
        k0 += tt
        sse, nx = eng.fit_terms(X[:k0], 0, A, B, C)
        fits_gpu.append(1.0 - float(np.sqrt(sse / nx)))
        fits_or.append(oracle.fit_dense(Xh[:k0], Ao, Bo, Co)[0])
    d = [abs(a - b) for a, b in zip(fits_gpu, fits_or)]
    gate = {"stream": f"{c.t0} initial slices then {ngate} batches of {t} (K = {k0})",
            "form": "f64", "fit_gpu": fits_gpu, "fit_oracle": fits_or, "max_abs_dfit": max(d),
            "bar": 1e-3, "pass": bool(max(d) <= 1e-3)}
    b0 = ngate + 1
    for b in range(b0, b0 + args.warmup):
        step(b, k0, t)
        k0 += t
    torch.cuda.synchronize()
    k_timed = k0
    t_start = time.perf_counter()
    for b in range(b0 + args.warmup, b0 + nsteps):
        step(b, k0, t)
        k0 += t
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    st = {name: (float(np.mean(eng.stage_ms(stage, args.steps))) if eng.stage_ms(stage, args.steps)
                 else None)
          for name, stage in (("compress_main", oc.OCTEN_STAGE_COMPRESS_MAIN),
                              ("compress_mode3", oc.OCTEN_STAGE_COMPRESS_MODE3),
                              ("update", oc.OCTEN_STAGE_UPDATE), ("als", oc.OCTEN_STAGE_ALS),
                              ("recover", oc.OCTEN_STAGE_RECOVER))}
    # the oracle on the same timed batches (continuing its own stream state
    # from the gate), up to about 10 s
    dt_or, n_or, ko = 0.0, 0, c.t0 + t * ngate
    for b in range(b0, b0 + nsteps):
        t0_ = time.perf_counter()
        o.compress_batch(Xh[ko:ko + t], Ws[b])
        o.update_replicas()
        o.cp_als_replicas(args.iters)
        o.recover_factors()
        dt_or += time.perf_counter() - t0_
        ko += t
        n_or += 1
        if dt_or > 10.0:
            break
    als_flops = 4.0 * c.Q ** 3 * c.R * c.P * args.iters
    als_ms = st["als"]
    out = {
        "metric": METRIC, "value": round(t * args.steps / elapsed, 3), "unit": "slices/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4), "us_per_batch": round(1e6 * elapsed / args.steps, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded host generator; rank-5 U[0,1] CP model + N(0, 0.01^2))",
        "config": {"workload": f"dense50_f64: I=J=50, R=5, {c.t0} initial slices then batches of "
                               f"{t}; P=4, Q=20, S=3; {args.iters} ALS sweeps; FP64 throughout; "
                               f"timed batches continue the stream after its two gate batches",
                   "I": c.I, "J": c.J, "R": c.R, "P": c.P, "Q": c.Q, "S": c.S, "batch": t,
                   "initial_slices": c.t0, "als_iters": args.iters, "first_timed_slice": k_timed},
        "fit_gate": gate, "fit_oracle": fits_or[-1], "abs_dfit": max(d),
        "stage_ms": {k: (round(v, 4) if v is not None else None) for k, v in st.items()},
        "roofline": {"bound": "mfma", "achieved": round(als_flops / (als_ms * 1e-3) / 1e12, 4),
                     "peak": 78.6, "unit": "TFLOP/s",
                     "frac": round(als_flops / (als_ms * 1e-3) / 1e12 / 78.6, 6), "traffic": None,
                     "kernel": "replica ALS (4 Q^3 R flop per replica and sweep, FP64 MFMA); "
                               "the whole batch is bound by launch latency"},
        "cpu_baseline": {"value": round(t * n_or / dt_or, 3), "unit": "slices/s",
                         "cores": cores_used(), "kind": "oracle",
                         "sample": f"{n_or} update batches of {t} slices of the same stream through "
                                   f"the FP64 oracle, {dt_or:.2f} s"},
    }
    eng.close()
    print(json.dumps(out))


def run_nmode(args):
    """The four-mode stream of the N-mode extension (supplement, higher-order
    tensors): X of 100 x 100 x 100 x K with rank-5 U[0,1] factors plus
    N(0, 0.01^2) noise, streamed along the fourth mode: 20 initial slices, then
    batches of 10; P = 10 replicas of 16^4 with S = 4 shared anchor rows
    (M1 = 124 >= 100, every mode determined), 50 ALS sweeps, FP64 throughout.
    Fit gate against the N-mode oracle over the first three batches, then
    timed batches continuing the stream; the oracle is timed on the same
    batches (about 10 s of them)."""
    import torch
    from oracle.nmode import OctenNOracle, fit_dense_n
    from paper_1807_01350_amd import octen as oc
    from paper_1807_01350_amd import synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    dims, R, P, Q, S, sigma, cid = (100, 100, 100), 5, 10, 16, 4, 0.01, 50
    N = len(dims) + 1
    M1 = S + P * (Q - S)
    t0, t = 20, 10
    ngate = 3
    nsteps = args.warmup + args.steps
    sched = [t0] + [t] * (ngate - 1 + nsteps)
    K = sum(sched)
    fac, Ct = synth.nmode_factors(dims, K, R, cid)
    Us = synth.compression_Us(dims, P, Q, S, cid)
    init = synth.nmode_als_init(P, N, Q, R, cid)
    Xh, Ws, k0 = [], [], 0
    for b, tt in enumerate(sched):
        Xh.append(synth.nmode_slices(fac, Ct, k0, tt, sigma, cid, b))
        Ws.append(synth.temporal_W(tt, M1, cid, b))
        k0 += tt
    X = [torch.from_numpy(x).to(dev) for x in Xh]
    tW = [torch.from_numpy(w).to(dev) for w in Ws]
    eng = oc.OctenN(dims, R, P, Q, S, [torch.from_numpy(u).to(dev) for u in Us])
    As = [torch.empty((d, R), dtype=torch.float64, device=dev) for d in dims]
    C = torch.empty((K, R), dtype=torch.float64, device=dev)
    tinit = torch.from_numpy(init).to(dev)
    stream = torch.cuda.current_stream()
    ev = {k: [] for k in ("compress", "als", "step")}

    def step(b, timed=False):
        if timed:
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record(stream)
        eng.compress_batch(X[b], tW[b])
        if timed:
            e[1].record(stream)
        eng.update_replicas()
        if timed:
            e[2].record(stream)
        eng.cp_als_replicas(args.iters, init=tinit if b == 0 else None)
        if timed:
            e[3].record(stream)
            ev["compress"].append((e[0], e[1]))
            ev["als"].append((e[2], e[3]))
        eng.recover_factors_async(As, C, sched[b])

    o = OctenNOracle(dims, R, P, Q, S, Us)
    fits_gpu, fits_or, k0 = [], [], 0
    for b in range(ngate):
        step(b)
        o.compress_batch(Xh[b], Ws[b])
        o.update_replicas()
        o.cp_als_replicas(args.iters, init=init if b == 0 else None)
        Ao, Co = o.recover_factors()
        k0 += sched[b]
        acc = (0.0, 0.0)
        kk = 0
        for bb in range(b + 1):
            acc = eng.fit_terms(X[bb], kk, As, C, acc)
            kk += sched[bb]
        fits_gpu.append(1.0 - float(np.sqrt(acc[0] / acc[1])))
        fits_or.append(fit_dense_n(np.concatenate(Xh[:b + 1]), Ao, Co)[0])
    d = [abs(a - b) for a, b in zip(fits_gpu, fits_or)]
    gate = {"stream": f"{t0} initial slices then {ngate - 1} batches of {t} (K = {k0})",
            "form": "f64", "fit_gpu": fits_gpu, "fit_oracle": fits_or, "max_abs_dfit": max(d),
            "bar": 1e-3, "pass": bool(max(d) <= 1e-3)}
    for b in range(ngate, ngate + args.warmup):
        step(b)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for b in range(ngate + args.warmup, ngate + nsteps):
        step(b, timed=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms = {k: float(np.mean([a.elapsed_time(z) for a, z in v])) for k, v in ev.items() if v}
    # the oracle on the timed batches, continuing its own stream state, up to ~10 s
    dt_or, n_or = 0.0, 0
    for b in range(ngate, ngate + nsteps):
        t0_ = time.perf_counter()
        o.compress_batch(Xh[b], Ws[b])
        o.update_replicas()
        o.cp_als_replicas(args.iters)
        o.recover_factors()
        dt_or += time.perf_counter() - t0_
        n_or += 1
        if dt_or > 10.0:
            break
    # replica ALS: 4 Q^N R flop per replica and sweep (two contractions of the
    # whole summary with a factor per sweep, as a dimension tree needs)
    als_flops = 4.0 * Q ** N * R * P * args.iters
    als_tf = als_flops / (ms["als"] * 1e-3) / 1e12
    # compression: the batch read once, Z written once (FP64 bytes); FP64
    # flops of the mode products (the GEMM over all M1 columns of the last
    # non-temporal mode, then the other modes per replica, then the temporal)
    comp_bytes = 8.0 * (t * np.prod(dims) + P * Q ** N)
    comp_flops = 2.0 * t * np.prod(dims) * M1
    lead = t * np.prod(dims[:-1])
    post = Q
    for d_ in reversed(dims[:-1]):
        lead //= d_
        comp_flops += 2.0 * P * lead * d_ * Q * post
        post *= Q
    comp_flops += 2.0 * P * t * Q ** N
    t_hbm = comp_bytes / (HBM_PEAK_GBS * 1e9)
    t_mfma = comp_flops / (MFMA_PEAK_TFLOPS["f64"] * 1e12)
    comp_s = ms["compress"] * 1e-3
    if t_mfma > t_hbm:
        comp_roof = {"bound": "mfma", "achieved": round(comp_flops / comp_s / 1e12, 3),
                     "peak": MFMA_PEAK_TFLOPS["f64"], "unit": "TFLOP/s",
                     "frac": round(comp_flops / comp_s / 1e12 / MFMA_PEAK_TFLOPS["f64"], 6)}
    else:
        comp_roof = {"bound": "hbm", "achieved": round(comp_bytes / comp_s / 1e9, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(comp_bytes / comp_s / 1e9 / HBM_PEAK_GBS, 6)}
    comp_roof.update({"algorithmic_bytes": comp_bytes, "algorithmic_flops": comp_flops,
                      "kernel": "compression of one batch (FP64 GEMM over all M1 columns, mode "
                                "products on FP64 matrix cores, temporal product)"})
    out = {
        "metric": METRIC, "value": round(t * args.steps / elapsed, 3), "unit": "slices/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded host generator; rank-5 U[0,1] CP model of four modes + "
                "N(0, 0.01^2))",
        "config": {"workload": f"nmode4_f64: 100 x 100 x 100 x K, R=5, {t0} initial slices then "
                               f"batches of {t}; P=10, Q=16, S=4 (replicas of 16^4); "
                               f"{args.iters} ALS sweeps; FP64 throughout",
                   "dims": list(dims), "R": R, "P": P, "Q": Q, "S": S, "batch": t,
                   "initial_slices": t0, "als_iters": args.iters},
        "fit_gate": gate, "fit_oracle": fits_or[-1], "abs_dfit": max(d),
        "stage_ms": {"compress": round(ms["compress"], 4), "als": round(ms["als"], 4)},
        "roofline": {"bound": "alu", "achieved": round(als_tf, 4), "peak": 78.6,
                     "unit": "TFLOP/s", "frac": round(als_tf / 78.6, 6),
                     "traffic": traffic_from_profile(None, source="nmode.hip",
                                                     profile="nm_als_nmode4_f64_counters.md"),
                     "kernel": "nm_als_kernel (4 Q^N R flop per replica and sweep, FP64 vector "
                               "arithmetic; up to 8 cooperative workgroups per replica); timed "
                               "with the ALS call's small commit kernels"},
        "roofline_compression": comp_roof,
        "cpu_baseline": {"value": round(t * n_or / dt_or, 3), "unit": "slices/s",
                         "cores": cores_used(), "kind": "oracle",
                         "sample": f"{n_or} update batches of {t} slices of the same stream "
                                   f"through the FP64 N-mode oracle, {dt_or:.2f} s"},
    }
    eng.close()
    print(json.dumps(out))


def long_shape(I):
    """Replica layout of the long-stream workload for slices of I x I: Q = 20,
    S = 3, R = 5 and the fewest replicas with M1 = S + P (Q - S) > I (modes 1
    and 2 determined, Eq. 8's first two terms), at least two."""
    Q, S, R = 20, 3, 5
    P = max(2, (I - S) // (Q - S) + 1)
    return R, P, Q, S


def run_long(args):
    """The long-stream workload of the scalability experiment (Sec. 5.4.2):
    small slices (I = J = --long-I, 100 by default), a long time mode
    (K = --long-K slices, 10^5 by default), an initial summary of at most
    10 % of the stream and at most M1 slices, then batches of 10 slices.  Each batch runs compress, update,
    ALS (--iters sweeps from the previous factors) and recovery; the stream is
    run twice, eagerly and with compress + update + ALS replayed as one
    captured HIP graph per batch.  Reports per-batch latency at the start
    and at the end of the stream (the temporal carry keeps the cost of a
    batch independent of K), the fit over all K slices, a fit gate against
    the FP64 oracle on a prefix (the initial summary and 20 batches) and the
    oracle's speed on that prefix."""
    import torch
    import oracle
    from paper_1807_01350_amd import octen as oc
    from paper_1807_01350_amd import synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    I = J = args.long_I
    K = args.long_K
    R, P, Q, S = long_shape(I)
    M1 = S + P * (Q - S)
    # the initial summary: at most 10 % of the stream (as the experiment
    # sets it) and at most M1 slices, so that its temporal rows are
    # determined by the M1 compressed rows (reading R-C1)
    t = 10
    t0 = max(t, (min(K // 10, M1) // t) * t)
    nb = (K - t0) // t
    K = t0 + nb * t
    cid = 6
    print(f"[bench] long stream: I=J={I}, K={K}, P={P}, Q={Q}, S={S}, R={R}", file=sys.stderr,
          flush=True)
    X = gen_stream(torch, I, J, K, R, 0.01, synth.seed_of(cid, 1), dev)
    U, V = synth.compression_UV(I, J, P, Q, S, cid)
    init = synth.als_init(P, Q, R, cid)
    g = torch.Generator(device=dev)
    g.manual_seed(synth.seed_of(cid, 2))
    Wall = torch.randn((K, M1), generator=g, device=dev, dtype=torch.float64)
    tinit = torch.from_numpy(init).to(dev)
    results = {}
    for mode in ("eager", "graph"):
        eng = oc.Octen(I, J, R, P, Q, S, torch.from_numpy(U).to(dev), torch.from_numpy(V).to(dev),
                       x_dtype="f32", compress_dtype="f32")
        A = torch.empty((I, R), dtype=torch.float64, device=dev)
        B = torch.empty((J, R), dtype=torch.float64, device=dev)
        C = torch.empty((K, R), dtype=torch.float64, device=dev)
        eng.compress_batch(X[:t0], Wall[:t0])
        eng.update_replicas()
        eng.cp_als_replicas(args.iters, init=tinit)
        eng.recover_factors(A, B, C)
        group = None
        if mode == "graph":
            group = oc.Group([eng])
            xb = torch.empty((t, I, J), dtype=torch.float32, device=dev)
            wb = torch.empty((t, M1), dtype=torch.float64, device=dev)
        lat = []
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        k0 = t0
        for b in range(nb):
            timed = b < 200 or b >= nb - 200
            if timed:
                ev[0].record()
            if group is not None:
                xb.copy_(X[k0:k0 + t])
                wb.copy_(Wall[k0:k0 + t])
                group.step([(xb, wb)], args.iters)
            else:
                eng.compress_batch(X[k0:k0 + t], Wall[k0:k0 + t])
                eng.update_replicas()
                eng.cp_als_replicas(args.iters)
            eng.recover_factors_async(A, B, C)
            if timed:
                ev[1].record()
                ev[1].synchronize()
                lat.append(ev[0].elapsed_time(ev[1]))
            k0 += t
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        sse = nx = 0.0
        for q0 in range(0, K, 4096):
            sse, nx = eng.fit_terms(X[q0:min(K, q0 + 4096)], q0, A, B, C, acc=(sse, nx))
        results[mode] = {"slices_per_s": round(nb * t / elapsed, 1),
                         "us_per_batch_first200": round(1e3 * float(np.mean(lat[:200])), 1),
                         "us_per_batch_last200": round(1e3 * float(np.mean(lat[-200:])), 1),
                         "fit_all_slices": 1.0 - float(np.sqrt(sse / nx))}
        print(f"[bench] long {mode}: {results[mode]}", file=sys.stderr, flush=True)
        if group is not None:
            group.close()
        eng.close()
    # fit gate and oracle speed on a prefix: the initial summary and 20 batches
    nb_or = min(20, nb)
    kp = t0 + nb_or * t
    Xp = X[:kp].double().cpu().numpy()
    Wp = Wall[:kp].cpu().numpy()
    o = oracle.OctenOracle(I, J, R, P, Q, S, U, V)
    eng = oc.Octen(I, J, R, P, Q, S, torch.from_numpy(U).to(dev), torch.from_numpy(V).to(dev),
                   x_dtype="f32", compress_dtype="f32")
    A = torch.empty((I, R), dtype=torch.float64, device=dev)
    B = torch.empty((J, R), dtype=torch.float64, device=dev)
    C = torch.empty((kp, R), dtype=torch.float64, device=dev)
    k0, dt_or = 0, 0.0
    for b in range(nb_or + 1):
        tt = t0 if b == 0 else t
        eng.compress_batch(X[k0:k0 + tt], Wall[k0:k0 + tt])
        eng.update_replicas()
        eng.cp_als_replicas(args.iters, init=tinit if b == 0 else None)
        eng.recover_factors(A, B, C)
        t1 = time.perf_counter()
        o.compress_batch(Xp[k0:k0 + tt], Wp[k0:k0 + tt])
        o.update_replicas()
        o.cp_als_replicas(args.iters, init=init if b == 0 else None)
        Ao, Bo, Co = o.recover_factors()
        if b > 0:
            dt_or += time.perf_counter() - t1
        k0 += tt
    sse, nx = eng.fit_terms(X[:kp], 0, A, B, C)
    fit_g = 1.0 - float(np.sqrt(sse / nx))
    fit_o = oracle.fit_dense(Xp, Ao, Bo, Co)[0]
    eng.close()
    e = results["eager"]
    out = {
        "metric": METRIC, "value": e["slices_per_s"], "unit": "slices/s", "n_gpus": 1,
        "steps": nb, "warmup": 0, "ms_per_step": round(1e3 * t / e["slices_per_s"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded on-device generator; rank-5 U[0,1] CP model + N(0, 0.01^2))",
        "config": {"workload": f"long{I}: I=J={I}, K={K} ({t0} initial slices, then {nb} batches "
                               f"of {t}), R={R}, P={P}, Q={Q}, S={S}; {args.iters} ALS sweeps per "
                               f"batch from the previous factors; FP32 compression, FP64 solves",
                   "I": I, "J": J, "K": K, "R": R, "P": P, "Q": Q, "S": S, "batch": t,
                   "initial_slices": t0, "als_iters": args.iters},
        "modes": results,
        "fit_gate": {"prefix": f"{t0} initial slices then {nb_or} batches", "fit_gpu": fit_g,
                     "fit_oracle": fit_o, "abs_dfit": abs(fit_g - fit_o),
                     "pass": bool(abs(fit_g - fit_o) <= 1e-3)},
        "roofline": None,
        "cpu_baseline": {"value": round(nb_or * t / dt_or, 3), "unit": "slices/s",
                         "cores": cores_used(), "kind": "oracle",
                         "sample": f"{nb_or} update batches of {t} slices through the FP64 oracle, "
                                   f"{dt_or:.2f} s"},
    }
    print(json.dumps(out))


def run_sweep(args):
    """The parameter sensitivity experiment (Sec. 5.4.3) and an empirical look
    at Eq. 8: one dense FP64 stream (I = J = K = 100, rank 5, noise 0.01; 10
    initial slices, then batches of 10 = 0.1 K), run through the whole
    update for a range of p (Q = 20, S = 4), of Q (p = 7, S = 4) and of S
    (p = 7, Q = 20), each with --sweep-seeds seeds of the compression
    matrices and ALS start; reports the mean and spread of the final fit
    with M1, Eq. 8's bound and the determinacy verdicts of every setting."""
    import torch
    from paper_1807_01350_amd import octen as oc
    from paper_1807_01350_amd import synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    I = J = K = 100
    R, sigma, t0, t = 5, 0.01, 10, 10
    _, _, _, Xh = synth.dense_stream(I, J, K, R, sigma, 5)
    X = torch.from_numpy(Xh).to(dev)
    grid = ([("p", P, 20, 4) for P in range(2, 13)] +
            [("Q", 7, Q, 4) for Q in (8, 12, 16, 20, 24, 30, 40)] +
            [("shared", 7, 20, Sv) for Sv in (1, 2, 4, 6, 8, 10, 12, 16)])
    rows = []
    gpu_s, slices = 0.0, 0
    for what, P, Q, Sv in grid:
        M1 = Sv + P * (Q - Sv)
        fits = []
        for seed in range(args.sweep_seeds):
            cid = 500 + seed
            U, V = synth.compression_UV(I, J, P, Q, Sv, cid)
            init = torch.from_numpy(synth.als_init(P, Q, R, cid)).to(dev)
            eng = oc.Octen(I, J, R, P, Q, Sv, torch.from_numpy(U).to(dev),
                           torch.from_numpy(V).to(dev))
            A = torch.empty((I, R), dtype=torch.float64, device=dev)
            B = torch.empty((J, R), dtype=torch.float64, device=dev)
            C = torch.empty((K, R), dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            k0, b = 0, 0
            while k0 < K:
                tt = t0 if b == 0 else t
                W = torch.from_numpy(synth.temporal_W(tt, M1, cid, b)).to(dev)
                eng.compress_batch(X[k0:k0 + tt], W)
                eng.update_replicas()
                eng.cp_als_replicas(args.iters, init=init if b == 0 else None)
                eng.recover_factors_async(A, B, C)
                k0 += tt
                b += 1
            torch.cuda.synchronize()
            gpu_s += time.perf_counter() - t1
            slices += K
            sse, nx = eng.fit_terms(X, 0, A, B, C)
            fits.append(1.0 - float(np.sqrt(sse / nx)))
            eng.close()
        st_, bits, pmin = oc.octen_check_identifiable(oc.make_config(I, J, R, P, Q, Sv), K, t)
        if st_ != oc.OCTEN_OK:
            raise RuntimeError(f"octen_check_identifiable: status {st_}")
        rows.append({"vary": what, "p": P, "Q": Q, "shared": Sv, "M1": M1,
                     "p_min_eq8": round(pmin, 3), "eq8_holds": bool(bits & 1),
                     "modes12_determined": bool(bits & 2 and bits & 4),
                     "fit_median": float(np.median(fits)), "fit_max": max(fits),
                     "fit_min": min(fits)})
        print(f"[bench] sweep {rows[-1]}", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC, "value": round(slices / gpu_s, 1), "unit": "slices/s", "n_gpus": 1,
        "steps": len(grid) * args.sweep_seeds, "warmup": 0,
        "ms_per_step": round(1e3 * gpu_s / (len(grid) * args.sweep_seeds), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded host generator; rank-5 U[0,1] CP model + N(0, 0.01^2))",
        "config": {"workload": f"sweep: I=J=K={I}, R={R}, {t0} initial slices then batches of "
                               f"{t}; {args.iters} ALS sweeps; FP64; {args.sweep_seeds} seeds "
                               f"per setting; one step = one whole stream",
                   "seeds": args.sweep_seeds},
        "sweep": rows,
        "roofline": None,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        # the oracle on one whole stream of the grid (p = 6, Q = 20, S = 4,
        # first seed), timed from its first batch to its last recovery
        import oracle
        P, Q, Sv, cid = 6, 20, 4, 500
        M1 = Sv + P * (Q - Sv)
        U, V = synth.compression_UV(I, J, P, Q, Sv, cid)
        o = oracle.OctenOracle(I, J, R, P, Q, Sv, U, V)
        t1 = time.perf_counter()
        k0, b = 0, 0
        while k0 < K:
            tt = t0 if b == 0 else t
            o.compress_batch(Xh[k0:k0 + tt], synth.temporal_W(tt, M1, cid, b))
            o.update_replicas()
            o.cp_als_replicas(args.iters, init=synth.als_init(P, Q, R, cid) if b == 0 else None)
            o.recover_factors()
            k0 += tt
            b += 1
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": round(K / dt, 3), "unit": "slices/s",
                               "cores": cores_used(), "kind": "oracle",
                               "sample": f"one whole stream of the grid (p = {P}, Q = {Q}, "
                                         f"shared = {Sv}, {K} slices) through the FP64 oracle, "
                                         f"{dt:.2f} s"}
    print(json.dumps(out))


def run_copy(args):
    """Counter calibration: a plain device-to-device copy of 256 MiB, three
    times, whose hardware byte counters (FETCH_SIZE, WRITE_SIZE) are compared
    with the 3 x 256 MiB read and written."""
    import torch
    n = 64 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "copy", "bytes_per_copy": n * 4, "copies": 3}))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload == "copy":
        return run_copy(args)
    if args.workload == "dense50":
        return run_dense50(args)
    if args.workload == "long":
        return run_long(args)
    if args.workload == "sweep":
        return run_sweep(args)
    if args.workload == "sparse":
        return run_sparse(args)
    if args.workload == "forms":
        return run_forms(args)
    if args.workload == "nmode":
        return run_nmode(args)
    if args.workload == "batched":
        if args.warmup + args.steps > 4:
            args.warmup, args.steps = 1, 3
        return run_batched(args)
    return run_dense(args)


if __name__ == "__main__":
    main()
