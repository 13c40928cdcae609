"""Throughput of the Neural Bounding hot path on one GPU.

Default workload (`voxel3d_point`): 3-D point queries against a 128^3 voxel
grid of 16 seeded metaballs; bound 3 -> 64^3 -> 1 (ReLU, float32 on the
matrix cores); trained on the device (batches of 2^16 regions drawn and
labelled per step; FN weight ramped 1 -> 100 over 5000 steps, then the
paper's step-wise schedule until a validation set shows FN = 0); evaluated
on 2^24 held-out queries (disjoint seed).

A timed step is one pass of the trained bound over the 2^24 held-out queries
(forward + decision, inputs resident in HBM).  Reported beside it: training
samples/s over the whole training run, the exact indicator test on the same
queries and GPU, the cascade (bound, then exact test on the positives), FN /
FP on the held-out set, the roofline of the forward kernel, and the CPU
oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--also]

--workload picks another workload (voxel3d_ray: 6 -> 128^4 bfloat16 bound
over rays); --also appends the other workloads' measurements under "also".
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0}   # MI355X dense matrix peaks (FP32, BF16)


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def sources_sha256(sources) -> str:
    """SHA-256 over the bytes of the given files (repository paths), in order."""
    h = hashlib.sha256()
    for src in sources:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()


def committed_traffic(name: str, sources, kernel: str = ""):
    """HBM bytes per launch from a committed rocprofv3 counter summary (the
    line of `kernel`, the tuned variant's name, when the summary lists it), or
    None if a source file of the kernel has changed since the counters were
    taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv, per_variant = {}, {}
    for line in open(path):
        if line.startswith("variant:"):
            parts = [x.strip() for x in line[len("variant:"):].split("|")]
            for x in parts[1:]:
                if x.startswith("traffic_bytes"):
                    per_variant[parts[0]] = int(x.split()[1])
        elif ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("sources", kv.get("source")) != " ".join(sources):
        return None
    if kv.get("source_sha256") != sources_sha256(sources):
        return None
    if kernel and kernel in per_variant:
        return per_variant[kernel]
    try:
        return int(float(kv["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


# Kernel names of the bfloat16 forward variants (the variant tables of
# csrc/mlp_bf16.hip): widths 32..128 take (blocks per wave, threads), width
# 256 (streamed) (SPLIT, blocks per wave, threads, half-layer accumulators).
BF16_FWD_VARIANTS = [(2, 768), (2, 512), (3, 512), (1, 1024), (4, 256), (2, 256)]
BF16_STREAM_VARIANTS = [(2, 3, 256, False), (1, 3, 256, False), (3, 3, 256, False), (2, 2, 512, False),
                        (1, 2, 512, False), (2, 2, 512, True), (1, 2, 512, True)]


def bf16_forward_kernel(width: int, n_hidden: int, variant: int) -> str:
    if width == 256:
        sp, nbk, th, hv = BF16_STREAM_VARIANTS[variant]
        return f"k_fwd_bf16_stream<{n_hidden}, {sp}, {nbk}, {th}, {'true' if hv else 'false'}>"
    nbk, th = BF16_FWD_VARIANTS[variant]
    return f"k_fwd_bf16<{width}, {n_hidden}, {nbk}, {th}>"


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_label_fn(W):
    """The oracle's exact query g for the workload's scene (host copy)."""
    import synth
    from oracle import indicators as I
    sc = W.scene
    if sc["type"] == "discs":
        discs = synth.discs2d(W.seeds["scene"], k=sc["k"])
        return lambda q: I.discs2d(q, discs)
    if sc["type"] == "metaballs4d":
        a, b, r = synth.metaballs4d(W.seeds["scene"], k=sc["k"], rlo=sc["rlo"], rhi=sc["rhi"])
        return lambda q: I.metaballs4d(q, a, b, r)
    c, r = synth.metaballs3d(1000 + sc.get("seed_of", W.index), k=sc["k"], rlo=sc["rlo"], rhi=sc["rhi"])
    grid = I.voxelize_metaballs(c, r, sc["n"])
    fn = {"point": I.voxel_points, "ray": I.voxel_rays, "box": I.voxel_boxes, "plane": I.voxel_planes}[W.kind]
    return lambda q: fn(q, grid, sc["n"])


def cpu_baseline(W, theta, q_sample, pos_q, pos_h, seconds: float = 15.0):
    """The oracle (float64 numpy; the bfloat16 rounding model for bfloat16
    bounds) on the host cores, on bounded samples of the held-out queries:
    forward + decision (all BLAS threads for `seconds`, then one core), the
    exact query g, and one training step (Eq. 1 loss and gradient, Adam).
    Also recounts the held-out false negatives with the trained weights on
    every held-out query whose exact answer is 1 (pos_q, with the GPU's
    decisions pos_h): h >= g must hold there (Sec. 3.1)."""
    import concurrent.futures as cf

    from oracle import loss as L, mlp, train as T
    from oracle.adam import Adam
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count() or 1
    widths = [W.width] * W.n_hidden
    bf16 = W.precision == "bf16"
    act = W.act
    chunk = 1 << 14 if W.width <= 128 else 1 << 12
    q = np.ascontiguousarray(q_sample[:chunk])

    def run_for(fn, limit):
        """fn() back to back until `limit` seconds have passed: (calls, seconds)."""
        reps, t0 = 0, time.perf_counter()
        while True:
            fn()
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= limit:
                return reps, dt

    fwd = lambda: L.decide(mlp.forward(theta, W.in_dim, widths, q, bf16=bf16, act=act))
    fwd()   # warm-up (thread pool, first touch)
    reps, dt = run_for(fwd, seconds)
    out = {"value": reps * chunk / dt, "unit": "bound queries/s", "cores": int(cores), "kind": "oracle",
           "sample": f"{reps} x {chunk} held-out queries of the {W.name} workload, float64 numpy forward"
                     f"{' (bfloat16 rounding model)' if bf16 else ''} + decision, {dt:.1f} s on {cores} BLAS "
                     f"threads",
           "host": {"cpu_model": cpu_model(), "logical_cpus": os.cpu_count()}}
    if threadpool_limits is not None:
        with threadpool_limits(1):
            reps1, dt1 = run_for(fwd, seconds / 3)
        out["value_one_core"] = reps1 * chunk / dt1
    # the exact query on a sample of the same queries
    label = oracle_label_fn(W)
    ne = {"ray": 1 << 10, "plane": 1 << 8}.get(W.kind, 1 << 14)
    label(q[:64])
    reps_e, dt_e = run_for(lambda: label(q[:ne]), seconds / 3)
    out["exact"] = {"value": reps_e * ne / dt_e, "unit": "exact queries/s",
                    "sample": f"{reps_e} x {ne} queries, one thread (numpy)"}
    # one training step of Alg. 1: labels, Eq. 1 loss and gradient, Adam
    nt = 1 << 10 if W.width >= 256 else 1 << 12
    qt = np.ascontiguousarray(q_sample[chunk:chunk + nt] if q_sample.shape[0] >= chunk + nt else q[:nt])
    opt = Adam(theta.size)

    def step():
        y = label(qt)
        _, g, _ = T.step_grad(theta, W.in_dim, widths, qt, y, 50.0, 1.0, bf16=bf16, act=act)
        opt.step(theta.astype(np.float64), g)

    step()
    reps_t, dt_t = run_for(step, seconds / 3)
    out["train"] = {"value": reps_t * nt / dt_t, "unit": "train samples/s",
                    "sample": f"{reps_t} steps x {nt} samples (labels + loss + gradient + Adam), {cores} BLAS threads"}
    # recount of the held-out false negatives by the oracle
    t0 = time.perf_counter()
    rc = 1 << 14
    parts = [(pos_q[i:i + rc], pos_h[i:i + rc]) for i in range(0, pos_q.shape[0], rc)]

    def recount(part):
        qq, hh = part
        z = mlp.forward(theta, W.in_dim, widths, qq, bf16=bf16, act=act)
        sure = ~(np.abs(z) < 1e-4)
        d = L.decide(z)
        return int(((d == 0) & sure).sum()), int((~sure).sum()), int(((d != hh) & sure).sum())

    workers = max(1, min(16, os.cpu_count() or 1))
    ctx = threadpool_limits(1) if threadpool_limits is not None else None
    if ctx is not None:
        ctx.__enter__()
    try:
        with cf.ThreadPoolExecutor(workers) as ex:
            res = list(ex.map(recount, parts))
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    out["oracle_recount"] = {
        "positives": int(pos_q.shape[0]), "fn_outside_band": sum(r[0] for r in res),
        "band_rows": sum(r[1] for r in res), "decision_differs_outside_band": sum(r[2] for r in res),
        "band": "|z| < 1e-4", "seconds": round(time.perf_counter() - t0, 2), "threads": workers,
        "what": "oracle float64 forward with the trained weights on every held-out query with g = 1"}
    return out


def build_indicator(W, nb, synth):
    sc = W.scene
    if sc["type"] == "discs":
        return nb.Indicator.discs2d(synth.discs2d(W.seeds["scene"], k=sc["k"]))
    if sc["type"] == "metaball_voxels":
        seed = 1000 + sc.get("seed_of", W.index)
        c, r = synth.metaballs3d(seed, k=sc["k"], rlo=sc["rlo"], rhi=sc["rhi"])
        return nb.Indicator.metaball_voxels(c, r, sc["n"])
    if sc["type"] == "metaballs4d":
        a, b, r = synth.metaballs4d(W.seeds["scene"], k=sc["k"], rlo=sc["rlo"], rhi=sc["rhi"])
        return nb.Indicator.metaballs4d(a, b, r)
    raise ValueError(sc["type"])


def timed(fn, steps, warmup, torch):
    """(mean ms per call from HIP events around each call, wall seconds)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return float(np.mean([a.elapsed_time(b) for a, b in ev])), wall


def run_early_out(W, args, nb, synth, trainer, ind, bound, q, g, kind, prec, bound_ms, torch):
    """Neural early-out: a small bound trained on the same stream with the same
    schedule answers first; only its positives reach the workload's bound."""
    ew, enh = W.early
    small = nb.Bound(W.in_dim, enh, ew, prec)
    theta0 = synth.init_params(W.seeds["init"] + 100, W.in_dim, [ew] * enh)
    over = {"steps": args.train_steps} if args.train_steps is not None else {}
    if args.no_adapt:
        over["max_iters"] = 0
    sched = W.schedule(**over)
    small.set_params(theta0)
    nb.nb_bound_train_step(small.handle, ind.handle, kind, W.seeds["train"], 0, W.batch, 1.0)
    small.set_params(theta0)
    res = trainer.train(small, ind, W.kind, W.seeds["train"], sched, val_seed=W.seeds["val"],
                        log=lambda m: log(f"[{W.name} early] {m}"))
    n = q.shape[0]
    h = torch.empty(n, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    eo_ms, wall = timed(lambda: nb.nb_early_out(small.handle, bound.handle, q, h, cnt), args.steps, args.warmup, torch)
    small_counts = small.counts(q, g).tolist()
    tp = int(((h == 1) & (g == 1)).sum().item())
    fp = int(((h == 1) & (g == 0)).sum().item())
    fn = int(((h == 0) & (g == 1)).sum().item())
    second = int(cnt.item())
    log(f"[{W.name}] early-out: {eo_ms:.3f} ms vs {bound_ms:.3f} ms, second bound on {second / n:.3f} of the queries, "
        f"FN {fn} FP {fp}")
    return {"net": f"{W.in_dim}x{ew}^{enh}x1 then {W.in_dim}x{W.width}^{W.n_hidden}x1",
            "queries_per_s": n * args.steps / wall, "avg_ms": round(eo_ms, 4),
            "speedup_vs_bound": bound_ms / eo_ms, "second_bound_fraction": second / n,
            "early_train": {"steps": res.steps, "seconds": res.seconds, "validation_fn_zero": res.converged},
            "early_bound_heldout": dict(zip(["tp", "fp", "tn", "fn"], small_counts)),
            "heldout": {"n": n, "tp": tp, "fp": fp, "fn": fn, "fp_rate": fp / n}, "fn_zero": fn == 0}


def run_kdop(W, args, nb, synth, trainer, ind, q, g, bound_ms, torch):
    """The paper's OurkDOP: k slabs trained with the same loss and schedule."""
    kd = nb.KDop(W.dim, W.kdop_k)
    kd.set_params(synth.kdop_init(W.dim, W.kdop_k))
    over = {"steps": args.train_steps} if args.train_steps is not None else {}
    if args.no_adapt:
        over["max_iters"] = 0
    sched = W.schedule(**over)
    sched.lr = 3e-3
    res = trainer.train(kd, ind, W.kind, W.seeds["train"], sched, val_seed=W.seeds["val"],
                        log=lambda m: log(f"[{W.name} kdop] {m}"))
    n = q.shape[0]
    h = torch.empty(n, dtype=torch.uint8, device="cuda")
    ms, wall = timed(lambda: nb.nb_kdop_forward(kd.handle, nb.KINDS[W.kind], q, h=h), args.steps, args.warmup, torch)
    tp, fp, tn, fn = kd.counts(W.kind, q, g).tolist()
    log(f"[{W.name}] k-DOP (k={W.kdop_k}): {ms:.3f} ms, FN {fn} FP {fp}")
    return {"k": W.kdop_k, "queries_per_s": n * args.steps / wall, "avg_ms": round(ms, 4),
            "speedup_vs_bound": bound_ms / ms,
            "train": {"steps": res.steps, "seconds": res.seconds, "validation_fn_zero": res.converged},
            "heldout": {"n": n, "tp": tp, "fp": fp, "tn": tn, "fn": fn, "fp_rate": fp / n}, "fn_zero": fn == 0}


def run_workload(W, args, with_cpu: bool):
    import torch

    import paper_2310_06822_amd as nb
    import synth
    from paper_2310_06822_amd import autotune, trainer

    dev = "cuda"
    seeds = W.seeds
    widths = [W.width] * W.n_hidden
    kind = nb.KINDS[W.kind]
    prec = nb.BF16 if W.precision == "bf16" else nb.F32
    n_eval = args.eval_n if args.eval_n is not None else W.eval_n

    ind = build_indicator(W, nb, synth)
    bound = nb.Bound(W.in_dim, W.n_hidden, W.width, prec)
    if W.recompute:
        nb.nb_bound_set_recompute(bound.handle, W.recompute)
    if W.act == "sine":
        nb.nb_bound_set_activation(bound.handle, nb.SINE)
    if W.real_width:
        real = [W.real_width] * W.n_hidden
        theta0 = synth.pad_params(synth.init_params(seeds["init"], W.in_dim, real), W.in_dim, real, widths)
    else:
        theta0 = synth.init_params(seeds["init"], W.in_dim, widths)

    # ---- training (Alg. 1 on the device): ramp, then the step-wise schedule
    over = {"steps": args.train_steps} if args.train_steps is not None else {}
    if getattr(args, "lr_decay", None) is not None:
        over["lr_decay"] = args.lr_decay
    if getattr(args, "adapt_iters", None) is not None:
        over["max_iters"] = args.adapt_iters
    sched = W.schedule(**over)
    if args.no_adapt:
        sched.max_iters = 0
    bound.set_params(theta0)
    nb.nb_bound_train_step(bound.handle, ind.handle, kind, seeds["train"], 0, W.batch, 1.0)   # work space
    bound.set_params(theta0)
    res = trainer.train(bound, ind, W.kind, seeds["train"], sched, val_seed=seeds["val"],
                        log=lambda m: log(f"[{W.name}] {m}"))
    log(f"[{W.name}] train: {res.steps} steps x {W.batch} in {res.seconds:.2f} s -> {res.samples_per_s:.3e} "
        f"samples/s; alpha final {res.alpha_final:g}, schedule iterations {res.iters}, converged {res.converged}")

    # ---- held-out queries and exact answers
    q = torch.empty((n_eval, W.in_dim), dtype=torch.float32, device=dev)
    nb.nb_sample_queries(kind, W.dim, seeds["eval"], 0, q)
    g = torch.empty(n_eval, dtype=torch.uint8, device=dev)
    ind.query(W.kind, q, g)
    variant = autotune.tune(bound, q) if prec == nb.BF16 else 0
    counts = bound.counts(q, g)
    torch.cuda.synchronize()
    tp, fp, tn, fn = counts.tolist()
    log(f"[{W.name}] held-out {n_eval}: TP {tp} FP {fp} TN {tn} FN {fn} (forward variant {variant})")

    # ---- timed: bound forward + decision over the held-out set
    h = torch.empty(n_eval, dtype=torch.uint8, device=dev)
    kern_ms, wall = timed(lambda: nb.nb_bound_forward(bound.handle, q, nb.EPS_OUT, h=h), args.steps, args.warmup,
                          torch)
    value = n_eval * args.steps / wall

    # ---- exact test and cascade on the same queries, same GPU
    exact_ms, _ = timed(lambda: ind.query(W.kind, q, g), args.steps, args.warmup, torch)
    ans = torch.empty(n_eval, dtype=torch.uint8, device=dev)
    n_exact = torch.empty(1, dtype=torch.int64, device=dev)
    casc_ms, _ = timed(lambda: nb.nb_cascade(bound.handle, ind.handle, kind, q, ans, n_exact), args.steps,
                       args.warmup, torch)
    casc_ok = bool(torch.equal(ans, g))

    early = run_early_out(W, args, nb, synth, trainer, ind, bound, q, g, kind, prec, kern_ms, torch) if W.early else None
    kdop = run_kdop(W, args, nb, synth, trainer, ind, q, g, kern_ms, torch) if W.kdop_k else None

    wr = W.real_width or W.width   # algorithmic work of the network itself (not its zero padding)
    macs = W.in_dim * wr + (W.n_hidden - 1) * wr * wr + wr
    flop_per_q = 2 * macs
    peak = PEAK_TFLOPS[W.precision]
    achieved = flop_per_q * n_eval / (kern_ms / 1e3) / 1e12
    csrc = "paper_2310_06822_amd/csrc/"
    srcs = ([csrc + "mlp_bf16.hip", csrc + "nb_bf16_fwd.h", csrc + "nb_mlp.h"] if prec == nb.BF16
            else [csrc + "mlp_f32.hip", csrc + "nb_mlp.h"])
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4),
                "traffic": committed_traffic(f"{W.name}_forward_traffic.txt", srcs,
                                             bf16_forward_kernel(W.width, W.n_hidden, variant) if prec == nb.BF16
                                             else ""),
                "kernel": f"{bf16_forward_kernel(W.width, W.n_hidden, variant) if prec == nb.BF16 else 'k_fwd'} "
                          f"({W.precision} MLP forward + decision)",
                "flop_per_query": flop_per_q, "avg_launch_ms": round(kern_ms, 4)}
    out = {
        "value": value, "ms_per_step": wall * 1e3 / args.steps, "dtype": W.precision,
        "config": {"workload": W.name, "query": W.kind, "queries_per_step": n_eval,
                   "net": f"{W.in_dim}x{W.width}^{W.n_hidden}x1 relu {W.precision}",
                   "train_steps": res.steps, "train_batch": W.batch, "scene": W.scene,
                   "activation_checkpoint_interval": W.recompute, "activation": W.act,
                   "real_width": W.real_width or W.width},
        "train_samples_per_s": res.samples_per_s,
        "train": {"steps": res.steps, "batch": W.batch, "seconds": res.seconds, "alpha_final": res.alpha_final,
                  "schedule_iterations": res.iters, "validation_fn_zero": res.converged,
                  "validation_n": sched.val_n if sched.max_iters else 0,
                  "validation_fn_history": res.val_fn_history[-20:]},
        "exact_queries_per_s": n_eval / (exact_ms / 1e3),
        "bound_speedup_vs_exact": exact_ms / kern_ms,
        "cascade": {"queries_per_s": n_eval / (casc_ms / 1e3), "exact_tests": int(n_exact.item()),
                    "answer_equals_exact": casc_ok},
        "heldout": {"n": n_eval, "tp": tp, "fp": fp, "tn": tn, "fn": fn, "fp_rate": fp / n_eval},
        "fn_zero": fn == 0,
        "roofline": roofline,
    }
    if early:
        out["early_out"] = early
    if kdop:
        out["kdop"] = kdop
    if with_cpu:
        rows = torch.nonzero(g).flatten()
        out["cpu_baseline"] = cpu_baseline(W, bound.params().cpu().numpy(), q[:1 << 16].cpu().numpy(),
                                           q[rows].cpu().numpy(), h[rows].cpu().numpy())
    return out


def build_group(GW, nb, synth, torch):
    """The object set of a grouped workload on the device: grids voxelised
    per object, a Group with per-object initial weights."""
    objs = synth.object_set(GW.seeds["scene"], GW.n_obj, GW.grid_sizes, GW.widths, GW.k_range)
    sizes = [o["n"] for o in objs]
    grids = torch.empty(int(sum(n ** 3 for n in sizes)), dtype=torch.uint8, device="cuda")
    off = 0
    for o in objs:
        nb.nb_voxelize_metaballs(o["centres"], o["radii"], 1.0, o["n"], grids[off:off + o["n"] ** 3])
        off += o["n"] ** 3
    widths = [o["width"] for o in objs]
    group = nb.Group(GW.in_dim, widths, GW.n_hidden)
    group.set_voxels(grids, sizes)
    theta0 = np.concatenate([synth.init_params(GW.seeds["init"] * 1000 + i, GW.in_dim, [w] * GW.n_hidden)
                             for i, w in enumerate(widths)]).astype(np.float32)
    return group, objs, theta0


def run_group_workload(GW, args):
    import torch

    import paper_2310_06822_amd as nb
    import synth
    from paper_2310_06822_amd import autotune, trainer

    kind = nb.KINDS[GW.kind]
    group, objs, theta0 = build_group(GW, nb, synth, torch)
    widths = group.widths
    sched = trainer.Schedule(steps=args.train_steps if args.train_steps is not None else GW.train_steps,
                             batch=GW.per_obj, alpha_max=GW.alpha_max, k=GW.adapt_k, inc=GW.adapt_inc,
                             patience=GW.patience, max_iters=0 if args.no_adapt else GW.adapt_iters,
                             val_n=GW.val_per_obj, lr_decay=GW.lr_decay, cont_batch=GW.cont_batch)
    if getattr(args, "lr_decay", None) is not None:
        sched.lr_decay = args.lr_decay
    if getattr(args, "adapt_iters", None) is not None and not args.no_adapt:
        sched.max_iters = args.adapt_iters
    group.set_params(theta0)
    nb.nb_group_train_step(group.handle, group.n_obj, kind, GW.seeds["train"], 0, GW.per_obj, 1.0)   # work space
    group.set_params(theta0)
    res = trainer.train_group(group, GW.kind, GW.seeds["train"], sched, val_seed=GW.seeds["val"], log=log)
    log(f"[{GW.name}] train: {res.steps} steps x {GW.n_obj} x {GW.per_obj} in {res.seconds:.2f} s -> "
        f"{res.samples_per_s:.3e} samples/s; converged {res.converged}")

    per = args.eval_n // GW.n_obj if args.eval_n is not None else GW.eval_per_obj
    n_eval = per * GW.n_obj
    q = torch.empty((n_eval, GW.in_dim), dtype=torch.float32, device="cuda")
    nb.nb_sample_queries(kind, 3, GW.seeds["eval"], 0, q)
    qoff = torch.arange(0, n_eval + 1, per, dtype=torch.int64, device="cuda")
    g = torch.empty(n_eval, dtype=torch.uint8, device="cuda")
    nb.nb_group_query_exact(group.handle, group.n_obj, kind, q, qoff, g)
    variant = autotune.tune_group(group, q, qoff)
    cnt = group.counts(q, qoff, g).cpu().numpy()
    tp, fp, tn, fn = (int(x) for x in cnt.sum(0))
    fn_objects = [{"object": int(o), "width": widths[o], "grid": objs[o]["n"], "balls": objs[o]["k"],
                   "alpha": round(res.alpha_obj[o], 1) if res.alpha_obj else None, "fn": int(cnt[o, 3]),
                   "positives": int(cnt[o, 0] + cnt[o, 3])} for o in np.nonzero(cnt[:, 3])[0]]
    log(f"[{GW.name}] held-out {n_eval}: TP {tp} FP {fp} TN {tn} FN {fn}; objects with FN "
        f"{int((cnt[:, 3] > 0).sum())} (tile variant {variant})")

    h = torch.empty(n_eval, dtype=torch.uint8, device="cuda")
    kern_ms, wall = timed(lambda: nb.nb_group_forward(group.handle, group.n_obj, GW.in_dim, q, qoff, h=h),
                          args.steps, args.warmup, torch)
    exact_ms, _ = timed(lambda: nb.nb_group_query_exact(group.handle, group.n_obj, kind, q, qoff, g), args.steps,
                        args.warmup, torch)
    # the exact box test by its definition (scan every cell in the box)
    nb.nb_group_set_box_method(group.handle, nb.BOX_SCAN)
    g_scan = torch.empty_like(g)
    scan_ms, _ = timed(lambda: nb.nb_group_query_exact(group.handle, group.n_obj, kind, q, qoff, g_scan),
                       max(1, args.steps // 4), 1, torch)
    nb.nb_group_set_box_method(group.handle, nb.BOX_TABLE)
    scan_same = bool(torch.equal(g_scan, g))
    del g_scan

    def flop(w):
        return 2 * (GW.in_dim * w + (GW.n_hidden - 1) * w * w + w)

    total_flop = float(sum(flop(w) for w in widths)) * per
    achieved = total_flop / (kern_ms / 1e3) / 1e12
    # per width class: the same launch over that class's objects only
    by_width = {}
    for w in sorted(set(widths)):
        mask = np.array([x == w for x in widths])
        rows = torch.from_numpy(np.repeat(mask, per)).cuda()
        qc = q[rows].contiguous()
        counts_c = np.where(mask, per, 0)
        qoff_c = torch.from_numpy(np.concatenate([[0], np.cumsum(counts_c)]).astype(np.int64)).cuda()
        hc = torch.empty(qc.shape[0], dtype=torch.uint8, device="cuda")
        ms_c, _ = timed(lambda: nb.nb_group_forward(group.handle, group.n_obj, GW.in_dim, qc, qoff_c, h=hc),
                        args.steps, args.warmup, torch)
        f_c = flop(w) * qc.shape[0]
        by_width[str(w)] = {"objects": int(mask.sum()), "queries": int(qc.shape[0]), "ms": round(ms_c, 4),
                            "tflops": round(f_c / (ms_c / 1e3) / 1e12, 2),
                            "frac": round(f_c / (ms_c / 1e3) / 1e12 / PEAK_TFLOPS["bf16"], 4)}
        del qc, hc
    return {
        "bound_queries_per_s": n_eval * args.steps / wall,
        "config": {"workload": GW.name, "query": GW.kind, "objects": GW.n_obj, "queries_per_step": n_eval,
                   "net": f"{GW.in_dim}x{{32|64|128}}^{GW.n_hidden}x1 relu bf16, width per object",
                   "widths": {str(w): widths.count(w) for w in sorted(set(widths))},
                   "grids": {str(n): [o["n"] for o in objs].count(n) for n in GW.grid_sizes},
                   "train_per_object": GW.per_obj},
        "train_samples_per_s": res.samples_per_s,
        "train": {"steps": res.steps, "seconds": res.seconds, "schedule_iterations": res.iters,
                  "validation_fn_zero": res.converged, "validation_per_object": sched.val_n if sched.max_iters else 0,
                  "validation_fn_history": res.val_fn_history[-20:],
                  "objects_with_fn_history": res.objects_with_fn[-20:], "alpha_max_final": res.alpha_final},
        "exact_queries_per_s": n_eval / (exact_ms / 1e3),
        "exact_method": "count table per object (constant time per box)",
        "bound_speedup_vs_exact": exact_ms / kern_ms,
        "exact_scan_queries_per_s": n_eval / (scan_ms / 1e3),
        "bound_speedup_vs_exact_scan": scan_ms / kern_ms,
        "exact_scan_equals_table": scan_same,
        "heldout": {"n": n_eval, "tp": tp, "fp": fp, "tn": tn, "fn": fn, "fp_rate": fp / n_eval,
                    "objects_with_fn": int((cnt[:, 3] > 0).sum()), "fn_objects": fn_objects[:32]},
        "fn_zero": fn == 0,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["bf16"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["bf16"], 4), "traffic": None,
                     "kernel": "k_group_fwd (grouped bf16 forward + decision)", "avg_launch_ms": round(kern_ms, 4),
                     "tile_variant": variant, "by_width": by_width},
    }


def hier_tree(HW):
    """Breadth-first child ranges of the complete tree that splits space
    fan_axis ways per axis at each level, each node's level, and the lattice
    cell (x fastest) of each leaf."""
    f3 = HW.fan_axis ** 3
    first = [0]
    for d in range(HW.depth):
        first.append(first[-1] + f3 ** d)
    n_nodes = first[-1]
    cb, ce, level, leaf_cell = [0] * n_nodes, [0] * n_nodes, [0] * n_nodes, {}
    L = HW.lattice
    for d in range(HW.depth):
        for k in range(f3 ** d):
            v = first[d] + k
            level[v] = d
            if d + 1 < HW.depth:
                cb[v], ce[v] = first[d + 1] + k * f3, first[d + 1] + (k + 1) * f3
            else:
                x = y = z = 0
                for i in range(d):      # path digits, most significant first
                    j = (k // f3 ** (d - 1 - i)) % f3
                    a = HW.fan_axis
                    x = x * a + j % a
                    y = y * a + (j // a) % a
                    z = z * a + j // (a * a)
                leaf_cell[v] = x + L * (y + L * z)
    return cb, ce, level, leaf_cell


def run_hier_workload(HW, args):
    import torch

    import paper_2310_06822_amd as nb
    import synth
    from paper_2310_06822_amd import autotune, trainer

    cb, ce, level, leaf_cell = hier_tree(HW)
    n_nodes = len(cb)
    widths = [HW.widths[level[v]] for v in range(n_nodes)]
    objs = synth.lattice_objects(HW.seeds["scene"], HW.lattice, HW.k_range, HW.rlo, HW.rhi)
    cells = HW.n ** 3
    grids = torch.zeros(n_nodes * cells, dtype=torch.uint8, device="cuda")
    for v in reversed(range(n_nodes)):          # children before their parents
        gv = grids[v * cells:(v + 1) * cells]
        if cb[v] == ce[v]:
            c, r = objs[leaf_cell[v]]
            nb.nb_voxelize_metaballs(c, r, 1.0, HW.n, gv)
        else:
            for c in range(cb[v], ce[v]):
                torch.bitwise_or(gv, grids[c * cells:(c + 1) * cells], out=gv)
    group = nb.Group(3, widths, HW.n_hidden)
    group.set_voxels(grids, [HW.n] * n_nodes)
    occupancy = [float(grids[v * cells:(v + 1) * cells].float().mean()) for v in (0, 1, n_nodes - 1)]
    del grids
    theta0 = np.concatenate([synth.init_params(HW.seeds["init"] + v, 3, [w] * HW.n_hidden)
                             for v, w in enumerate(widths)]).astype(np.float32)
    sched = trainer.Schedule(steps=args.train_steps if args.train_steps is not None else HW.train_steps,
                             batch=HW.per_obj, alpha_max=HW.alpha_max, k=HW.adapt_k, inc=HW.adapt_inc,
                             patience=HW.patience, max_iters=0 if args.no_adapt else HW.adapt_iters,
                             val_n=HW.val_per_obj, lr_decay=HW.lr_decay)
    if getattr(args, "adapt_iters", None) is not None and not args.no_adapt:
        sched.max_iters = args.adapt_iters
    group.set_params(theta0)
    nb.nb_group_train_step(group.handle, n_nodes, nb.POINT, HW.seeds["train"], 0, HW.per_obj, 1.0)   # work space
    group.set_params(theta0)
    res = trainer.train_group(group, "point", HW.seeds["train"], sched, val_seed=HW.seeds["val"],
                              log=lambda m: log(f"[{HW.name}] {m}"))
    log(f"[{HW.name}] train: {res.steps} steps x {n_nodes} x {HW.per_obj} in {res.seconds:.2f} s -> "
        f"{res.samples_per_s:.3e} samples/s; converged {res.converged}")

    hier = nb.Hierarchy(group, cb, ce)
    n_eval = args.eval_n if args.eval_n is not None else HW.eval_n
    q = torch.empty((n_eval, 3), dtype=torch.float32, device="cuda")
    nb.nb_sample_queries(nb.POINT, 3, HW.seeds["eval"], 0, q)
    variant = autotune.tune_hierarchy(hier, q)
    hier_ms, wall = timed(lambda: hier.query(q), args.steps, args.warmup, torch)
    leaf_off, qidx = hier.query(q)
    pairs = hier.level_pairs()

    def flop(w):
        return 2 * (3 * w + (HW.n_hidden - 1) * w * w + w)

    hier_flop = float(sum(int(pairs[d]) * flop(HW.widths[d]) for d in range(HW.depth)))

    # every leaf's exact answer on the first m rows, against the pairs found
    m = min(HW.check_n, n_eval)
    leaves = [v for v in range(n_nodes) if cb[v] == ce[v]]
    nl = len(leaves)
    q_rep = q[:m].repeat(nl, 1)
    sizes = np.zeros(n_nodes, dtype=np.int64)
    sizes[leaves] = m
    qoff_rep = torch.from_numpy(np.concatenate([[0], np.cumsum(sizes)])).cuda()
    g_rep = torch.empty(nl * m, dtype=torch.uint8, device="cuda")
    nb.nb_group_query_exact(group.handle, n_nodes, nb.POINT, q_rep, qoff_rep, g_rep)
    loff = leaf_off.cpu().numpy()
    leaf_of_pair = torch.repeat_interleave(torch.arange(nl, device="cuda"),
                                           torch.from_numpy(np.diff(loff)).cuda())
    sel = qidx < m
    mark = torch.zeros((nl, m), dtype=torch.bool, device="cuda")
    mark[leaf_of_pair[sel], qidx[sel].long()] = True
    G = g_rep.view(nl, m).bool()
    fn = int((G & ~mark).sum())
    fp = int((mark & ~G).sum())
    tp = int((G & mark).sum())
    fn_leaves = int((G & ~mark).any(1).sum())
    # the flat alternative: every leaf's bound on every row (no tree), and
    # every leaf's exact test on every row
    h_rep = torch.empty(nl * m, dtype=torch.uint8, device="cuda")
    flat_ms, _ = timed(lambda: nb.nb_group_forward(group.handle, n_nodes, 3, q_rep, qoff_rep, h=h_rep),
                       args.steps, args.warmup, torch)
    flat_exact_ms, _ = timed(lambda: nb.nb_group_query_exact(group.handle, n_nodes, nb.POINT, q_rep, qoff_rep, g_rep),
                             args.steps, args.warmup, torch)
    flat_fn = int((G & ~h_rep.view(nl, m).bool()).sum())
    del q_rep, g_rep, h_rep, mark, G
    hier_rate = n_eval / (hier_ms / 1e3)
    log(f"[{HW.name}] hierarchy query {n_eval}: {hier_ms:.3f} ms ({hier_rate:.3e} q/s), pairs per level "
        f"{list(map(int, pairs))}, output {int(qidx.numel())}; FN {fn} over {fn_leaves} leaves, FP {fp} "
        f"(checked {m} rows x {nl} leaves); flat leaves {flat_ms * n_eval / m:.3f} ms-equivalent")
    achieved = hier_flop / (hier_ms / 1e3) / 1e12
    return {
        "bound_queries_per_s": hier_rate,
        "config": {"workload": HW.name, "query": "point", "nodes": n_nodes, "leaves": nl, "depth": HW.depth,
                   "tree": f"complete, {HW.fan_axis ** 3} children per node (space split {HW.fan_axis} ways per axis)",
                   "net": f"3x{{{'|'.join(map(str, HW.widths))}}}^{HW.n_hidden}x1 relu bf16, width per level",
                   "world_grid": HW.n, "occupancy_root_octant_leaf": [round(x, 5) for x in occupancy],
                   "queries_per_step": n_eval, "train_per_object": HW.per_obj},
        "ms_per_query_batch": hier_ms,
        "level_pairs": [int(x) for x in pairs],
        "output_pairs": int(qidx.numel()),
        "leaves_per_query": int(qidx.numel()) / n_eval,
        "train_samples_per_s": res.samples_per_s,
        "train": {"steps": res.steps, "seconds": res.seconds, "schedule_iterations": res.iters,
                  "validation_fn_zero": res.converged, "validation_fn_history": res.val_fn_history[-20:],
                  "objects_with_fn_history": res.objects_with_fn[-20:]},
        "heldout": {"rows": m, "leaves": nl, "tp": tp, "fp": fp, "fn": fn, "leaves_with_fn": fn_leaves,
                    "fp_rate_per_pair": fp / (m * nl), "flat_leaf_bounds_fn": flat_fn},
        "fn_zero": fn == 0,
        "flat_leaf_bounds_queries_per_s": m / (flat_ms / 1e3),
        "hierarchy_speedup_vs_flat_leaf_bounds": (flat_ms / m) / (hier_ms / n_eval),
        "flat_exact_queries_per_s": m / (flat_exact_ms / 1e3),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["bf16"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["bf16"], 4), "traffic": None,
                     "kernel": "nb_hier_query (grouped forward per level + scan + expansion; host sync per level)",
                     "flop": hier_flop, "tile_variant": variant},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="metaball4d_point")
    ap.add_argument("--also", action="store_true", help="also measure the other workloads")
    ap.add_argument("--train-steps", type=int, default=None)
    ap.add_argument("--eval-n", type=int, default=None)
    ap.add_argument("--no-adapt", action="store_true", help="ramp phase only (no step-wise continuation)")
    ap.add_argument("--adapt-iters", type=int, default=None, help="cap on step-wise scheduling iterations")
    ap.add_argument("--lr-decay", type=float, default=None,
                    help="learning-rate factor per scheduling iteration (default: the workload's)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (scales HBM byte counters in profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the bound's queries are "
              f"independent, so a multi-GPU run would shard them by rows", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_06822_amd.configs import GROUP_WORKLOADS, HIER_WORKLOADS, WORKLOADS

    torch.cuda.set_device(0)
    metric = "bound queries/s & train samples/s at FN=0 vs exact indicator test, same GPU"
    if args.workload not in WORKLOADS:
        # a grouped or hierarchical workload on its own (no CPU leg)
        if args.workload in GROUP_WORKLOADS:
            r = run_group_workload(GROUP_WORKLOADS[args.workload], args)
        elif args.workload in HIER_WORKLOADS:
            r = run_hier_workload(HIER_WORKLOADS[args.workload], args)
        else:
            sys.exit(f"unknown workload {args.workload}")
        value = r.pop("bound_queries_per_s")
        n = r["config"]["queries_per_step"]
        out = {"metric": metric, "value": value, "unit": "bound queries/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": n / value * 1e3, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "bf16", "data": "synthetic", "config": r.pop("config")}
        out.update(r)
        print(json.dumps(out), flush=True)
        return
    W = WORKLOADS[args.workload]
    r = run_workload(W, args, with_cpu=not args.no_cpu)
    out = {"metric": metric,
           "value": r.pop("value"), "unit": "bound queries/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": r.pop("ms_per_step"), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": r.pop("dtype"), "data": "synthetic",
           "config": r.pop("config")}
    out.update(r)
    if args.also:
        out["also"] = {}
        for name, W2 in WORKLOADS.items():
            if name == args.workload or not W2.bench_also:
                continue
            r2 = run_workload(W2, args, with_cpu=False)
            r2["bound_queries_per_s"] = r2.pop("value")
            out["also"][name] = r2
    if args.also:
        for name, GW in GROUP_WORKLOADS.items():
            out["also"][name] = run_group_workload(GW, args)
        for name, HW in HIER_WORKLOADS.items():
            out["also"][name] = run_hier_workload(HW, args)
    if args.copy_calibration:
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 2 x 256 MiB device-to-device copies")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
