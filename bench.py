"""Throughput of the Neural Bounding hot path on one GPU.

Workload (default): 3-D point queries against a 128^3 voxel grid of 16 seeded
metaballs; bound 3 -> 64^3 -> 1 (ReLU, float32 on the matrix cores); trained
for 5000 Adam steps on batches of 2^16 regions drawn and labelled on the
device, with the FN weight ramped 1 -> 100; evaluated on 2^24 held-out
queries (disjoint seed).

A timed step is one pass of the deployed bound over the 2^24 held-out queries
(forward + decision, all resident in HBM).  Reported beside it: training
samples/s over the whole training run, the exact indicator test on the same
queries and GPU, FN / FP on the held-out set, the roofline of the forward
kernel, and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_MFMA_PEAK_TFLOPS = 157.3     # MI355X dense FP32 matrix peak
HBM_PEAK_GBS = 8000.0


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def committed_traffic(name: str, source: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None
    if the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    sha = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()
    if kv.get("source_sha256") != sha:
        return None
    try:
        return int(float(kv["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def cpu_baseline(theta, in_dim, widths, target_s: float = 10.0):
    """Oracle forward + decision on a bounded sample of held-out queries."""
    import synth
    from oracle import loss as L, mlp
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    chunk = 1 << 16
    q = synth.points(3001, chunk, in_dim)
    t0 = time.perf_counter()
    L.decide(mlp.forward(theta, in_dim, widths, q))
    dt = time.perf_counter() - t0
    reps = max(1, int(target_s / max(dt, 1e-3)))
    t0 = time.perf_counter()
    for _ in range(reps):
        L.decide(mlp.forward(theta, in_dim, widths, q))
    dt = time.perf_counter() - t0
    return {"value": reps * chunk / dt, "unit": "bound queries/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{reps} x {chunk} held-out queries, float64 numpy forward + decision, "
                      f"{dt:.1f} s on {os.cpu_count()} host cores"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--train-steps", type=int, default=None)
    ap.add_argument("--eval-n", type=int, default=None)
    ap.add_argument("--no-adapt", action="store_true", help="ramp phase only (no step-wise continuation)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (scales HBM byte counters in profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the bound's queries are "
              f"independent, so a multi-GPU run would shard them by rows", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2310_06822_amd as nb
    import synth
    from paper_2310_06822_amd.configs import VOXEL3D_POINT as W

    torch.cuda.set_device(0)
    dev = "cuda"
    n_eval = args.eval_n if args.eval_n is not None else W.eval_n
    seeds = W.seeds
    widths = [W.width] * W.n_hidden

    # scene: metaball field voxelised on the GPU
    c, r = synth.metaballs3d(seeds["scene"], k=W.scene["k"], rlo=W.scene["rlo"], rhi=W.scene["rhi"])
    gn = W.scene["n"]
    grid = torch.empty(gn ** 3, dtype=torch.uint8, device=dev)
    nb.nb_voxelize_metaballs(c, r, 1.0, gn, grid)
    ind = nb.Indicator.voxels(grid, gn)
    log(f"scene: {gn}^3 grid, occupancy {grid.float().mean().item():.4f}")

    bound = nb.Bound(W.in_dim, W.n_hidden, W.width)
    theta0 = synth.init_params(seeds["init"], W.in_dim, widths)
    bound.set_params(theta0)

    # ---- training (Alg. 1 on the device): ramp, then the step-wise schedule
    from paper_2310_06822_amd import trainer
    sched = W.schedule(**({"steps": args.train_steps} if args.train_steps is not None else {}))
    if args.no_adapt:
        sched.max_iters = 0
    nb.nb_bound_train_step(bound.handle, ind.handle, nb.POINT, seeds["train"], 0, W.batch, 1.0)   # work space
    bound.set_params(theta0)
    res = trainer.train(bound, ind, W.kind, seeds["train"], sched, val_seed=seeds["val"], log=None)
    train_sps = res.samples_per_s
    log(f"train: {res.steps} steps x {W.batch} in {res.seconds:.2f} s -> {train_sps:.3e} samples/s; "
        f"alpha final {res.alpha_final:g}, schedule iterations {res.iters}, converged {res.converged}")

    # ---- held-out queries and exact answers
    q = torch.empty((n_eval, W.in_dim), dtype=torch.float32, device=dev)
    nb.nb_sample_queries(nb.POINT, W.dim, seeds["eval"], 0, q)
    g = torch.empty(n_eval, dtype=torch.uint8, device=dev)
    ind.query("point", q, g)
    counts = bound.counts(q, g)
    torch.cuda.synchronize()
    tp, fp, tn, fn = counts.tolist()
    log(f"held-out {n_eval}: TP {tp} FP {fp} TN {tn} FN {fn}")

    # ---- timed: bound forward + decision over the held-out set
    h = torch.empty(n_eval, dtype=torch.uint8, device=dev)

    def step():
        nb.nb_bound_forward(bound.handle, q, nb.EPS_OUT, h=h)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    ms_step = wall * 1e3 / args.steps
    avg_kern = float(np.mean(kern_ms))
    value = n_eval * args.steps / wall

    # ---- exact test on the same queries, same GPU
    for _ in range(args.warmup):
        ind.query("point", q, g)
    torch.cuda.synchronize()
    x0, x1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    x0.record()
    for _ in range(args.steps):
        ind.query("point", q, g)
    x1.record()
    torch.cuda.synchronize()
    exact_ms = x0.elapsed_time(x1) / args.steps
    exact_qps = n_eval / (exact_ms / 1e3)

    macs = W.in_dim * W.width + (W.n_hidden - 1) * W.width * W.width + W.width
    flop_per_q = 2 * macs
    achieved = flop_per_q * n_eval / (avg_kern / 1e3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_MFMA_PEAK_TFLOPS, 4),
                "traffic": committed_traffic("k_fwd_f32_voxel3d_point_traffic.txt",
                                             "paper_2310_06822_amd/csrc/mlp_f32.hip"),
                "kernel": "k_fwd<1,64,3> (float32 MLP forward + decision)",
                "flop_per_query": flop_per_q, "avg_launch_ms": round(avg_kern, 4)}

    out = {
        "metric": "bound queries/s & train samples/s at FN=0 vs exact indicator test, same GPU",
        "value": value, "unit": "bound queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": W.name, "queries_per_step": n_eval, "grid": gn, "metaballs": W.scene["k"],
                   "net": f"{W.in_dim}x{W.width}^{W.n_hidden}x1 relu", "train_steps": res.steps, "train_batch": W.batch},
        "train_samples_per_s": train_sps,
        "train": {"steps": res.steps, "batch": W.batch, "seconds": res.seconds, "alpha_final": res.alpha_final,
                  "schedule_iterations": res.iters, "validation_fn_zero": res.converged,
                  "validation_n": sched.val_n if sched.max_iters else 0},
        "exact_queries_per_s": exact_qps,
        "bound_vs_exact": value / exact_qps,
        "heldout": {"n": n_eval, "tp": tp, "fp": fp, "tn": tn, "fn": fn, "fp_rate": fp / n_eval},
        "fn_zero": fn == 0,
        "roofline": roofline,
    }
    if args.copy_calibration:
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 2 x 256 MiB device-to-device copies")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(bound.params().cpu().numpy(), W.in_dim, widths)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
