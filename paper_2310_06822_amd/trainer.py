"""Host-side training schedule around nb_bound_train_step (Alg. 1; Sec. 3.4).

Two phases, both run entirely on the GPU kernels:

1. Ramp: T steps with the FN weight alpha rising linearly from 1 to
   alpha_max and beta fixed (the cost of a false negative must grow without
   bound for the bound to become conservative, Sec. 3.1).
2. Step-wise continuation (Sec. 3.4, "Training", and the supplemental weight
   schedule): in scheduling iterations of K steps, alpha is incremented by
   `inc` after every iteration whose validation set still has a false
   negative; training stops once FN = 0 has held for `patience` consecutive
   iterations (six in the paper) or after `max_iters` iterations.  The
   validation set is drawn with its own seed, disjoint from the training
   stream and from any held-out test set.

Optional L1 + L2 regularisation ramps lambda linearly from 0 to lam_max over
the ramp phase and keeps it there (supplemental "Regularization").
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field

import torch

from . import KINDS, POINT, Bound, Indicator, nb_bound_train_step, nb_query_exact, nb_sample_queries


@dataclass
class Schedule:
    steps: int = 5000
    batch: int = 1 << 16
    alpha_max: float = 100.0
    beta: float = 1.0
    lr: float = 1e-3
    lam_max: float = 0.0
    # step-wise continuation (0 iterations disables it)
    k: int = 250
    inc: float = 50.0
    patience: int = 6
    max_iters: int = 400
    val_n: int = 1 << 24


@dataclass
class TrainResult:
    steps: int = 0
    samples: int = 0
    seconds: float = 0.0
    alpha_final: float = 0.0
    iters: int = 0
    val_fn_history: list = field(default_factory=list)
    converged: bool = False

    @property
    def samples_per_s(self) -> float:
        return self.samples / self.seconds if self.seconds > 0 else 0.0


def validation_set(ind: Indicator, kind: str, seed: int, n: int):
    k = KINDS[kind]
    d = ind.dim if k == POINT else 6
    q = torch.empty((n, d), dtype=torch.float32, device="cuda")
    nb_sample_queries(k, ind.dim, seed, 0, q)
    g = torch.empty(n, dtype=torch.uint8, device="cuda")
    nb_query_exact(ind.handle, k, q, g)
    return q, g


def train(bound: Bound, ind: Indicator, kind: str, seed: int, sched: Schedule, val_seed: int | None = None,
          log=None) -> TrainResult:
    k = KINDS[kind]
    res = TrainResult()
    val = validation_set(ind, kind, val_seed, sched.val_n) if (val_seed is not None and sched.max_iters > 0) else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = sched.steps
    step = 0
    for t in range(T):
        frac = t / (T - 1) if T > 1 else 1.0
        a = 1.0 + (sched.alpha_max - 1.0) * frac
        lam = sched.lam_max * frac
        nb_bound_train_step(bound.handle, ind.handle, k, seed, step, sched.batch, a, sched.beta, sched.lr, lam, lam)
        step += 1
    a = sched.alpha_max
    lam = sched.lam_max
    if val is not None:
        ok = 0
        while ok < sched.patience and res.iters < sched.max_iters:
            for _ in range(sched.k):
                nb_bound_train_step(bound.handle, ind.handle, k, seed, step, sched.batch, a, sched.beta, sched.lr,
                                    lam, lam)
                step += 1
            fn = int(bound.counts(*val)[3].item())
            res.val_fn_history.append(fn)
            res.iters += 1
            if fn == 0:
                ok += 1
            else:
                ok = 0
                a += sched.inc
            if log:
                log(f"schedule iteration {res.iters}: step {step} alpha {a:g} validation FN {fn}")
        res.converged = ok >= sched.patience
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    res.steps = step
    res.samples = step * sched.batch
    res.alpha_final = a
    return res
