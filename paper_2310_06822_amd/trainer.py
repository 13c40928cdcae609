"""Host-side training schedule around nb_bound_train_step (Alg. 1; Sec. 3.4).

Two phases, both run entirely on the GPU kernels:

1. Ramp: T steps with the FN weight alpha rising linearly from 1 to
   alpha_max and beta fixed (the cost of a false negative must grow without
   bound for the bound to become conservative, Sec. 3.1).
2. Step-wise continuation (Sec. 3.4, "Training", and the supplemental weight
   schedule): in scheduling iterations of K steps, alpha is incremented by
   `inc` after every iteration whose validation set still has a false
   negative; training stops once FN = 0 has held for `patience` consecutive
   iterations (six in the paper) or after `max_iters` iterations.  Every
   iteration checks a fresh validation draw (its own seed, the iteration
   number as the sampler's step), disjoint from the training stream and from
   any held-out test set, so six FN-free iterations have seen six distinct
   validation sets.

Optional L1 + L2 regularisation ramps lambda linearly from 0 to lam_max over
the ramp phase and keeps it there (supplemental "Regularization").
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field

import torch

from . import KINDS, POINT, Bound, Indicator, KDop, nb_bound_train_step, nb_kdop_train_step, nb_query_exact, \
    nb_sample_queries


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
    lr_decay: float = 1.0     # learning-rate factor per continuation iteration (1: constant)
    lr_min: float = 1e-5
    # inverted ("certainly hit") bound: the FP weight follows the schedule and
    # the continuation counts false positives, so h = 1 implies g = 1
    inverted: bool = False
    # groups: per-object batch of the continuation (0: the ramp's), which
    # trains only the objects still in training
    cont_batch: int = 0


@dataclass
class TrainResult:
    steps: int = 0
    samples: int = 0
    seconds: float = 0.0
    alpha_final: float = 0.0
    iters: int = 0
    val_fn_history: list = field(default_factory=list)
    alpha_history: list = field(default_factory=list)   # FN weight of each continuation iteration's steps
    lr_history: list = field(default_factory=list)      # learning rate of each continuation iteration's steps
    converged: bool = False

    @property
    def samples_per_s(self) -> float:
        return self.samples / self.seconds if self.seconds > 0 else 0.0


class Continuation:
    """State of the step-wise continuation of one bound: the FN weight and
    learning rate its next K steps use, and the stopping rule.  After each
    iteration, update() takes that iteration's validation FN count: a false
    negative raises alpha by `inc` and resets the FN-free run; `patience`
    FN-free iterations in a row (six in the paper) or `max_iters` iterations
    end the schedule.  The learning rate is multiplied by lr_decay after
    every iteration, down to lr_min."""

    def __init__(self, sched: Schedule, alpha: float):
        self.s = sched
        self.alpha = float(alpha)
        self.lr = float(sched.lr)
        self.run = 0
        self.iters = 0

    @property
    def converged(self) -> bool:
        return self.run >= self.s.patience

    @property
    def done(self) -> bool:
        return self.converged or self.iters >= self.s.max_iters

    def update(self, fn: int):
        self.lr = max(self.s.lr_min, self.lr * self.s.lr_decay)
        self.iters += 1
        if fn == 0:
            self.run += 1
        else:
            self.run = 0
            self.alpha += self.s.inc


class GroupContinuation:
    """The continuation of a group of bounds: per-object FN weights (raised
    after each iteration in which the object shows a validation FN) and
    learning rates (0 for an object FN-free for `patience` iterations in a
    row, until a later draw shows it a false negative again; the others take
    the decayed rate).  The group stops once its whole validation draw has
    been FN-free for `patience` iterations in a row, or after max_iters."""

    def __init__(self, sched: Schedule, n_obj: int):
        import numpy as np
        self.s = sched
        self.alpha = np.full(n_obj, sched.alpha_max, dtype=np.float32)
        self.lr = np.full(n_obj, sched.lr, dtype=np.float32)
        self.clean = np.zeros(n_obj, dtype=np.int64)
        self.lr_now = float(sched.lr)
        self.clean_all = 0
        self.iters = 0

    @property
    def converged(self) -> bool:
        return self.clean_all >= self.s.patience

    @property
    def done(self) -> bool:
        return self.converged or self.iters >= self.s.max_iters

    def update(self, fn):
        import numpy as np
        bad = np.asarray(fn) > 0
        self.lr_now = max(self.s.lr_min, self.lr_now * self.s.lr_decay)
        self.alpha[bad] += self.s.inc
        self.lr[(self.lr > 0) | bad] = self.lr_now
        self.clean[bad] = 0
        self.clean[~bad] += 1
        self.lr[self.clean >= self.s.patience] = 0.0
        self.clean_all = 0 if bad.any() else self.clean_all + 1
        self.iters += 1
        return bad


def validation_set(ind: Indicator, kind: str, seed: int, n: int, draw: int = 0, out=None):
    """Validation regions (draw `draw` of the stream `seed`) and their exact
    answers; refills `out` = (q, g) when given."""
    k = KINDS[kind]
    d = ind.dim if k == POINT else 6
    q, g = out if out is not None else (torch.empty((n, d), dtype=torch.float32, device="cuda"),
                                        torch.empty(n, dtype=torch.uint8, device="cuda"))
    nb_sample_queries(k, ind.dim, seed, draw, q)
    nb_query_exact(ind.handle, k, q, g)
    return q, g


def train(bound, ind: Indicator, kind: str, seed: int, sched: Schedule, val_seed: int | None = None,
          log=None) -> TrainResult:
    """Train a Bound (or a KDop: its planes take the same loss and schedule)."""
    k = KINDS[kind]
    if isinstance(bound, KDop):
        from . import nb_kdop_sync as sync

        def nb_bound_train_step(h, ih, kk, sd, st, batch, a, b, lr, lam1, lam2):
            nb_kdop_train_step(h, ih, kk, sd, st, batch, a, b, lr)

        def counts(q, g):
            return bound.counts(kind, q, g)
    else:
        from . import nb_bound_train_step
        from . import nb_bound_sync as sync

        def counts(q, g):
            return bound.counts(q, g)
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
        fn_w, fp_w = (sched.beta, a) if sched.inverted else (a, sched.beta)
        nb_bound_train_step(bound.handle, ind.handle, k, seed, step, sched.batch, fn_w, fp_w, sched.lr, lam, lam)
        step += 1
        if log and (t + 1) % 1000 == 0:
            sync(bound.handle)   # raises if a step met a non-finite loss or gradient
            log(f"ramp step {t + 1}/{T}: alpha {a:g}")
    sync(bound.handle)
    a = sched.alpha_max
    lam = sched.lam_max
    if val is not None:
        cont = Continuation(sched, a)
        while not cont.done:
            fn_w, fp_w = (sched.beta, cont.alpha) if sched.inverted else (cont.alpha, sched.beta)
            res.alpha_history.append(cont.alpha)
            res.lr_history.append(cont.lr)
            for _ in range(sched.k):
                nb_bound_train_step(bound.handle, ind.handle, k, seed, step, sched.batch, fn_w, fp_w, cont.lr,
                                    lam, lam)
                step += 1
            sync(bound.handle)
            val = validation_set(ind, kind, val_seed, sched.val_n, draw=cont.iters, out=val)
            # the error the bound must not make: FN, or FP for an inverted bound
            fn = int(counts(*val)[1 if sched.inverted else 3].item())
            res.val_fn_history.append(fn)
            cont.update(fn)
            if log:
                log(f"schedule iteration {cont.iters}: step {step} alpha {cont.alpha:g} validation FN {fn}")
        res.iters = cont.iters
        res.converged = cont.converged
        a = cont.alpha
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    res.steps = step
    res.samples = step * sched.batch
    res.alpha_final = a
    return res


# ------------------------------------------------------------------ groups

@dataclass
class GroupTrainResult(TrainResult):
    alpha_obj: list = field(default_factory=list)       # final per-object FN weights
    objects_with_fn: list = field(default_factory=list)  # per iteration: objects whose validation FN > 0
    fn_obj_history: list = field(default_factory=list)   # per iteration: each object's validation FN


def group_validation_set(group, kind: str, seed: int, per_obj: int, draw: int = 0, out=None):
    """per_obj regions per object (object o: rows o*per_obj ..; draw `draw`
    of the stream `seed`) and their exact answers on each object's own grid;
    refills `out` = (q, qoff, g) when given."""
    from . import nb_group_query_exact
    k = KINDS[kind]
    n = group.n_obj * per_obj
    if out is None:
        out = (torch.empty((n, 3 if k == POINT else 6), dtype=torch.float32, device="cuda"),
               torch.arange(0, n + 1, per_obj, dtype=torch.int64, device="cuda"),
               torch.empty(n, dtype=torch.uint8, device="cuda"))
    q, qoff, g = out
    nb_sample_queries(k, 3, seed, draw, q)
    nb_group_query_exact(group.handle, group.n_obj, k, q, qoff, g)
    return q, qoff, g


def train_group(group, kind: str, seed: int, sched: Schedule, val_seed: int | None = None,
                log=None) -> GroupTrainResult:
    """Alg. 1 for every object of a group at once.  Ramp: alpha rises
    linearly 1 -> alpha_max for all objects.  Continuation in iterations of k
    steps, each followed by a fresh validation draw of sched.val_n regions
    per object: an object with a false negative gets alpha += inc (and
    trains); an object FN-free for `patience` iterations in a row stops
    training (learning rate 0) until a later draw shows it a false negative
    again.  Training ends once the whole group has been FN-free for
    `patience` iterations in a row (the paper's stopping rule applied to all
    of the group's validation regions), or after max_iters iterations.
    sched.batch is the per-object batch."""
    import numpy as np

    from . import nb_group_set_active, nb_group_sync, nb_group_train_step
    k = KINDS[kind]
    res = GroupTrainResult()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = sched.steps
    step = 0
    for t in range(T):
        a = 1.0 + (sched.alpha_max - 1.0) * (t / (T - 1) if T > 1 else 1.0)
        nb_group_train_step(group.handle, group.n_obj, k, seed, step, sched.batch, a, sched.beta, sched.lr)
        step += 1
        if log and (t + 1) % 1000 == 0:
            nb_group_sync(group.handle)   # raises if a step met a non-finite gradient
            log(f"group ramp step {t + 1}/{T}: alpha {a:g}")
    nb_group_sync(group.handle)
    samples = step * sched.batch * group.n_obj
    cont = GroupContinuation(sched, group.n_obj)
    if val_seed is not None and sched.max_iters > 0:
        val = None
        a_dev = torch.from_numpy(cont.alpha).cuda()
        lr_dev = torch.from_numpy(cont.lr).cuda()
        while not cont.done:
            active = cont.lr > 0
            res.alpha_history.append(cont.alpha.copy())
            res.lr_history.append(cont.lr.copy())
            if active.any():
                # only the objects still training are evaluated and updated
                nb_group_set_active(group.handle, active.astype(np.uint8))
                for _ in range(sched.k):
                    nb_group_train_step(group.handle, group.n_obj, k, seed, step, sched.cont_batch or sched.batch,
                                        0.0, sched.beta, sched.lr, alpha_obj=a_dev, lr_obj=lr_dev)
                    step += 1
                samples += sched.k * (sched.cont_batch or sched.batch) * int(active.sum())
            nb_group_sync(group.handle)
            val = group_validation_set(group, kind, val_seed, sched.val_n, draw=cont.iters, out=val)
            fn = group.counts(*val)[:, 3].cpu().numpy()
            bad = cont.update(fn)
            a_dev.copy_(torch.from_numpy(cont.alpha))
            lr_dev.copy_(torch.from_numpy(cont.lr))
            res.val_fn_history.append(int(fn.sum()))
            res.objects_with_fn.append(int(bad.sum()))
            res.fn_obj_history.append(fn.copy())
            if log:
                log(f"group schedule iteration {cont.iters}: step {step}, validation FN {int(fn.sum())} over "
                    f"{int(bad.sum())} objects, {int((cont.lr > 0).sum())} training, alpha max {cont.alpha.max():g}")
        res.iters = cont.iters
        res.converged = cont.converged
        nb_group_set_active(group.handle, None)
    torch.cuda.synchronize()
    res.seconds = time.perf_counter() - t0
    res.steps = step
    res.samples = samples
    res.alpha_final = float(cont.alpha.max())
    res.alpha_obj = cont.alpha.tolist()
    return res
