"""Training loop of Alg. 1 (test infrastructure; see oracle/__init__).

Each step follows Alg. 1 in its order: draw regions uniformly (oracle.sampling
with the step number as part of the counter), label them with the exact
query (y = any of the indicator over the region), evaluate the bound, take
the weighted BCE of Eq. 1 and one Adam step (Sec. 3.4 "Training").

FN-weight schedule (Sec. 3.1: the FN cost must grow without bound; Sec. 3.4:
a linear step-wise schedule).  Default: alpha ramps linearly from 1 to 100
over the run, alpha(t) = 1 + 99 t / (T - 1), with beta = 1.

Optional L1 + L2 regularisation on the weight matrices, lambda ramping
linearly from 0 to lam_max over the run (supplemental "Regularization").

Parity: one step is pinned piece by piece (sampling, labels, loss, gradient,
Adam); a trajectory longer than a few steps is chaotic and its parity is
unpinned beyond k <= 10 steps.
"""

from __future__ import annotations

import numpy as np

from . import loss as L
from . import mlp
from . import sampling
from .adam import Adam


def alpha_ramp(t: int, T: int, a0: float = 1.0, a1: float = 100.0) -> float:
    return a0 + (a1 - a0) * (t / (T - 1) if T > 1 else 1.0)


def lam_ramp(t: int, T: int, lam_max: float) -> float:
    return lam_max * (t / (T - 1) if T > 1 else 1.0)


def step_grad(theta, in_dim, widths, q, y, alpha, beta, bf16=False, lam1=0.0, lam2=0.0, act="relu"):
    """(loss, gradient) of Eq. 1 (+ regulariser) at theta on the batch (q, y)."""
    z = mlp.forward(theta, in_dim, widths, q, bf16=bf16, act=act)
    lv = L.loss(z, y, alpha, beta) + mlp.reg_value(theta, in_dim, widths, lam1, lam2)
    g = mlp.backward(theta, in_dim, widths, q, L.dloss_dz(z, y, alpha, beta), bf16=bf16, act=act)
    if lam1 or lam2:
        g = g + mlp.reg_grad(theta, in_dim, widths, lam1, lam2)
    return lv, g, z


def train(label_fn, kind: str, dim: int, in_dim: int, widths, theta0, seed: int,
          steps: int, batch: int, a_max: float = 100.0, beta: float = 1.0,
          lr: float = 1e-3, bf16: bool = False, lam_max: float = 0.0,
          log=None):
    """Run `steps` steps of Alg. 1.  label_fn maps a query batch to uint8 g.
    Returns (theta float64, list of per-step (loss, TP, FP, TN, FN))."""
    theta = np.asarray(theta0, dtype=np.float64).copy()
    opt = Adam(theta.size, lr=lr)
    hist = []
    for t in range(steps):
        q = sampling.sample(kind, seed, t, batch, dim)
        y = label_fn(q)
        a = alpha_ramp(t, steps, 1.0, a_max)
        lam = lam_ramp(t, steps, lam_max)
        lv, g, z = step_grad(theta, in_dim, widths, q, y, a, beta, bf16, lam, lam)
        hist.append((lv, *L.counts(L.decide(z), y).tolist()))
        theta = opt.step(theta, g)
        if log is not None:
            log(t, hist[-1])
    return theta, hist


# ------------------------------------------------------------ continuation

def continuation(fn_trace, alpha0: float, inc: float, lr0: float, patience: int = 6, max_iters: int = 400,
                 lr_decay: float = 1.0, lr_min: float = 0.0):
    """The step-wise FN-weight schedule after the ramp (Sec. 3.4 "Training";
    supplemental "Weight schedule"), as a function of the validation FN
    counts.  Scheduling iteration i trains K steps with FN weight alpha_i and
    learning rate lr_i and then counts the false negatives fn_trace[i] on a
    fresh validation draw.  The weight is stepped up by `inc` after every
    iteration that still shows a false negative (the supplemental raises the
    FN:FP ratio linearly "if not 0 FNs"); training stops early once FN = 0 has
    held for the last `patience` iterations (six in the paper), and in any
    case after max_iters iterations.  The learning rate of iteration i is
    max(lr_min, lr0 * lr_decay^i) (lr_decay = 1: the paper's constant rate).

    Returns dict(alpha=[alpha_i], lr=[lr_i], iters, converged, alpha_final),
    the lists holding the values iterations 0 .. iters-1 trained with."""
    alphas, lrs = [], []
    alpha = float(alpha0)
    i = 0
    while i < max_iters:
        alphas.append(alpha)
        lrs.append(max(lr_min, lr0 * lr_decay ** i))
        if fn_trace[i] > 0:
            alpha += inc
        i += 1
        # FN = 0 on each of the last `patience` validation draws
        if i >= patience and all(f == 0 for f in fn_trace[i - patience:i]):
            return dict(alpha=alphas, lr=lrs, iters=i, converged=True, alpha_final=alpha)
    return dict(alpha=alphas, lr=lrs, iters=i, converged=False, alpha_final=alpha)


def group_continuation(fn_trace, alpha0: float, inc: float, lr0: float, patience: int = 6, max_iters: int = 400,
                       lr_decay: float = 1.0, lr_min: float = 0.0):
    """The same schedule for a group of bounds trained side by side, one
    network per object (Sec. 3.4 "Training"): fn_trace[i][o] is object o's
    validation FN count after iteration i.  Each object's FN weight steps up
    after each iteration in which it shows a false negative.  An object whose
    last `patience` draws were FN-free has met the paper's stopping rule and
    does not train (learning rate 0) until a later draw shows it a false
    negative; every other object trains with the iteration's rate
    max(lr_min, lr0 * lr_decay^i).  The group stops once all objects were
    FN-free on the last `patience` draws, or after max_iters iterations.

    Returns dict(alpha=[[alpha_io]], lr=[[lr_io]], iters, converged,
    alpha_final=[alpha_o])."""
    n_obj = len(fn_trace[0])
    alpha = [float(alpha0)] * n_obj
    alphas, lrs = [], []
    i = 0
    while i < max_iters:
        rate = max(lr_min, lr0 * lr_decay ** i)
        row = []
        for o in range(n_obj):
            # stopped: FN-free on each of the last `patience` draws
            stopped = i >= patience and all(fn_trace[j][o] == 0 for j in range(i - patience, i))
            row.append(0.0 if stopped else rate)
        alphas.append(list(alpha))
        lrs.append(row)
        for o in range(n_obj):
            if fn_trace[i][o] > 0:
                alpha[o] += inc
        i += 1
        if i >= patience and all(fn_trace[j][o] == 0 for j in range(i - patience, i) for o in range(n_obj)):
            return dict(alpha=alphas, lr=lrs, iters=i, converged=True, alpha_final=alpha)
    return dict(alpha=alphas, lr=lrs, iters=i, converged=False, alpha_final=alpha)
