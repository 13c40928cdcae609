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


def step_grad(theta, in_dim, widths, q, y, alpha, beta, bf16=False, lam1=0.0, lam2=0.0):
    """(loss, gradient) of Eq. 1 (+ regulariser) at theta on the batch (q, y)."""
    z = mlp.forward(theta, in_dim, widths, q, bf16=bf16)
    lv = L.loss(z, y, alpha, beta) + mlp.reg_value(theta, in_dim, widths, lam1, lam2)
    g = mlp.backward(theta, in_dim, widths, q, L.dloss_dz(z, y, alpha, beta), bf16=bf16)
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
