"""Asymmetric loss, decision and confusion counts (test infrastructure).

Eq. 1: L = -E_i[ alpha(t) y_i log yhat_i + beta(t) (1 - y_i) log(1 - yhat_i) ]
with yhat = sigmoid(z).  Written on logits:
    -log sigmoid(z)     = softplus(-z)
    -log(1 - sigmoid(z)) = softplus(z)
so l_i = alpha y_i softplus(-z_i) + beta (1 - y_i) softplus(z_i) and L is the
plain mean over the batch.  The ideal cost of Sec. 3.1 charges alpha for a
false negative (g = 1, h = 0) and beta for a false positive (g = 0, h = 1).

Decision (Sec. 3.4 "Architecture": sigmoid, then rounding to {0,1}; the
supplemental "Numerics" adds an epsilon of 1e-5 to the output): h = 1 iff
sigmoid(z) + eps >= 1/2, i.e. iff z >= tau = ln((1/2 - eps) / (1/2 + eps)).
Ties and NaN count as positive (the conservative side).  The comparison is
made in float32 against tau rounded to float32.
"""

from __future__ import annotations

import numpy as np

EPS_OUT = 1e-5


def softplus(x):
    x = np.asarray(x, dtype=np.float64)
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def sigmoid(x):
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(-np.abs(x))
    return np.where(x >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def loss(z, y, alpha: float, beta: float) -> float:
    """Eq. 1, mean over the batch (float64)."""
    y = np.asarray(y, dtype=np.float64)
    li = alpha * y * softplus(-np.asarray(z, np.float64)) + beta * (1.0 - y) * softplus(z)
    return float(li.mean())


def dloss_dz(z, y, alpha: float, beta: float) -> np.ndarray:
    """dL/dz_i = (beta (1 - y_i) sigmoid(z_i) - alpha y_i (1 - sigmoid(z_i))) / B."""
    y = np.asarray(y, dtype=np.float64)
    s = sigmoid(z)
    return (beta * (1.0 - y) * s - alpha * y * (1.0 - s)) / y.shape[0]


def tau(eps: float = EPS_OUT) -> float:
    """Logit threshold equivalent to sigmoid(z) + eps >= 1/2 (float64)."""
    return float(np.log((0.5 - eps) / (0.5 + eps)))


def decide(z, eps: float = EPS_OUT) -> np.ndarray:
    """h = not (z < tau) in float32; NaN -> 1."""
    z32 = np.asarray(z).astype(np.float32)
    return (~(z32 < np.float32(tau(eps)))).astype(np.uint8)


def counts(h, g) -> np.ndarray:
    """uint64[4] = (TP, FP, TN, FN) of decisions h against exact answers g.
    Rates divide by the number of all queries."""
    h = np.asarray(h).astype(bool)
    g = np.asarray(g).astype(bool)
    return np.array([(h & g).sum(), (h & ~g).sum(), (~h & ~g).sum(), (~h & g).sum()],
                    dtype=np.uint64)
