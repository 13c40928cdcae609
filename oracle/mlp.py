"""The bound h_theta as an MLP (test infrastructure; see oracle/__init__).

Sec. 3.4 ("Architecture"): h_theta is an MLP whose single output is squashed
by a sigmoid and rounded to {0, 1}.  Layer sizes are written "a x b x c"
(supplemental architecture tables) and mean in_dim -> hidden widths -> 1
output logit, with a bias on every layer; the 3 x 50 x 50 network then has
the 2,801 parameters the paper quotes (Sec. 6, "Limitations").  Hidden
layers use ReLU, or (act="sine") the paper's sinusoidal activation
a = sin(z) (Sec. 3.4, "Architecture").

Parameters are one flat vector, layer by layer: W_l[out, in] row-major, then
b_l[out].  Forward and backward run in float64 on float32 inputs.

bfloat16 mode is the precision the bfloat16 workloads ask for (the paper
states none): bfloat16 operands with wide accumulation in the hidden ->
hidden layers only.
  * first layer: the float32 weights on the float32 region parameters,
    exactly as in float32 mode (how a kernel evaluates that small product is
    its own choice; its error is judged against this);
  * hidden -> hidden layers: weights rounded to bfloat16, input activations
    rounded first to float32 and then to bfloat16;
  * output layer: float32 weights on float32 activations.
Rounding is to nearest, ties to even.  Products and sums stay in float64.
"""

from __future__ import annotations

import numpy as np


def layer_shapes(in_dim: int, widths) -> list:
    dims = [int(in_dim)] + [int(w) for w in widths] + [1]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def num_params(in_dim: int, widths) -> int:
    return sum(o * i + o for o, i in layer_shapes(in_dim, widths))


def unpack(theta: np.ndarray, in_dim: int, widths, dtype=np.float64):
    """Flat vector -> [(W [out,in], b [out])]."""
    theta = np.asarray(theta)
    out, off = [], 0
    for o, i in layer_shapes(in_dim, widths):
        W = theta[off:off + o * i].reshape(o, i).astype(dtype)
        off += o * i
        b = theta[off:off + o].astype(dtype)
        off += o
        out.append((W, b))
    if off != theta.size:
        raise ValueError(f"parameter vector has {theta.size} entries, net needs {off}")
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as
    float32.  Written from the definition: add 0x7FFF plus the lowest kept bit
    to the bit pattern, then clear the 16 discarded bits."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32)


def _hidden_bf16(l: int, n_layers: int) -> bool:
    return 0 < l < n_layers - 1


def _act(z, act: str):
    if act == "relu":
        return np.maximum(z, 0.0)
    if act == "sine":
        return np.sin(z)
    raise ValueError(act)


def _act_deriv(z, act: str):
    return (z > 0.0).astype(np.float64) if act == "relu" else np.cos(z)


def forward(theta, in_dim: int, widths, x, bf16: bool = False, keep: bool = False, act: str = "relu"):
    """Logits z [n] (float64).  With keep=True also returns the per-layer
    inputs a_{l-1} and pre-activations z_l used by the backward pass."""
    layers = unpack(theta, in_dim, widths)
    a = np.asarray(x, dtype=np.float32).astype(np.float64)
    inputs, pre = [], []
    for l, (W, b) in enumerate(layers):
        if bf16 and _hidden_bf16(l, len(layers)):
            W = bf16_round(W.astype(np.float32)).astype(np.float64)
            a = bf16_round(a.astype(np.float32)).astype(np.float64)
        inputs.append(a)
        z = a @ W.T + b
        pre.append(z)
        a = _act(z, act) if l + 1 < len(layers) else z
    z = a[:, 0]
    # a region with a non-finite parameter cannot be bounded: its logit is NaN,
    # which the decision takes as positive (the conservative side, h >= g)
    z = np.where(np.all(np.isfinite(np.asarray(x, dtype=np.float32)), axis=1), z, np.nan)
    if keep:
        return z, inputs, pre
    return z


def abs_forward(theta, in_dim: int, widths, x, bf16: bool = False, act: str = "relu") -> np.ndarray:
    """Scale s = |W_L| |a_{L-1}| + |b_L| of the last layer, per query: the sum
    of the magnitudes of the terms that make up the logit."""
    layers = unpack(theta, in_dim, widths)
    _, inputs, _ = forward(theta, in_dim, widths, x, bf16=bf16, keep=True, act=act)
    W, b = layers[-1]
    return (np.abs(inputs[-1]) @ np.abs(W).T)[:, 0] + abs(b[0])


def backward(theta, in_dim: int, widths, x, dz, bf16: bool = False, act: str = "relu") -> np.ndarray:
    """Gradient of sum_i dz_i * z_i with respect to theta (flat, float64).
    delta_L = dz; delta_{l-1} = (W_l^T delta_l) * act'(z_{l-1})
    (1[z > 0] for ReLU, cos z for sine);
    dW_l = sum_i delta_l a_{l-1}^T, db_l = sum_i delta_l.
    In bfloat16 mode the weights and layer inputs are the rounded ones the
    forward pass used (the first layer's input is the float32 query); the
    gradient is taken with respect to the float32 master weights (straight
    through the rounding)."""
    layers = unpack(theta, in_dim, widths)
    _, inputs, pre = forward(theta, in_dim, widths, x, bf16=bf16, keep=True, act=act)
    delta = np.asarray(dz, dtype=np.float64)[:, None]
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        if bf16 and _hidden_bf16(l, len(layers)):
            W = bf16_round(W.astype(np.float32)).astype(np.float64)
        grads[l] = (delta.T @ inputs[l], delta.sum(axis=0))
        if l:
            delta = (delta @ W) * _act_deriv(pre[l - 1], act)
    return pack(grads)


def reg_grad(theta, in_dim: int, widths, lam1: float, lam2: float) -> np.ndarray:
    """Gradient of lam1 * sum|W| + lam2 * sum W^2 over weight matrices only
    (biases are not regularised); sign(0) = 0."""
    g = []
    for W, b in unpack(theta, in_dim, widths):
        g.append((lam1 * np.sign(W) + 2.0 * lam2 * W, np.zeros_like(b)))
    return pack(g)


def reg_value(theta, in_dim: int, widths, lam1: float, lam2: float) -> float:
    return float(sum(lam1 * np.abs(W).sum() + lam2 * (W * W).sum()
                     for W, _ in unpack(theta, in_dim, widths)))
