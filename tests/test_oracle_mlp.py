"""Pins for the oracle MLP, loss, decision, Adam, cascade and the benefit
inequality: library routines (torch float64 on the CPU), central finite
differences, closed forms and the paper's printed numbers."""

import os

import numpy as np
import pytest
import torch

import synth
from oracle import adam, cascade, loss as L, mlp

GOLDEN = os.path.dirname(os.path.abspath(__file__)) + "/golden/"

# Network shapes of the five synthetic workloads: (in_dim, widths, #params).
SHAPES = [(2, [32] * 3, 2241), (3, [64] * 3, 8641), (6, [128] * 4, 50561),
          (4, [256] * 6, 330497), (6, [32] * 3, 2369), (6, [64] * 3, 8833), (6, [128] * 3, 34049)]


def test_paper_parameter_count():
    # Sec. 6 "Limitations": the 3D point network (3 x 50 x 50) has 2,801 parameters.
    assert mlp.num_params(3, [50, 50]) == 2801


@pytest.mark.parametrize("in_dim,widths,n", SHAPES)
def test_workload_parameter_counts(in_dim, widths, n):
    assert mlp.num_params(in_dim, widths) == n == synth.num_params(in_dim, widths)
    theta = synth.init_params(1, in_dim, widths)
    assert theta.size == n
    layers = mlp.unpack(theta, in_dim, widths)
    for (W, b), (o, i) in zip(layers, mlp.layer_shapes(in_dim, widths)):
        assert W.shape == (o, i) and np.abs(W).max() <= 1 / np.sqrt(i) and np.abs(b).max() <= 1 / np.sqrt(i)


def _torch_net(theta, in_dim, widths):
    mods = []
    layers = mlp.unpack(theta, in_dim, widths)
    for l, (W, b) in enumerate(layers):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
        mods.append(lin)
        if l + 1 < len(layers):
            mods.append(torch.nn.ReLU())
    return torch.nn.Sequential(*mods)


@pytest.mark.parametrize("in_dim,widths", [(2, [32] * 3), (3, [64] * 3), (6, [128] * 4)])
def test_forward_vs_torch_sequential(in_dim, widths):
    theta = synth.init_params(5, in_dim, widths)
    x = synth.points(6, 300, in_dim)
    z = mlp.forward(theta, in_dim, widths, x)
    ref = _torch_net(theta, in_dim, widths)(torch.from_numpy(x.astype(np.float64)))[:, 0].detach().numpy()
    assert np.allclose(z, ref, rtol=1e-12, atol=1e-13)


def test_backward_vs_torch_autograd():
    in_dim, widths = 3, [16, 16, 16]
    theta = synth.init_params(7, in_dim, widths)
    x = synth.points(8, 200, in_dim)
    y = (synth.points(9, 200, 1)[:, 0] > 0).astype(np.uint8)
    z = mlp.forward(theta, in_dim, widths, x)
    g = mlp.backward(theta, in_dim, widths, x, L.dloss_dz(z, y, 7.0, 1.5))
    net = _torch_net(theta, in_dim, widths)
    zt = net(torch.from_numpy(x.astype(np.float64)))[:, 0]
    yt = torch.from_numpy(y.astype(np.float64))
    lt = (7.0 * yt * torch.nn.functional.softplus(-zt) + 1.5 * (1 - yt) * torch.nn.functional.softplus(zt)).mean()
    lt.backward()
    ref = np.concatenate([np.concatenate([m.weight.grad.numpy().ravel(), m.bias.grad.numpy()])
                          for m in net if isinstance(m, torch.nn.Linear)])
    assert np.allclose(g, ref, rtol=1e-10, atol=1e-14)


def test_backward_vs_central_differences():
    in_dim, widths = 2, [8, 8]
    theta = synth.init_params(11, in_dim, widths).astype(np.float64)
    x = synth.points(12, 64, in_dim)
    y = (synth.points(13, 64, 1)[:, 0] > 0.2).astype(np.uint8)
    alpha, beta = 4.0, 1.0

    def f(th):
        return L.loss(mlp.forward(th, in_dim, widths, x), y, alpha, beta)

    _, _, pre = mlp.forward(theta, in_dim, widths, x, keep=True)
    if min(np.abs(p).min() for p in pre[:-1]) < 1e-4:
        pytest.skip("a pre-activation sits on the ReLU kink")
    z = mlp.forward(theta, in_dim, widths, x)
    g = mlp.backward(theta, in_dim, widths, x, L.dloss_dz(z, y, alpha, beta))
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        fd[k] = (f(theta + e) - f(theta - e)) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-6 * max(1.0, np.abs(g).max())


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000), rng.normal(size=4000) * 1e-30,
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 65504.0, 3.4e38]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)
    # ties go to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert mlp.bf16_round(np.float32(1 + 2 ** -8)) == np.float32(1.0)
    assert mlp.bf16_round(np.float32(1 + 3 * 2 ** -8)) == np.float32(1 + 2 ** -6)


def test_bf16_forward_quantisation_points():
    """Independent route: torch float64 with explicit bfloat16 casts of the
    hidden -> hidden operands; the first and the output layer unrounded."""
    in_dim, widths = 6, [32, 32, 32]
    theta = synth.init_params(3, in_dim, widths)
    x = synth.points(4, 100, in_dim)
    layers = mlp.unpack(theta, in_dim, widths)
    a = torch.from_numpy(x.astype(np.float64))
    for l, (W, b) in enumerate(layers):
        Wt = torch.from_numpy(W)
        if l == 0:
            a = a @ Wt.T + torch.from_numpy(b)
        elif l < len(layers) - 1:
            Wq = Wt.float().to(torch.bfloat16).double()
            aq = a.float().to(torch.bfloat16).double()
            a = aq @ Wq.T + torch.from_numpy(b)
        else:
            a = a @ Wt.T + torch.from_numpy(b)
        if l + 1 < len(layers):
            a = torch.relu(a)
    z = mlp.forward(theta, in_dim, widths, x, bf16=True)
    assert np.allclose(z, a[:, 0].numpy(), rtol=1e-12, atol=1e-13)
    z32 = mlp.forward(theta, in_dim, widths, x)
    assert not np.allclose(z, z32, rtol=1e-6)
    assert np.allclose(z, z32, rtol=0.05, atol=0.05)


def test_bf16_backward_vs_torch():
    """bfloat16-mode gradient = float64 autograd through the rounded forward
    with straight-through rounding."""
    in_dim, widths = 4, [16, 16, 16]
    theta = synth.init_params(13, in_dim, widths)
    x = synth.points(14, 50, in_dim)
    y = (synth.points(15, 50, 1)[:, 0] > 0).astype(np.uint8)
    z = mlp.forward(theta, in_dim, widths, x, bf16=True)
    dz = L.dloss_dz(z, y, 5.0, 1.0)
    g = mlp.backward(theta, in_dim, widths, x, dz, bf16=True)
    layers = mlp.unpack(theta, in_dim, widths)
    params = []
    a = torch.from_numpy(x.astype(np.float64))
    for l, (W, b) in enumerate(layers):
        Wp = torch.from_numpy(W.copy()).requires_grad_(True)
        bp = torch.from_numpy(b.copy()).requires_grad_(True)
        params += [Wp, bp]
        if l == 0:
            a = a @ Wp.T + bp
        elif l < len(layers) - 1:
            Wq = Wp.detach().float().to(torch.bfloat16).double()
            aq = a.detach().float().to(torch.bfloat16).double()
            a = aq @ (Wq + (Wp - Wp.detach())).T + (a - a.detach()) @ Wq.T + bp
        else:
            a = a @ Wp.T + bp
        if l + 1 < len(layers):
            a = torch.relu(a)
    (a[:, 0] * torch.from_numpy(dz)).sum().backward()
    ref = np.concatenate([p.grad.numpy().ravel() for p in params])
    assert np.allclose(g, ref, rtol=1e-10, atol=1e-14)


# ------------------------------------------------------------------- loss

def test_loss_symmetric_is_bce_with_logits():
    z = np.random.default_rng(1).normal(size=1000) * 5
    y = (np.random.default_rng(2).random(1000) < 0.3).astype(np.uint8)
    ref = torch.nn.functional.binary_cross_entropy_with_logits(
        torch.from_numpy(z), torch.from_numpy(y.astype(np.float64))).item()
    assert abs(L.loss(z, y, 1.0, 1.0) - ref) < 1e-12


def test_loss_weights_and_gradient():
    rng = np.random.default_rng(3)
    z = rng.normal(size=500) * 3
    y = (rng.random(500) < 0.4).astype(np.uint8)
    w = np.where(y == 1, 9.0, 0.5)
    ref = torch.nn.functional.binary_cross_entropy_with_logits(
        torch.from_numpy(z), torch.from_numpy(y.astype(np.float64)), weight=torch.from_numpy(w)).item()
    assert abs(L.loss(z, y, 9.0, 0.5) - ref) < 1e-12
    zt = torch.from_numpy(z).requires_grad_(True)
    torch.nn.functional.binary_cross_entropy_with_logits(
        zt, torch.from_numpy(y.astype(np.float64)), weight=torch.from_numpy(w)).backward()
    assert np.allclose(L.dloss_dz(z, y, 9.0, 0.5), zt.grad.numpy(), rtol=1e-12, atol=1e-16)
    # extreme logits stay finite
    assert np.isfinite(L.loss(np.array([800.0, -800.0]), np.array([0, 1]), 1, 1))


def test_tau_closed_form_and_decision():
    t = L.tau(1e-5)
    # sigmoid(tau) + eps = 1/2 exactly (up to float64)
    assert abs(1.0 / (1.0 + np.exp(-t)) + 1e-5 - 0.5) < 1e-15
    assert abs(t - (-4.0000000005e-5)) < 1e-14
    z = np.array([0.0, -1e-5, -3.9e-5, -4.1e-5, -1e-4, np.nan, np.inf, -np.inf, 1.0])
    assert L.decide(z).tolist() == [1, 1, 1, 0, 0, 1, 1, 0, 1]


def test_counts():
    h = np.array([1, 1, 0, 0, 1, 0], np.uint8)
    g = np.array([1, 0, 0, 1, 1, 0], np.uint8)
    assert L.counts(h, g).tolist() == [2, 1, 2, 1]


# ------------------------------------------------------------------- Adam

def test_adam_vs_torch():
    rng = np.random.default_rng(4)
    theta = rng.normal(size=50)
    opt = adam.Adam(50)
    p = torch.from_numpy(theta.copy()).requires_grad_(True)
    topt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(20):
        g = rng.normal(size=50)
        theta = opt.step(theta, g)
        p.grad = torch.from_numpy(g.copy())
        topt.step()
    assert np.allclose(theta, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -2e-3, 0.0, 1e-12])
    th = adam.Adam(4).step(np.zeros(4), g)
    assert np.allclose(th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


# ------------------------------------------------- cascade and Eq. Benefit

def test_cascade_equals_g_iff_no_false_negative():
    rng = np.random.default_rng(5)
    g = (rng.random(1000) < 0.3).astype(np.uint8)
    h = np.maximum(g, (rng.random(1000) < 0.2).astype(np.uint8))      # conservative
    assert np.array_equal(cascade.cascade(h, g), g)
    h2 = h.copy()
    h2[np.nonzero(g)[0][0]] = 0
    assert not np.array_equal(cascade.cascade(h2, g), g)
    assert L.counts(h2, g)[3] == 1


def test_benefit_worked_example():
    # Sec. 6: t_a = 5 t_b, p_a = 0.1, p_b = 0.3  =>  t > 20 t_b
    tb = 1.0
    assert abs(cascade.break_even(5 * tb, tb, 0.1, 0.3) - 20 * tb) < 1e-12
    assert cascade.a_wins(5 * tb, tb, 0.1, 0.3, 21 * tb)
    assert not cascade.a_wins(5 * tb, tb, 0.1, 0.3, 19 * tb)


def test_benefit_reproduces_table2_ratio_column():
    rows = [l.split() for l in open(GOLDEN + "tab2_benefit_ratio.txt") if l.strip() and not l.startswith("#")]
    _, _, ta, pa = rows[0]
    ta, pa = float(ta), float(pa) / 100
    for name, tb, pb, ratio in rows[1:]:
        tb, pb, ratio = float(tb), float(pb) / 100, float(ratio)
        got = cascade.break_even(ta, tb, pa, pb)
        if name == "AABox":
            assert abs(got - ratio) / ratio > 0.05                     # the printed slip
            assert abs(cascade.break_even(ta, tb, pa, 0.656) - ratio) / ratio < 1e-3
        else:
            assert abs(got - ratio) / ratio < 5e-3, name


def test_throughput_units_table2():
    # Table 2 throughput = 10M queries / time: 70.82 ms -> 0.14 G rays/s, 2.58 ms -> 3.88
    assert round(1e7 / 70.82e-3 / 1e9, 2) == 0.14
    assert round(1e7 / 2.58e-3 / 1e9, 2) == 3.88


# ------------------------------------------------------------- sine networks

class _Sin(torch.nn.Module):
    def forward(self, x):
        return torch.sin(x)


def _torch_sine_net(theta, in_dim, widths):
    mods = []
    layers = mlp.unpack(theta, in_dim, widths)
    for l, (W, b) in enumerate(layers):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
        mods.append(lin)
        if l + 1 < len(layers):
            mods.append(_Sin())
    return torch.nn.Sequential(*mods)


def test_sine_forward_backward_vs_torch():
    """Sinusoidal hidden activations (Sec. 3.4): forward and the gradient of
    Eq. 1 against torch float64 autograd."""
    in_dim, widths = 3, [50, 50]
    theta = synth.init_params(21, in_dim, widths)
    x = synth.points(22, 300, in_dim)
    y = (synth.points(23, 300, 1)[:, 0] > 0).astype(np.uint8)
    z = mlp.forward(theta, in_dim, widths, x, act="sine")
    net = _torch_sine_net(theta, in_dim, widths)
    zt = net(torch.from_numpy(x.astype(np.float64)))[:, 0]
    assert np.allclose(z, zt.detach().numpy(), rtol=1e-12, atol=1e-13)
    g = mlp.backward(theta, in_dim, widths, x, L.dloss_dz(z, y, 5.0, 1.0), act="sine")
    yt = torch.from_numpy(y.astype(np.float64))
    lt = (5.0 * yt * torch.nn.functional.softplus(-zt) + (1 - yt) * torch.nn.functional.softplus(zt)).mean()
    lt.backward()
    ref = np.concatenate([np.concatenate([m.weight.grad.numpy().ravel(), m.bias.grad.numpy()])
                          for m in net if isinstance(m, torch.nn.Linear)])
    assert np.allclose(g, ref, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("in_dim,small,big", [(3, [50, 50], [64, 64]), (4, [75, 75], [80, 80])])
def test_sine_zero_padding_is_exact(in_dim, small, big):
    """A sine network padded with zero neurons computes the same logits and
    its padded parameters get zero gradient (sin 0 = 0; the padding's
    outgoing weights are zero), so a 3 x 50 x 50 network runs exactly as a
    3 x 64 x 64 one and a 4 x 75 x 75 one as a 4 x 80 x 80 one."""
    theta = synth.init_params(24, in_dim, small)
    padded = synth.pad_params(theta, in_dim, small, big)
    x = synth.points(25, 200, in_dim)
    y = (synth.points(26, 200, 1)[:, 0] > 0.1).astype(np.uint8)
    z = mlp.forward(theta, in_dim, small, x, act="sine")
    zp = mlp.forward(padded, in_dim, big, x, act="sine")
    assert np.allclose(z, zp, rtol=1e-12, atol=1e-14)
    gp = mlp.backward(padded, in_dim, big, x, L.dloss_dz(zp, y, 3.0, 1.0), act="sine")
    mask = synth.pad_params(np.ones_like(theta), in_dim, small, big) != 0
    assert np.all(gp[~mask] == 0)
    g = mlp.backward(theta, in_dim, small, x, L.dloss_dz(z, y, 3.0, 1.0), act="sine")
    assert np.allclose(gp[mask], g, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("bf16", [False, True])
def test_nonfinite_rows_are_nan_and_positive(bf16):
    """A region with a non-finite parameter gets logit NaN and decision 1;
    every other row's logit is what it is without those rows."""
    in_dim, widths = 6, [32] * 2
    theta = synth.init_params(77, in_dim, widths)
    q = synth.points(78, 50, in_dim)
    bad = np.zeros(50, bool)
    for r, v in ((3, np.nan), (10, np.inf), (11, -np.inf), (49, np.nan)):
        q[r, r % in_dim] = v
        bad[r] = True
    z = mlp.forward(theta, in_dim, widths, q, bf16=bf16)
    assert np.all(np.isnan(z[bad])) and np.all(np.isfinite(z[~bad]))
    assert np.all(L.decide(z[bad]) == 1)
    assert np.array_equal(z[~bad], mlp.forward(theta, in_dim, widths, q[~bad], bf16=bf16))
