"""Oracle training behaviour (Alg. 1 with the FN-weight ramp) on the 2-D disc
workload, CPU only: the asymmetric loss pushes false negatives toward zero at
the cost of false positives, the symmetric loss does not (Sec. 5 "Convergence",
Sec. 4.1 OccNet ablation)."""

import numpy as np

import synth
from oracle import indicators as I, loss as L, mlp, train


def test_ramp_schedule_endpoints():
    assert train.alpha_ramp(0, 200) == 1.0 and train.alpha_ramp(199, 200) == 100.0
    assert train.lam_ramp(0, 10, 5e-7) == 0.0 and abs(train.lam_ramp(9, 10, 5e-7) - 5e-7) < 1e-20


def test_regulariser_gradient_central_differences():
    theta = synth.init_params(1, 2, [4, 4]).astype(np.float64)
    g = mlp.reg_grad(theta, 2, [4, 4], 0.3, 0.7)
    h = 1e-6
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        fd = (mlp.reg_value(theta + e, 2, [4, 4], 0.3, 0.7) - mlp.reg_value(theta - e, 2, [4, 4], 0.3, 0.7)) / (2 * h)
        assert abs(fd - g[k]) < 1e-6


def test_asymmetric_beats_symmetric_on_false_negatives():
    discs = synth.discs2d(1001)
    theta0 = synth.init_params(4001, 2, [32] * 3)
    label = lambda q: I.discs2d(q, discs)
    steps, batch = 300, 1024
    th_a, _ = train.train(label, "point", 2, 2, [32] * 3, theta0, 2001, steps, batch, a_max=100.0)
    th_s, _ = train.train(label, "point", 2, 2, [32] * 3, theta0, 2001, steps, batch, a_max=1.0)
    q = synth.points(3001, 1 << 15, 2)
    g = label(q)
    ca = L.counts(L.decide(mlp.forward(th_a, 2, [32] * 3, q)), g)
    cs = L.counts(L.decide(mlp.forward(th_s, 2, [32] * 3, q)), g)
    # (TP, FP, TN, FN): fewer false negatives, more false positives
    assert ca[3] < cs[3] and ca[1] > cs[1]
    assert cs[3] > 0
