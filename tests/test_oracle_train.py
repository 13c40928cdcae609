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


# ------------------------------------------------------------ continuation

def _golden_schedule():
    import os
    rows = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "continuation_schedule.txt")):
        if line.startswith("#") or not line.strip():
            continue
        case, key, rest = line.split(None, 2)
        if "/" in rest:
            val = [[float(x) for x in part.split()] for part in rest.split("/")]
        else:
            val = [float(x) for x in rest.split()]
        rows.setdefault(case, {})[key] = val
    return rows


SINGLE_ARGS = {"single": dict(alpha0=100, inc=50, lr0=1e-3, lr_decay=0.5, lr_min=1e-4, patience=6, max_iters=20),
               "capped": dict(alpha0=100, inc=50, lr0=1e-3, lr_decay=1.0, lr_min=0.0, patience=6, max_iters=5)}
GROUP_ARGS = dict(alpha0=100, inc=10, lr0=1.0, lr_decay=0.5, lr_min=0.1, patience=2, max_iters=20)


def test_continuation_hand_worked_traces():
    gold = _golden_schedule()
    for case, kw in SINGLE_ARGS.items():
        g = gold[case]
        r = train.continuation([int(x) for x in g["fn"]], **kw)
        assert r["alpha"] == g["alpha"], case
        assert np.allclose(r["lr"], g["lr"], rtol=1e-12), case
        iters, conv, a_end = g["end"]
        assert (r["iters"], r["converged"], r["alpha_final"]) == (iters, bool(conv), a_end), case
    g = gold["group"]
    r = train.group_continuation([[int(x) for x in row] for row in g["fn"]], **GROUP_ARGS)
    assert r["alpha"] == g["alpha"]
    assert np.allclose(r["lr"], g["lr"], rtol=1e-12)
    assert (r["iters"], r["converged"]) == (int(g["end"][0]), bool(g["end"][1]))
    assert r["alpha_final"] == g["end"][2:]


def _trainer_single(fn_trace, alpha0, inc, lr0, lr_decay, lr_min, patience, max_iters):
    from paper_2310_06822_amd.trainer import Continuation, Schedule
    c = Continuation(Schedule(lr=lr0, inc=inc, patience=patience, max_iters=max_iters, lr_decay=lr_decay,
                              lr_min=lr_min), alpha0)
    alphas, lrs = [], []
    while not c.done:
        alphas.append(c.alpha)
        lrs.append(c.lr)
        c.update(fn_trace[c.iters])
    return alphas, lrs, c.iters, c.converged, c.alpha


def _trainer_group(fn_trace, alpha0, inc, lr0, lr_decay, lr_min, patience, max_iters):
    from paper_2310_06822_amd.trainer import GroupContinuation, Schedule
    c = GroupContinuation(Schedule(alpha_max=alpha0, lr=lr0, inc=inc, patience=patience, max_iters=max_iters,
                                   lr_decay=lr_decay, lr_min=lr_min), len(fn_trace[0]))
    alphas, lrs = [], []
    while not c.done:
        alphas.append(c.alpha.tolist())
        lrs.append(c.lr.tolist())
        c.update(fn_trace[c.iters])
    return alphas, lrs, c.iters, c.converged, c.alpha.tolist()


def test_trainer_schedule_equals_oracle():
    """The host schedule that drives the GPU training follows the oracle's
    schedule on the hand-worked traces and on random FN traces (single bounds
    and groups, with and without learning-rate decay)."""
    gold = _golden_schedule()
    rng = np.random.default_rng(7)
    cases = [([int(x) for x in gold[c]["fn"]], kw) for c, kw in SINGLE_ARGS.items()]
    for _ in range(300):
        p = float(rng.choice([0.05, 0.3, 0.7]))
        fn = list((rng.random(120) < p) * rng.integers(1, 9, 120))
        kw = dict(alpha0=float(rng.choice([1.0, 100.0])), inc=float(rng.choice([10.0, 50.0])),
                  lr0=1e-3, lr_decay=float(rng.choice([1.0, 0.99, 0.5])), lr_min=1e-5,
                  patience=int(rng.integers(1, 8)), max_iters=int(rng.integers(1, 100)))
        cases.append((fn, kw))
    for fn, kw in cases:
        r = train.continuation(fn, **kw)
        a, lr, iters, conv, a_end = _trainer_single(fn, **kw)
        assert a == r["alpha"] and (iters, conv, a_end) == (r["iters"], r["converged"], r["alpha_final"])
        assert np.allclose(lr, r["lr"], rtol=1e-9)
    gcases = [([[int(x) for x in row] for row in gold["group"]["fn"]], GROUP_ARGS)]
    for _ in range(100):
        n_obj = int(rng.integers(1, 7))
        p = float(rng.choice([0.02, 0.1, 0.4]))
        fn = ((rng.random((80, n_obj)) < p) * rng.integers(1, 5, (80, n_obj))).tolist()
        kw = dict(alpha0=100.0, inc=float(rng.choice([10.0, 50.0])), lr0=1e-3,
                  lr_decay=float(rng.choice([1.0, 0.998, 0.5])), lr_min=1e-5,
                  patience=int(rng.integers(1, 7)), max_iters=int(rng.integers(1, 80)))
        gcases.append((fn, kw))
    for fn, kw in gcases:
        r = train.group_continuation(fn, **kw)
        a, lr, iters, conv, a_end = _trainer_group(fn, **kw)
        assert a == r["alpha"] and (iters, conv) == (r["iters"], r["converged"]) and a_end == r["alpha_final"]
        assert np.allclose(lr, r["lr"], rtol=1e-6)   # the trainer keeps per-object rates in float32
