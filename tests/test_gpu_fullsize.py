"""Parity at the workloads' full sizes, in the launch configuration the bench
times: held-out queries drawn on the device with the bench's seeds, the
tuned tile variant, one launch over every row.  A seeded sample of rows is
checked against the oracle one by one (logits within 1e-5 (FP32) or 1e-3
(BF16) of max(|z|, s), decisions identical outside |z| < 1e-4, exact answers
bit for bit); properties that hold at any size are checked on all rows (the
decision is !(z < tau) on every row, the confusion counts add up to the
rows and equal those of h against g)."""

import numpy as np
import pytest
import torch

import synth
from oracle import indicators as I, loss as L, mlp

pytestmark = pytest.mark.gpu

nb = pytest.importorskip("paper_2310_06822_amd")
from paper_2310_06822_amd import autotune, configs  # noqa: E402

N_SAMPLE = 3000


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _scene(W):
    sc = W.scene
    if sc["type"] == "discs":
        d = synth.discs2d(W.seeds["scene"], k=sc["k"])
        return nb.Indicator.discs2d(d), lambda kind, q: I.discs2d(q, d)
    if sc["type"] == "metaball_voxels":
        c, r = synth.metaballs3d(1000 + sc.get("seed_of", W.index), k=sc["k"], rlo=sc["rlo"], rhi=sc["rhi"])
        ind = nb.Indicator.metaball_voxels(c, r, sc["n"])
        grid, n = host(ind.grid), sc["n"]
        exact = {"point": I.voxel_points, "ray": I.voxel_rays, "plane": I.voxel_planes}
        return ind, lambda kind, q: exact[kind](q, grid, n)
    a, b, r = synth.metaballs4d(W.seeds["scene"], k=sc["k"], rlo=sc["rlo"], rhi=sc["rhi"])
    return nb.Indicator.metaballs4d(a, b, r), lambda kind, q: I.metaballs4d(q, a, b, r)


def _check_rows(z, h, ref, s, bf16):
    tol = 1e-3 if bf16 else 1e-5
    err = np.abs(z.astype(np.float64) - ref)
    assert np.all(err <= tol * np.maximum(np.abs(ref), s)), f"max err/bound {np.max(err / (tol * np.maximum(np.abs(ref), s))):.3g}"
    sure = np.abs(ref) > 1e-4
    assert np.array_equal(h[sure], L.decide(ref)[sure])


def _check_all_rows(z, h, g, counts):
    tau = float(L.tau())
    dec = ~(z < tau)
    assert torch.equal(h.bool(), dec)
    gb = g.bool()
    want = torch.stack([(dec & gb).sum(), (dec & ~gb).sum(), (~dec & ~gb).sum(), (~dec & gb).sum()]).cpu()
    assert torch.equal(counts.cpu(), want)
    assert int(counts.sum()) == z.numel()


@pytest.mark.parametrize("name", ["disc2d_point", "voxel3d_point", "voxel3d_ray", "voxel3d_plane",
                                  "metaball4d_point", "voxel3d_point_sine", "metaball4d_point_sine"])
def test_full_size_forward_and_exact(name):
    W = configs.WORKLOADS[name]
    kind = nb.KINDS[W.kind]
    bf16 = W.precision == "bf16"
    widths = [W.width] * W.n_hidden
    ind, exact = _scene(W)
    if W.real_width:   # the paper's narrower layers, zero-padded
        real = [W.real_width] * W.n_hidden
        theta = synth.pad_params(synth.init_params(W.seeds["init"], W.in_dim, real), W.in_dim, real, widths)
    else:
        theta = synth.init_params(W.seeds["init"], W.in_dim, widths)
    # centre the output bias so that about half of the queries are positive
    theta[-1] -= np.float32(np.median(mlp.forward(theta, W.in_dim, widths, synth.points(7, 2000, W.in_dim),
                                                 bf16=bf16, act=W.act)))
    b = nb.Bound(W.in_dim, W.n_hidden, W.width, nb.BF16 if bf16 else nb.F32)
    if W.recompute:
        nb.nb_bound_set_recompute(b.handle, W.recompute)
    if W.act == "sine":
        nb.nb_bound_set_activation(b.handle, nb.SINE)
    b.set_params(theta)
    q = torch.empty((W.eval_n, W.in_dim), dtype=torch.float32, device="cuda")
    nb.nb_sample_queries(kind, W.dim, W.seeds["eval"], 0, q)
    if bf16:
        autotune.tune(b, q)
    z, h = b.forward(q)
    g = ind.query(W.kind, q)
    counts = b.counts(q, g)
    _check_all_rows(z, h, g, counts)
    idx = np.sort(np.random.default_rng(W.index).choice(W.eval_n, N_SAMPLE, replace=False))
    it = torch.from_numpy(idx).cuda()
    qs = host(q[it])
    ref = mlp.forward(theta, W.in_dim, widths, qs, bf16=bf16, act=W.act)
    s = mlp.abs_forward(theta, W.in_dim, widths, qs, bf16=bf16, act=W.act)
    _check_rows(host(z[it]), host(h[it]), ref, s, bf16)
    assert np.array_equal(host(g[it]).astype(bool), exact(W.kind, qs).astype(bool))
    hs = host(h)
    assert 0.05 < hs.mean() < 0.95


def test_full_size_grouped_boxes():
    """256 objects x 2^16 boxes in one grouped launch with the tuned tile shape;
    20 objects sampled, 150 rows each."""
    GW = configs.GROUP_WORKLOADS["batched_box"]
    objs = synth.object_set(GW.seeds["scene"], GW.n_obj, GW.grid_sizes, GW.widths, GW.k_range)
    sizes = [o["n"] for o in objs]
    goff = np.concatenate([[0], np.cumsum([n ** 3 for n in sizes])])
    grids = torch.empty(int(goff[-1]), dtype=torch.uint8, device="cuda")
    for o, ob in enumerate(objs):
        nb.nb_voxelize_metaballs(ob["centres"], ob["radii"], 1.0, ob["n"], grids[goff[o]:goff[o + 1]])
    widths = [o["width"] for o in objs]
    gr = nb.Group(GW.in_dim, widths, GW.n_hidden)
    gr.set_voxels(grids, sizes)
    probe = synth.points(8, 1000, GW.in_dim)
    thetas = []
    for i, w in enumerate(widths):
        th = synth.init_params(GW.seeds["init"] * 1000 + i, GW.in_dim, [w] * GW.n_hidden)
        th[-1] -= np.float32(np.median(mlp.forward(th, GW.in_dim, [w] * GW.n_hidden, probe, bf16=True)))
        thetas.append(th)
    gr.set_params(np.concatenate(thetas).astype(np.float32))
    per = GW.eval_per_obj
    n = per * GW.n_obj
    q = torch.empty((n, GW.in_dim), dtype=torch.float32, device="cuda")
    nb.nb_sample_queries(nb.BOX, 3, GW.seeds["eval"], 0, q)
    qoff = torch.arange(0, n + 1, per, dtype=torch.int64, device="cuda")
    autotune.tune_group(gr, q, qoff)
    z, h = gr.forward(q, qoff)
    g = gr.query("box", q, qoff)
    counts = gr.counts(q, qoff, g)
    _check_all_rows(z, h, g, counts.sum(0))
    rng = np.random.default_rng(3)
    for o in np.sort(rng.choice(GW.n_obj, 20, replace=False)):
        rows = o * per + np.sort(rng.choice(per, 150, replace=False))
        it = torch.from_numpy(rows).cuda()
        qs = host(q[it])
        wl = [widths[o]] * GW.n_hidden
        ref = mlp.forward(thetas[o], GW.in_dim, wl, qs, bf16=True)
        s = mlp.abs_forward(thetas[o], GW.in_dim, wl, qs, bf16=True)
        _check_rows(host(z[it]), host(h[it]), ref, s, True)
        grid_o = host(grids[goff[o]:goff[o + 1]])
        assert np.array_equal(host(g[it]).astype(bool), I.voxel_boxes(qs, grid_o, sizes[o]).astype(bool)), o
