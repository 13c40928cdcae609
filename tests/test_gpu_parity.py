"""GPU parity: every kernel of the hot path against the CPU oracle on the
same seeded inputs, called through the C ABI.

Bars: integer results (samples' bits, indicator answers, counts) are
bit-exact; float32 logits satisfy |dz| <= 1e-5 * max(|z|, s) with
s = |W_L| |a_{L-1}| + |b_L| (the magnitude sum of the last layer's terms);
decisions may differ only where |z| < 1e-4; gradients match per tensor to
1e-5 in relative Frobenius norm.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import indicators as I, loss as L, mlp, sampling
from oracle.adam import Adam

pytestmark = pytest.mark.gpu

nb = pytest.importorskip("paper_2310_06822_amd")


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


@pytest.fixture(scope="module")
def c2_grid():
    c, r = synth.metaballs3d(1001, k=16)
    return c, r, I.voxelize_metaballs(c, r, 128)


# ---------------------------------------------------------------- sampling

@pytest.mark.parametrize("kind,dim,n", [("point", 2, 4099), ("point", 3, 65536 + 17), ("point", 4, 1000),
                                        ("ray", 3, 5003), ("box", 3, 4097), ("plane", 3, 3001)])
def test_sampler_bit_exact(kind, dim, n):
    d = dim if kind == "point" else 6
    for seed, step in [(2001, 0), (2001, 7), (0xDEADBEEF12345, 123456)]:
        q = torch.empty((n, d), dtype=torch.float32, device="cuda")
        nb.nb_sample_queries(nb.KINDS[kind], dim, seed, step, q)
        ref = sampling.sample(kind, seed, step, n, dim)
        assert np.array_equal(bits(host(q)), bits(ref)), (kind, seed, step)


# --------------------------------------------------------------- indicators

@pytest.mark.parametrize("n,k", [(8, 3), (32, 16), (33, 5), (128, 16)])
def test_voxelize_bit_exact(n, k):
    c, r = synth.metaballs3d(1001 + n, k=k)
    grid = torch.empty(n ** 3, dtype=torch.uint8, device="cuda")
    nb.nb_voxelize_metaballs(c, r, 1.0, n, grid)
    ref = I.voxelize_metaballs(c, r, n)
    assert np.array_equal(host(grid), ref)
    assert 0 < ref.sum() < ref.size


def test_exact_discs():
    discs = synth.discs2d(1000)
    ind = nb.Indicator.discs2d(discs)
    q = synth.points(5, 70001, 2) * np.float32(1.2)
    g = ind.query("point", cuda(q))
    assert np.array_equal(host(g), I.discs2d(q, discs))


def test_exact_voxel_points(c2_grid):
    _, _, grid = c2_grid
    ind = nb.Indicator.voxels(cuda(grid), 128)
    q = synth.points(6, 100003, 3) * np.float32(1.1)
    q[:5] = [[1, 1, 1], [-1, -1, -1], [1.0000001, 0, 0], [np.nan, 0, 0], [0, 0, 0]]
    g = ind.query("point", cuda(q))
    assert np.array_equal(host(g), I.voxel_points(q, grid, 128))


@pytest.mark.parametrize("n", [(1 << 19) - 3, (1 << 19) + 77, (1 << 21) + 5])
def test_exact_rays_every_launch_shape(n, c2_grid):
    """The ray test runs with 8 lanes per ray up to 2^19 rays, 4 up to 2^21
    and 1 beyond: each shape against the oracle on a seeded sample of rows."""
    _, _, grid = c2_grid
    ind = nb.Indicator.voxels(cuda(grid), 128)
    q = torch.empty((n, 6), dtype=torch.float32, device="cuda")
    nb.nb_sample_queries(nb.RAY, 3, 31, 0, q)
    g = host(ind.query("ray", q))
    rows = np.sort(np.random.default_rng(n).choice(n, 4000, replace=False))
    qs = host(q[torch.from_numpy(rows).cuda()])
    assert np.array_equal(g[rows], I.voxel_rays(qs, grid, 128))
    assert 0.02 < g.mean() < 0.98


def test_exact_rays(c2_grid):
    _, _, grid = c2_grid
    ind = nb.Indicator.voxels(cuda(grid), 128)
    q = synth.rays(7, 8195)
    # edge cases: axis-parallel directions, origins on the cube faces, d = 0,
    # segments that end exactly on a face, rays starting inside the cube
    edge = np.array([[-2, 0.1, 0.1, 1, 0, 0], [0.3, -2, 0.2, 0, 1, 0], [0.1, 0.2, 3, 0, 0, -1],
                     [-1, -1, -1, 0.57735, 0.57735, 0.57735], [1, 1, 1, -0.57735, -0.57735, -0.57735],
                     [0.2, 0.3, 0.1, 0, 0, 0], [-5, 0, 0, 1, 0, 0], [-3, 0.05, -0.1, 1, 0, 0],
                     [0, 0, 0, 0, 0, 1], [0.99, 0.99, 0.99, 1, 0, 0], [1.5, 1.5, 1.5, 0, 0, 1]], np.float32)
    q = np.concatenate([edge, q]).astype(np.float32)
    g = ind.query("ray", cuda(q))
    ref = I.voxel_rays(q, grid, 128)
    assert np.array_equal(host(g), ref)
    assert 0.05 < ref.mean() < 0.95
    # a grid occupied everywhere: g = 1 iff some sample lies in the closed cube
    full = nb.Indicator.voxels(cuda(np.ones(32 ** 3, np.uint8)), 32)
    assert np.array_equal(host(full.query("ray", cuda(q))), I.voxel_rays(q, np.ones(32 ** 3, np.uint8), 32))


@pytest.mark.parametrize("n", [32, 128])
def test_exact_boxes(n):
    c, r = synth.metaballs3d(77, k=12)
    grid = I.voxelize_metaballs(c, r, n)
    ind = nb.Indicator.voxels(cuda(grid), n)
    q = synth.boxes(8, 3001)
    q[0] = [-2, -2, -2, 2, 2, 2]
    q[1] = [1.5, 0, 0, 2, 1, 1]
    q[2] = [0.1, 0.1, 0.1, 0.1, 0.1, 0.1]
    g = ind.query("box", cuda(q))
    assert np.array_equal(host(g), I.voxel_boxes(q, grid, n))


def test_exact_planes():
    n = 16
    c, r = synth.metaballs3d(78, k=6)
    grid = I.voxelize_metaballs(c, r, n)
    ind = nb.Indicator.voxels(cuda(grid), n)
    q = synth.planes(9, 1501)
    g = ind.query("plane", cuda(q))
    ref = I.voxel_planes(q, grid, n)
    assert np.array_equal(host(g), ref)
    assert 0.05 < ref.mean() < 0.95


def _plane_edge_cases(n, seed, grid):
    """Planes that stress the column search of the plane test: far-away
    points p0 (on and off the cube), scaled normals (tiny, huge, subnormal
    components, zero), axis-aligned planes on cell faces (|e| = rad exactly),
    ties between normal components, non-finite values, planes through the
    cube whose p0 lies up to 1e7 away along the plane (large rounding error
    in the float32 predicate), and planes grazing the object: just inside or
    just outside the extreme occupied cell along a random normal."""
    g = np.random.default_rng(seed)
    base = synth.planes(seed, 40)
    rows = list(base)
    P = np.stack(I._occupied_cells(grid, n), 1).astype(np.float64)
    for _ in range(20):
        nrm = g.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        j = int(np.argmax(P @ nrm))
        rad = np.abs(nrm).sum() / n
        for d in (0.3, 0.9, 0.999, 1.001, 1.2):
            rows.append(list(P[j] + d * rad * nrm) + list(nrm))
    for sc in (1e3, 1e6, 1e20):
        b = base[:8].copy()
        b[:, :3] *= sc
        rows += list(b)
    for sc in (1e-3, 1e5, 1e-20, 1e20, 2.0 ** -70):
        b = base[8:14].copy()
        b[:, 3:] *= sc
        rows += list(b)
    for ax in range(3):
        for f in range(0, n + 1, max(1, n // 5)):
            x = np.float32(-1.0 + 2.0 * f / n)
            r = [0.0] * 6
            r[ax], r[3 + ax] = x, 1.0
            rows.append(r)
            r = [0.0] * 6
            r[ax], r[3 + ax], r[3 + (ax + 1) % 3] = x, -0.5, 1e-30
            rows.append(r)
    for lam in (1e3, 1e4, 1e5, 1e6, 1e7):
        for _ in range(6):
            nrm = g.normal(size=3)
            nrm /= np.linalg.norm(nrm)
            tv = np.cross(nrm, g.normal(size=3))
            tv /= np.linalg.norm(tv)
            rows.append(list(g.uniform(-0.8, 0.8, 3) + lam * tv) + list(nrm))
    rows += [[0.1, 0.2, 0.3, 0.7071, 0.7071, 0.0], [0.1, 0.2, -0.3, 0.577, -0.577, 0.577],
             [0.0, 0.0, 0.0, 1e-40, 1.0, 1e-42], [0.3, 0.3, 0.3, 0.0, 0.0, 0.0],
             [np.nan, 0, 0, 0, 0, 1], [0, 0, 0, np.inf, 0, 1], [np.inf, 0, 0, 1, 0, 0],
             [1.5, 0, 0, 1, 0, 0], [-1.0, 0.0, 0.0, 1, 0, 0], [1.0, 0, 0, -1, 0, 0]]
    return np.asarray(rows, dtype=np.float32)


@pytest.mark.parametrize("n,k", [(5, 2), (16, 6), (33, 8), (64, 12), (128, 16)])
def test_exact_planes_edge_cases(n, k):
    c, r = synth.metaballs3d(50 + n, k=k, rlo=0.05, rhi=0.25)
    grid = I.voxelize_metaballs(c, r, n)
    ind = nb.Indicator.voxels(cuda(grid), n)
    q = _plane_edge_cases(n, n, grid)
    with np.errstate(invalid="ignore", over="ignore"):
        ref = I.voxel_planes(q, grid, n)
    assert np.array_equal(host(ind.query("plane", cuda(q))), ref)
    assert 0.2 < ref.mean() < 0.9


def test_exact_planes_empty_and_full_grids():
    q = synth.planes(12, 777)
    empty = nb.Indicator.voxels(cuda(np.zeros(20 ** 3, np.uint8)), 20)
    assert host(empty.query("plane", cuda(q))).sum() == 0
    full = np.ones(20 ** 3, np.uint8)
    ind = nb.Indicator.voxels(cuda(full), 20)
    assert np.array_equal(host(ind.query("plane", cuda(q))), I.voxel_planes(q, full, 20))


def test_exact_metaballs4d():
    a, b, r = synth.metaballs4d(1004)
    ind = nb.Indicator.metaballs4d(a, b, r)
    q = synth.points4d(10, 65537)
    g = ind.query("point", cuda(q))
    assert np.array_equal(host(g), I.metaballs4d(q, a, b, r))


# ------------------------------------------------------------ MLP forward

SHAPES = [(2, 32, 3), (3, 64, 3), (6, 16, 2), (4, 32, 4), (3, 16, 1), (6, 64, 4), (8, 64, 2), (4, 80, 2), (8, 80, 1), (8, 80, 2)]


def _check_logits(z, theta, in_dim, widths, q, rtol=1e-5):
    ref = mlp.forward(theta, in_dim, widths, q)
    s = mlp.abs_forward(theta, in_dim, widths, q)
    err = np.abs(z.astype(np.float64) - ref)
    bound = rtol * np.maximum(np.abs(ref), s)
    assert np.all(err <= bound), f"max err/bound {np.max(err / bound):.3g}"
    return ref


@pytest.mark.parametrize("in_dim,width,nh", SHAPES)
@pytest.mark.parametrize("n", [1, 16, 17, 3005])
def test_forward_parity(in_dim, width, nh, n):
    widths = [width] * nh
    theta = synth.init_params(40 + in_dim + width + nh, in_dim, widths)
    q = synth.points(41, n, in_dim)
    b = nb.Bound(in_dim, nh, width)
    b.set_params(theta)
    z, h = b.forward(cuda(q))
    z, h = host(z), host(h)
    ref = _check_logits(z, theta, in_dim, widths, q)
    band = np.abs(ref) < 1e-4
    assert np.array_equal(h[~band], L.decide(ref)[~band])
    assert np.array_equal(h, L.decide(z))


def test_forward_counts_and_edge_logits(c2_grid):
    _, _, grid = c2_grid
    in_dim, widths = 3, [64] * 3
    theta = synth.init_params(4001, in_dim, widths)
    b = nb.Bound(in_dim, 3, 64)
    b.set_params(theta)
    q = synth.points(3001, 50001, 3)
    g = I.voxel_points(q, grid, 128)
    cnt = b.counts(cuda(q), cuda(g))
    z, _ = b.forward(cuda(q))
    ref = mlp.forward(theta, in_dim, widths, q)
    band = np.abs(ref) < 1e-4
    want = L.counts(L.decide(host(z)), g)
    assert host(cnt).tolist() == want.tolist()
    assert np.array_equal(L.decide(host(z))[~band], L.decide(ref)[~band])


BF16_SHAPES = [(6, 128, 4), (4, 64, 3), (6, 32, 2), (8, 128, 5), (3, 64, 1), (2, 32, 4), (4, 256, 6),
               (6, 256, 2), (3, 256, 3)]


@pytest.mark.parametrize("in_dim,width,nh", BF16_SHAPES)
@pytest.mark.parametrize("n", [1, 17, 4099])
def test_forward_bf16_parity(in_dim, width, nh, n):
    """bfloat16 forward vs the oracle's bfloat16 model: |dz| <= 1e-3 max(|z|, s);
    decisions identical wherever that bar cannot flip the sign."""
    widths = [width] * nh
    theta = synth.init_params(80 + in_dim + width + nh, in_dim, widths)
    q = synth.points(81, n, in_dim)
    b = nb.Bound(in_dim, nh, width, nb.BF16)
    b.set_params(theta)
    z, h = b.forward(cuda(q))
    z, h = host(z).astype(np.float64), host(h)
    ref = mlp.forward(theta, in_dim, widths, q, bf16=True)
    s = mlp.abs_forward(theta, in_dim, widths, q, bf16=True)
    bound = 1e-3 * np.maximum(np.abs(ref), s)
    err = np.abs(z - ref)
    assert np.all(err <= bound), f"max err/bound {np.max(err / bound):.3g}"
    sure = np.abs(ref) > np.maximum(1e-4, bound)
    assert np.array_equal(h[sure], L.decide(ref)[sure])
    assert np.array_equal(h, L.decide(z))
    # the bfloat16 path is not the float32 one: its error is visible against
    # float32 wherever a hidden -> hidden layer exists (the first and output
    # layers are float32-accurate)
    if n > 1000 and nh >= 2:
        z32 = mlp.forward(theta, in_dim, widths, q)
        assert np.max(np.abs(z - z32)) > 1e-6


# ---------------------------------------------------------- loss / gradient

def _rel_frob(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("in_dim,width,nh", SHAPES)
@pytest.mark.parametrize("n", [5, 4099])
def test_loss_grad_parity(in_dim, width, nh, n):
    widths = [width] * nh
    theta = synth.init_params(50 + width, in_dim, widths)
    q = synth.points(51, n, in_dim)
    y = (synth.points(52, n, 1)[:, 0] > 0.3).astype(np.uint8)
    alpha, beta = 7.5, 1.25
    b = nb.Bound(in_dim, nh, width)
    b.set_params(theta)
    grad = torch.empty(b.n_params, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    cnt = torch.empty(4, dtype=torch.int64, device="cuda")
    nb.nb_bound_loss_grad(b.handle, cuda(q), cuda(y), alpha, beta, grad, loss, cnt)
    z = mlp.forward(theta, in_dim, widths, q)
    gref = mlp.backward(theta, in_dim, widths, q, L.dloss_dz(z, y, alpha, beta))
    g = host(grad).astype(np.float64)
    assert abs(host(loss)[0] - L.loss(z, y, alpha, beta)) <= 1e-5 * L.loss(z, y, alpha, beta)
    for (Wg, bg), (Wr, br) in zip(mlp.unpack(g, in_dim, widths), mlp.unpack(gref, in_dim, widths)):
        assert _rel_frob(Wg, Wr) <= 1e-5
        assert _rel_frob(bg, br) <= 1e-5
    band = np.abs(z) < 1e-4
    if not band.any():
        assert host(cnt).tolist() == L.counts(L.decide(z), y).tolist()


def test_loss_grad_deterministic():
    in_dim, widths = 3, [64] * 3
    theta = synth.init_params(60, in_dim, widths)
    q = cuda(synth.points(61, 65536, 3))
    y = cuda((synth.points(62, 65536, 1)[:, 0] > 0).astype(np.uint8))
    b = nb.Bound(3, 3, 64)
    b.set_params(theta)
    outs = []
    for _ in range(2):
        grad = torch.empty(b.n_params, dtype=torch.float32, device="cuda")
        nb.nb_bound_loss_grad(b.handle, q, y, 3.0, 1.0, grad)
        outs.append(host(grad))
    assert np.array_equal(bits(outs[0]), bits(outs[1]))


# ----------------------------------------------------------------- Adam

def test_adam_step_parity():
    in_dim, widths = 3, [64] * 3
    theta = synth.init_params(70, in_dim, widths)
    b = nb.Bound(3, 3, 64)
    b.set_params(theta)
    opt = Adam(theta.size)
    th = theta.astype(np.float64)
    rng = np.random.default_rng(0)
    for _ in range(5):
        g = (rng.normal(size=theta.size) * 1e-2).astype(np.float32)
        nb.nb_bound_adam_step(b.handle, cuda(g))
        th = opt.step(th, g)
    got = host(b.params()).astype(np.float64)
    assert np.max(np.abs(got - th)) <= 1e-6


# ------------------------------------------------------ checkpoint / resume

@pytest.mark.parametrize("prec,kind,in_dim,width,nh,act,every", [(nb.F32, "point", 3, 64, 3, "relu", 0),
                                                                 (nb.F32, "point", 4, 80, 2, "sine", 0),
                                                                 (nb.BF16, "ray", 6, 128, 4, "relu", 0),
                                                                 (nb.BF16, "point", 4, 256, 6, "relu", 3)])
def test_checkpoint_resume_is_bit_identical(prec, kind, in_dim, width, nh, act, every, c2_grid):
    """Training resumed from nb_bound_save / nb_bound_load in a fresh bound
    continues bit for bit like the run that never stopped (parameters, Adam
    moments and step all restored); a checkpoint of another shape or a
    truncated one is refused."""
    _, _, grid = c2_grid
    if in_dim == 4:
        ind = nb.Indicator.metaballs4d(*synth.metaballs4d(1005, k=24))
    else:
        ind = nb.Indicator.voxels(cuda(grid), 128)
    k = nb.KINDS[kind]
    batch = 1 << 14

    def make():
        b = nb.Bound(in_dim, nh, width, prec)
        if act == "sine":
            nb.nb_bound_set_activation(b.handle, nb.SINE)
        if every:
            nb.nb_bound_set_recompute(b.handle, every)
        return b

    def steps(b, t0, t1):
        for t in range(t0, t1):
            nb.nb_bound_train_step(b.handle, ind.handle, k, 177, t, batch, 5.0 + t, 1.0, 1e-3)

    a = make()
    a.set_params(synth.init_params(176 + width, in_dim, [width] * nh))
    steps(a, 0, 4)
    ck = nb.nb_bound_save(a.handle)
    assert len(ck) == 48 + 3 * 4 * a.n_params
    r = make()
    nb.nb_bound_load(r.handle, ck)
    steps(a, 4, 8)
    steps(r, 4, 8)
    assert np.array_equal(bits(host(a.params())), bits(host(r.params())))
    assert nb.nb_bound_save(a.handle) == nb.nb_bound_save(r.handle)
    q = cuda(synth.points(178, 2001, in_dim))
    za, _ = a.forward(q)
    zr, _ = r.forward(q)
    assert np.array_equal(bits(host(za)), bits(host(zr)))
    other = nb.Bound(in_dim, nh, 64 if width != 64 else 32, prec)
    with pytest.raises(nb.NBError):
        nb.nb_bound_load(other.handle, ck)
    with pytest.raises(nb.NBError):
        nb.nb_bound_load(r.handle, ck[:-4])


# ---------------------------------------------------------- training steps

@pytest.mark.parametrize("cfg", ["disc", "voxel"])
def test_train_steps_parity(cfg, c2_grid):
    if cfg == "disc":
        discs = synth.discs2d(1000)
        ind = nb.Indicator.discs2d(discs)
        label = lambda q: I.discs2d(q, discs)
        in_dim, width, dim = 2, 32, 2
    else:
        _, _, grid = c2_grid
        ind = nb.Indicator.voxels(cuda(grid), 128)
        label = lambda q: I.voxel_points(q, grid, 128)
        in_dim, width, dim = 3, 64, 3
    widths = [width] * 3
    theta0 = synth.init_params(4000, in_dim, widths)
    steps, batch, seed = 10, 2048, 2000
    b = nb.Bound(in_dim, 3, width)
    b.set_params(theta0)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    cnt = torch.empty(4, dtype=torch.int64, device="cuda")
    from oracle import train as T
    th, hist = T.train(label, "point", dim, in_dim, widths, theta0, seed, steps, batch)
    for t in range(steps):
        a = T.alpha_ramp(t, steps)
        nb.nb_bound_train_step(b.handle, ind.handle, nb.POINT, seed, t, batch, a, 1.0, 1e-3, loss=loss, counts=cnt)
        lv = host(loss)[0]
        assert abs(lv - hist[t][0]) <= 1e-4 * abs(hist[t][0]), (t, lv, hist[t][0])
    got = host(b.params()).astype(np.float64)
    d_gpu, d_ref = got - theta0, th - theta0
    assert _rel_frob(d_gpu, d_ref) <= 1e-2


@pytest.mark.parametrize("in_dim,width,nh,act,kind", [(3, 64, 3, "relu", "point"), (6, 32, 2, "relu", "ray"),
                                                      (4, 80, 2, "sine", "point"), (2, 16, 4, "relu", "point")])
def test_train_step_packs_weights(in_dim, width, nh, act, kind, c2_grid):
    """A float32 training step writes its updated weights straight into the
    packed fragments the kernels read: the logits after a few steps are
    bit-identical to those after rebuilding every fragment from theta."""
    _, _, grid = c2_grid
    if in_dim == 4:
        ind = nb.Indicator.metaballs4d(*synth.metaballs4d(1005, k=24))
    elif in_dim == 2:
        ind = nb.Indicator.discs2d(synth.discs2d(1000))
    else:
        ind = nb.Indicator.voxels(cuda(grid), 128)
    b = nb.Bound(in_dim, nh, width)
    if act == "sine":
        nb.nb_bound_set_activation(b.handle, nb.SINE)
    b.set_params(synth.init_params(170 + width, in_dim, [width] * nh))
    for t in range(3):
        nb.nb_bound_train_step(b.handle, ind.handle, nb.KINDS[kind], 171, t, 4096, 5.0, 1.0, 1e-2)
    q = cuda(synth.points(172, 3001, in_dim))
    z_fused, _ = b.forward(q)
    z_fused = bits(host(z_fused))
    b.set_params(b.params().clone())   # rebuilds every fragment from theta
    z_full, _ = b.forward(q)
    assert np.array_equal(z_fused, bits(host(z_full)))


# ------------------------------------------------------------------ cascade

@pytest.mark.parametrize("kind,prec", [("point", nb.F32), ("ray", nb.BF16), ("box", nb.BF16), ("point", nb.BF16),
                                       ("plane", nb.BF16)])
def test_cascade(kind, prec, c2_grid):
    _, _, grid = c2_grid
    ind = nb.Indicator.voxels(cuda(grid), 128)
    in_dim = 3 if kind == "point" else 6
    if prec == nb.F32:
        width, nh = 64, 3
    else:
        width, nh = 128, 4
    theta = synth.init_params(90, in_dim, [width] * nh)
    n = 3001 if kind == "plane" else 20011
    q = {"point": lambda: synth.points(91, n, 3), "ray": lambda: synth.rays(92, n),
         "box": lambda: synth.boxes(93, n), "plane": lambda: synth.planes(96, n)}[kind]()
    # centre the output bias so that about half of the queries are positive
    theta[-1] -= np.float32(np.median(mlp.forward(theta, in_dim, [width] * nh, q, bf16=prec == nb.BF16)))
    b = nb.Bound(in_dim, nh, width, prec)
    b.set_params(theta)
    qd = cuda(q)
    ans = torch.empty(n, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    nb.nb_cascade(b.handle, ind.handle, nb.KINDS[kind], qd, ans, cnt)
    _, h = b.forward(qd)
    h = host(h)
    g = {"point": I.voxel_points, "ray": I.voxel_rays, "box": I.voxel_boxes,
         "plane": I.voxel_planes}[kind](q, grid, 128)
    assert np.array_equal(host(ans), h & g)
    assert int(host(cnt)[0]) == int(h.sum())
    assert 0 < h.sum() < n


def test_cascade_equals_exact_for_conservative_bound(c2_grid):
    """A bound that says 1 everywhere (large output bias) is conservative: the
    cascade answer is exactly g and every query reaches the exact test."""
    _, _, grid = c2_grid
    ind = nb.Indicator.voxels(cuda(grid), 128)
    theta = synth.init_params(94, 3, [64] * 3)
    theta[-1] = 1e3
    b = nb.Bound(3, 3, 64)
    b.set_params(theta)
    q = synth.points(95, 9999, 3)
    ans = torch.empty(9999, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    nb.nb_cascade(b.handle, ind.handle, nb.POINT, cuda(q), ans, cnt)
    assert np.array_equal(host(ans), I.voxel_points(q, grid, 128))
    assert int(host(cnt)[0]) == 9999


# ----------------------------------------------------------------- autograd

def test_autograd_bound_loss():
    from paper_2310_06822_amd.autograd import bound_loss
    in_dim, widths = 3, [64] * 3
    theta0 = synth.init_params(96, in_dim, widths)
    q = synth.points(97, 5000, 3)
    y = (synth.points(98, 5000, 1)[:, 0] > 0.5).astype(np.uint8)
    b = nb.Bound(3, 3, 64)
    theta = cuda(theta0).requires_grad_(True)
    loss = bound_loss(theta, b, cuda(q), cuda(y), 20.0, 1.0)
    (2.0 * loss).backward()
    z = mlp.forward(theta0, in_dim, widths, q)
    gref = 2.0 * mlp.backward(theta0, in_dim, widths, q, L.dloss_dz(z, y, 20.0, 1.0))
    assert abs(loss.item() - L.loss(z, y, 20.0, 1.0)) <= 1e-5 * L.loss(z, y, 20.0, 1.0)
    assert _rel_frob(host(theta.grad).astype(np.float64), gref) <= 1e-5
    # a torch optimiser steps theta with the kernel's gradient
    opt = torch.optim.Adam([theta], lr=1e-3)
    opt.step()
    assert np.max(np.abs(host(theta.detach()) - theta0)) > 0


# ------------------------------------------------------- bfloat16 training

BF16_TRAIN_SHAPES = [(6, 128, 4), (4, 64, 3), (6, 32, 2), (3, 128, 2), (8, 64, 5), (4, 256, 6), (6, 256, 2)]


def _bf16_grad_check(in_dim, width, nh, q, y, alpha, beta):
    widths = [width] * nh
    theta = synth.init_params(100 + width + nh, in_dim, widths)
    b = nb.Bound(in_dim, nh, width, nb.BF16)
    b.set_params(theta)
    grad = torch.empty(b.n_params, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    cnt = torch.empty(4, dtype=torch.int64, device="cuda")
    nb.nb_bound_loss_grad(b.handle, cuda(q), cuda(y), alpha, beta, grad, loss, cnt)
    z = mlp.forward(theta, in_dim, widths, q, bf16=True)
    gref = mlp.backward(theta, in_dim, widths, q, L.dloss_dz(z, y, alpha, beta), bf16=True)
    lref = L.loss(z, y, alpha, beta)
    assert abs(host(loss)[0] - lref) <= 1e-3 * lref
    g = host(grad).astype(np.float64)
    worst = 0.0
    for (Wg, bg), (Wr, br) in zip(mlp.unpack(g, in_dim, widths), mlp.unpack(gref, in_dim, widths)):
        worst = max(worst, _rel_frob(Wg, Wr), _rel_frob(bg, br))
    assert worst <= 1e-2, worst
    return b, g


@pytest.mark.parametrize("in_dim,width,nh", BF16_TRAIN_SHAPES)
@pytest.mark.parametrize("n", [7, 4099])
def test_loss_grad_bf16_parity(in_dim, width, nh, n):
    q = synth.points(101, n, in_dim)
    y = (synth.points(102, n, 1)[:, 0] > 0.2).astype(np.uint8)
    _bf16_grad_check(in_dim, width, nh, q, y, 9.0, 1.5)


def test_loss_grad_bf16_deterministic():
    q = synth.points(103, 70001, 6)
    y = (synth.points(104, 70001, 1)[:, 0] > 0).astype(np.uint8)
    b, g1 = _bf16_grad_check(6, 128, 4, q, y, 3.0, 1.0)
    grad = torch.empty(b.n_params, dtype=torch.float32, device="cuda")
    nb.nb_bound_loss_grad(b.handle, cuda(q), cuda(y), 3.0, 1.0, grad)
    assert np.array_equal(bits(host(grad)), bits(g1.astype(np.float32)))


def test_train_steps_bf16_rays(c2_grid):
    _, _, grid = c2_grid
    ind = nb.Indicator.voxels(cuda(grid), 128)
    widths = [64] * 3
    theta0 = synth.init_params(4002, 6, widths)
    steps, batch, seed = 5, 2048, 2002
    b = nb.Bound(6, 3, 64, nb.BF16)
    b.set_params(theta0)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    from oracle import train as T
    th, hist = T.train(lambda q: I.voxel_rays(q, grid, 128), "ray", 3, 6, widths, theta0, seed, steps, batch,
                       bf16=True)
    for t in range(steps):
        nb.nb_bound_train_step(b.handle, ind.handle, nb.RAY, seed, t, batch, T.alpha_ramp(t, steps), 1.0, 1e-3,
                               loss=loss)
        assert abs(host(loss)[0] - hist[t][0]) <= 2e-3 * abs(hist[t][0]), t
    d_gpu = host(b.params()).astype(np.float64) - theta0
    assert _rel_frob(d_gpu, th - theta0) <= 5e-2


FUSED_SHAPES = [(6, 128, 4), (6, 128, 3), (3, 128, 2), (4, 64, 3), (6, 64, 4), (8, 64, 2), (6, 32, 2),
                (2, 32, 4), (5, 32, 3)]


@pytest.mark.parametrize("in_dim,width,nh", FUSED_SHAPES)
@pytest.mark.parametrize("n", [7, 4099, 70001])
def test_bf16_fused_vs_layerwise(in_dim, width, nh, n):
    """The fused training kernel and the layer-wise kernels compute the same
    loss, counts and gradient up to float32 summation order (single tile,
    several tiles per chunk with a ragged last one)."""
    q = synth.points(131, n, in_dim)
    y = (synth.points(132, n, 1)[:, 0] > 0.3).astype(np.uint8)
    theta = synth.init_params(133 + width + nh, in_dim, [width] * nh)
    out = {}
    for kern in (nb.TRAIN_AUTO, nb.TRAIN_LAYERWISE):
        b = nb.Bound(in_dim, nh, width, nb.BF16)
        nb.nb_bound_set_train_kernel(b.handle, kern)
        b.set_params(theta)
        g = torch.empty(b.n_params, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        cnt = torch.empty(4, dtype=torch.int64, device="cuda")
        nb.nb_bound_loss_grad(b.handle, cuda(q), cuda(y), 7.0, 1.0, g, loss, cnt)
        out[kern] = (host(g).astype(np.float64), float(host(loss)[0]), host(cnt))
    gf, lf, cf = out[nb.TRAIN_AUTO]
    gl, ll, cl = out[nb.TRAIN_LAYERWISE]
    assert np.array_equal(cf, cl)
    assert abs(lf - ll) <= 1e-5 * abs(ll)
    widths = [width] * nh
    for (Wf, bf), (Wl, bl) in zip(mlp.unpack(gf, in_dim, widths), mlp.unpack(gl, in_dim, widths)):
        assert _rel_frob(Wf, Wl) <= 2e-3 and _rel_frob(bf, bl) <= 2e-3


@pytest.mark.parametrize("in_dim,nh,every", [(4, 6, 3), (4, 6, 0), (8, 2, 0), (3, 3, 2), (5, 6, 2), (1, 4, 0), (6, 8, 3)])
@pytest.mark.parametrize("n", [7, 4099, 70001])
def test_bf16_train256_vs_layerwise(in_dim, nh, every, n):
    """Width 256: the streamed training forward (one launch for the first
    layer, the hidden layers and the head) and the one-launch backward layers
    write the same activation and D_l bits as the layer-wise kernels, and sum
    the weight-gradient tiles over the same 32-query slabs, so every weight
    gradient and the first layer's bias gradient are bit-identical; the
    hidden biases, the output layer's gradient and the loss are summed in
    other orders (float32 rounding only).  Checkpointed recomputation
    included; 70001 gives chunks of 320 queries (a ragged 256-query tile) and
    7 a chunk of one partial tile.  Eight hidden layers take the layer-wise
    forward either way (the streamed forward's LDS holds up to six layers'
    biases)."""
    q = synth.points(141, n, in_dim)
    y = (synth.points(142, n, 1)[:, 0] > 0.25).astype(np.uint8)
    theta = synth.init_params(143 + nh, in_dim, [256] * nh)
    out = {}
    for kern in (nb.TRAIN_AUTO, nb.TRAIN_LAYERWISE):
        b = nb.Bound(in_dim, nh, 256, nb.BF16)
        nb.nb_bound_set_train_kernel(b.handle, kern)
        nb.nb_bound_set_recompute(b.handle, every)
        b.set_params(theta)
        g = torch.empty(b.n_params, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        cnt = torch.empty(4, dtype=torch.int64, device="cuda")
        nb.nb_bound_loss_grad(b.handle, cuda(q), cuda(y), 7.0, 1.0, g, loss, cnt)
        out[kern] = (host(g).astype(np.float64), float(host(loss)[0]), host(cnt))
    gs, ls, cs = out[nb.TRAIN_AUTO]
    gl, ll, cl = out[nb.TRAIN_LAYERWISE]
    assert np.array_equal(cs, cl)
    assert abs(ls - ll) <= 1e-5 * abs(ll)
    layers_s = mlp.unpack(gs, in_dim, [256] * nh)
    layers_l = mlp.unpack(gl, in_dim, [256] * nh)
    for k, ((Ws, bs), (Wl, bl)) in enumerate(zip(layers_s[:-1], layers_l[:-1])):
        assert np.array_equal(Ws, Wl), k
        if k == 0:
            assert np.array_equal(bs, bl)
        else:
            assert _rel_frob(bs, bl) <= 1e-5, k
    (Ws, bs), (Wl, bl) = layers_s[-1], layers_l[-1]
    assert _rel_frob(Ws, Wl) <= 1e-5
    assert abs(float(bs[0]) - float(bl[0])) <= 1e-5 * max(abs(float(bl[0])), float(np.abs(Wl).max()))


@pytest.mark.parametrize("in_dim,width,nh", [(6, 128, 4), (4, 64, 3), (6, 32, 2)])
def test_loss_grad_bf16_fused_multi_tile(in_dim, width, nh):
    """The fused kernel against the oracle on a batch whose chunks hold
    several tiles of queries (70001: chunks of 320, the last tile half full)."""
    n = 70001
    q = synth.points(134, n, in_dim)
    y = (synth.points(135, n, 1)[:, 0] > 0.2).astype(np.uint8)
    _bf16_grad_check(in_dim, width, nh, q, y, 9.0, 1.5)


@pytest.mark.parametrize("in_dim,width,nh", [(4, 256, 6), (6, 128, 4), (3, 256, 8), (6, 64, 5), (6, 32, 3)])
def test_bf16_recompute_bit_identical(in_dim, width, nh):
    """Checkpointed activation recomputation gives the same gradient bits as
    keeping every activation, for several checkpoint intervals (layer-wise
    kernels: the fused one keeps no activations in memory)."""
    n = 3001
    q = synth.points(111, n, in_dim)
    y = (synth.points(112, n, 1)[:, 0] > 0.1).astype(np.uint8)
    theta = synth.init_params(113 + nh, in_dim, [width] * nh)
    b = nb.Bound(in_dim, nh, width, nb.BF16)
    nb.nb_bound_set_train_kernel(b.handle, nb.TRAIN_LAYERWISE)
    b.set_params(theta)
    grads = {}
    for every in (0, 2, 3, nh):
        nb.nb_bound_set_recompute(b.handle, every)
        g = torch.empty(b.n_params, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        nb.nb_bound_loss_grad(b.handle, cuda(q), cuda(y), 5.0, 1.0, g, loss)
        grads[every] = bits(host(g))
    for every in (2, 3, nh):
        assert np.array_equal(grads[every], grads[0]), every


def test_bf16_recompute_training_step(c2_grid):
    """A fused training step with recomputation matches the one without."""
    _, _, grid = c2_grid
    ind = nb.Indicator.voxels(cuda(grid), 128)
    theta0 = synth.init_params(4003, 6, [128] * 4)
    out = []
    for every in (0, 2):
        b = nb.Bound(6, 4, 128, nb.BF16)
        nb.nb_bound_set_train_kernel(b.handle, nb.TRAIN_LAYERWISE)
        nb.nb_bound_set_recompute(b.handle, every)
        b.set_params(theta0)
        for t in range(3):
            nb.nb_bound_train_step(b.handle, ind.handle, nb.RAY, 9, t, 5000, 3.0, 1.0, 1e-3)
        out.append(bits(host(b.params())))
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("in_dim,width,nh", [(6, 128, 4), (4, 256, 6), (4, 256, 8), (3, 64, 3), (6, 32, 2)])
def test_forward_bf16_variants_identical(in_dim, width, nh):
    """Every tile-shape variant of the bfloat16 forward gives the same bits."""
    theta = synth.init_params(120 + nh, in_dim, [width] * nh)
    q = cuda(synth.points(121, 5003, in_dim))
    b = nb.Bound(in_dim, nh, width, nb.BF16)
    b.set_params(theta)
    ref = None
    for v in range(nb.nb_bound_num_variants(b.handle)):
        nb.nb_bound_set_variant(b.handle, v)
        z, _ = b.forward(q)
        zb = bits(host(z))
        if ref is None:
            ref = zb
        assert np.array_equal(zb, ref), v


# ------------------------------------------------------------ early-out

@pytest.mark.parametrize("first,second,n", [
    ((3, 32, 1, "f32"), (3, 64, 3, "f32"), 70001),
    ((6, 32, 2, "bf16"), (6, 128, 4, "bf16"), 4099),
    ((4, 16, 2, "f32"), (4, 256, 6, "bf16"), 3001),
    ((3, 32, 1, "f32"), (3, 64, 3, "f32"), 1),
])
def test_early_out(first, second, n):
    """h = h_first AND h_second, the second bound evaluated only on the first's
    positives (Sec. 3, "Neural Early-out"): equal bit for bit to the two
    bounds' own decisions, and to the oracle's outside the |z| < 1e-4 band."""
    nets = []
    q = synth.points(140, n, first[0])
    qs = synth.points(141, 2001, first[0])
    for k, (d, w, nh, p) in enumerate((first, second)):
        theta = synth.init_params(130 + k + w, d, [w] * nh)
        # output bias at minus the median logit: each bound reports about half positive
        theta[-1] -= np.median(mlp.forward(theta, d, [w] * nh, qs, bf16=(p == "bf16")))
        b = nb.Bound(d, nh, w, nb.BF16 if p == "bf16" else nb.F32)
        b.set_params(theta)
        nets.append((b, theta, d, [w] * nh, p == "bf16"))
    qd = cuda(q)
    h = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    nb.nb_early_out(nets[0][0].handle, nets[1][0].handle, qd, h, cnt)
    h = host(h)
    z1, h1 = nets[0][0].forward(qd)
    z2, h2 = nets[1][0].forward(qd)
    h1, h2 = host(h1), host(h2)
    assert np.array_equal(h, h1 & h2)
    assert int(host(cnt)[0]) == int(h1.sum())
    ref = []
    for b, theta, d, widths, bf in nets:
        ref.append(mlp.forward(theta, d, widths, q, bf16=bf))
    sure = (np.abs(ref[0]) > 1e-4) & (np.abs(ref[1]) > 1e-4)
    expect = L.decide(ref[0]) & L.decide(ref[1])
    assert np.array_equal(h[sure], expect[sure])
    if n > 1000:
        assert 0 < h1.sum() < n and 0 < h.sum() < h1.sum()


def test_inverted_bound_has_no_false_positives():
    """An inverted ("certainly hit") bound, trained with the FP weight on the
    schedule, reaches FP = 0 on held-out points while keeping true positives."""
    from paper_2310_06822_amd import trainer
    discs = synth.discs2d(1000, k=8)
    ind = nb.Indicator.discs2d(discs)
    b = nb.Bound(2, 3, 32, nb.F32)
    b.set_params(synth.init_params(4000, 2, [32] * 3))
    sched = trainer.Schedule(steps=1000, batch=4096, alpha_max=100.0, k=100, inc=50.0, max_iters=200,
                             val_n=1 << 16, lr_decay=0.98, inverted=True)
    res = trainer.train(b, ind, "point", 2000, sched, val_seed=5000)
    assert res.converged
    q = torch.empty((1 << 18, 2), dtype=torch.float32, device="cuda")
    nb.nb_sample_queries(nb.POINT, 2, 3000, 0, q)
    g = ind.query("point", q)
    tp, fp, tn, fn = b.counts(q, g).tolist()
    assert fp == 0
    assert tp > 0.5 * (tp + fn)   # it still certifies most of the inside


# ------------------------------------------------------ sine activations

SINE_SHAPES = [(3, 64, 2), (2, 32, 2), (3, 64, 3), (6, 64, 1), (4, 32, 3), (4, 80, 2), (8, 80, 2), (6, 80, 1)]


@pytest.mark.parametrize("in_dim,width,nh", SINE_SHAPES)
@pytest.mark.parametrize("n", [1, 17, 3005])
def test_forward_sine_parity(in_dim, width, nh, n):
    """Sinusoidal hidden layers (Sec. 3.4): logits within 1e-5 of the
    magnitude of their terms, decisions equal outside the band."""
    widths = [width] * nh
    theta = synth.init_params(140 + in_dim + width + nh, in_dim, widths)
    q = synth.points(141, n, in_dim)
    b = nb.Bound(in_dim, nh, width)
    nb.nb_bound_set_activation(b.handle, nb.SINE)
    b.set_params(theta)
    z, h = b.forward(cuda(q))
    z, h = host(z).astype(np.float64), host(h)
    ref = mlp.forward(theta, in_dim, widths, q, act="sine")
    s = mlp.abs_forward(theta, in_dim, widths, q, act="sine")
    assert np.all(np.abs(z - ref) <= 1e-5 * np.maximum(np.abs(ref), s))
    band = np.abs(ref) < 1e-4
    assert np.array_equal(h[~band], L.decide(ref)[~band])


def test_sine_activation_accuracy():
    """The kernels' sine against float64 sin: a 1 -> 32 -> 1 sine network with
    one neuron passing x through (weights 1 in and out, the rest 0) returns
    sin x exactly up to the activation's own error, here bounded by 2e-7 for
    |x| up to 2^16 (the reduced-argument path) and beyond (the fallback)."""
    theta = np.zeros(32 + 32 + 32 + 1, np.float32)   # W0 [32x1], b0, w_out [1x32], b_out
    theta[0] = 1.0
    theta[64] = 1.0
    b = nb.Bound(1, 1, 32)
    nb.nb_bound_set_activation(b.handle, nb.SINE)
    b.set_params(theta)
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.uniform(-8, 8, 20000), rng.uniform(-1000, 1000, 20000),
                        rng.uniform(-65536, 65536, 20000), rng.uniform(-3e6, 3e6, 2000),
                        np.float32([0.0, -0.0, np.pi / 2, np.pi, 65536.0, -65536.0, 65537.0, 1e-30])]).astype(np.float32)
    z, _ = b.forward(cuda(x[:, None]))
    err = np.abs(host(z).astype(np.float64) - np.sin(x.astype(np.float64)))
    assert err.max() <= 2e-7, (err.max(), x[err.argmax()])


def test_sine_derivative_accuracy():
    """The training kernel's cosine (the sine activation's derivative) against
    float64 cos: the same pass-through network trained on one query x at a
    time has dL/db0[0] = dL/dz * cos x and dL/db_out = dL/dz, so their ratio
    is cos x up to the activation's error and two roundings."""
    theta = np.zeros(32 + 32 + 32 + 1, np.float32)
    theta[0] = 1.0
    theta[64] = 1.0
    b = nb.Bound(1, 1, 32)
    nb.nb_bound_set_activation(b.handle, nb.SINE)
    b.set_params(theta)
    rng = np.random.default_rng(12)
    x = np.concatenate([rng.uniform(-8, 8, 40), rng.uniform(-1000, 1000, 40), rng.uniform(-65536, 65536, 40),
                        rng.uniform(-3e6, 3e6, 8),
                        np.float32([0.0, np.pi / 2, np.pi, -np.pi / 4, 65536.0, -65537.0])]).astype(np.float32)
    grad = torch.empty(b.n_params, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    y = cuda(np.ones(1, np.uint8))
    worst = 0.0
    for v in x:
        nb.nb_bound_loss_grad(b.handle, cuda(np.float32([[v]])), y, 1.0, 1.0, grad, loss)
        g = host(grad).astype(np.float64)
        assert g[96] != 0.0
        worst = max(worst, abs(g[32] / g[96] - np.cos(np.float64(v))))
    assert worst <= 3e-7, worst


@pytest.mark.parametrize("in_dim,width,nh", SINE_SHAPES)
def test_loss_grad_sine_parity(in_dim, width, nh):
    widths = [width] * nh
    theta = synth.init_params(150 + width + nh, in_dim, widths)
    n = 4099
    q = synth.points(151, n, in_dim)
    y = (synth.points(152, n, 1)[:, 0] > 0.3).astype(np.uint8)
    b = nb.Bound(in_dim, nh, width)
    nb.nb_bound_set_activation(b.handle, nb.SINE)
    b.set_params(theta)
    grad = torch.empty(b.n_params, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    nb.nb_bound_loss_grad(b.handle, cuda(q), cuda(y), 6.0, 1.0, grad, loss)
    z = mlp.forward(theta, in_dim, widths, q, act="sine")
    gref = mlp.backward(theta, in_dim, widths, q, L.dloss_dz(z, y, 6.0, 1.0), act="sine")
    assert abs(host(loss)[0] - L.loss(z, y, 6.0, 1.0)) <= 1e-5 * L.loss(z, y, 6.0, 1.0)
    g = host(grad).astype(np.float64)
    for (Wg, bg), (Wr, br) in zip(mlp.unpack(g, in_dim, widths), mlp.unpack(gref, in_dim, widths)):
        assert _rel_frob(Wg, Wr) <= 1e-5
        assert _rel_frob(bg, br) <= 1e-5


@pytest.mark.parametrize("in_dim,real,padded", [(3, 50, 64), (4, 75, 80)])
def test_sine_paper_architecture_padded(in_dim, real, padded):
    """The paper's sine networks (3 x 50 x 50 for 3-D points, 4 x 75 x 75 for
    4-D points) run zero-padded to 64 / 80: the same logits as the unpadded
    oracle network, and a training step leaves the padding at zero."""
    small, big = [real] * 2, [padded] * 2
    theta_s = synth.init_params(160, in_dim, small)
    theta = synth.pad_params(theta_s, in_dim, small, big)
    b = nb.Bound(in_dim, 2, padded)
    nb.nb_bound_set_activation(b.handle, nb.SINE)
    b.set_params(theta)
    q = synth.points(161, 5000, in_dim)
    z, _ = b.forward(cuda(q))
    ref = mlp.forward(theta_s, in_dim, small, q, act="sine")
    s = mlp.abs_forward(theta_s, in_dim, small, q, act="sine")
    assert np.all(np.abs(host(z) - ref) <= 1e-5 * np.maximum(np.abs(ref), s))
    if in_dim == 3:
        ind = nb.Indicator.voxels(cuda(I.voxelize_metaballs(*synth.metaballs3d(1001, k=16), 64)), 64)
    else:
        ind = nb.Indicator.metaballs4d(*synth.metaballs4d(1005, k=24))
    for t in range(3):
        nb.nb_bound_train_step(b.handle, ind.handle, nb.POINT, 5, t, 8192, 10.0)
    th = host(b.params())
    mask = synth.pad_params(np.ones_like(theta_s), in_dim, small, big) != 0
    assert np.all(th[~mask] == 0) and np.any(th[mask] != theta[mask])


def test_sine_unsupported_shapes():
    b = nb.Bound(6, 4, 128, nb.BF16)
    with pytest.raises(nb.NBError):
        nb.nb_bound_set_activation(b.handle, nb.SINE)
    b = nb.Bound(3, 4, 64)
    with pytest.raises(nb.NBError):
        nb.nb_bound_set_activation(b.handle, nb.SINE)
    with pytest.raises(nb.NBError):   # width 80 holds at most two hidden layers
        nb.Bound(4, 3, 80)


def _oracle_recount(theta, in_dim, widths, q, g, h, bf16=False, act="relu", tol=0.0, chunk=1 << 16):
    """Conservativeness recounted by the oracle (Sec. 3.1: h >= g): on every
    row whose exact answer is 1 (only those can be false negatives), the
    float64 oracle's decision with the trained weights, against the GPU's.
    Returns (oracle FN outside the band |z| < 1e-4, rows in the band, rows
    where the two decisions differ although |z| >= 1e-4 and, with tol > 0,
    |z| > tol max(|z|, s) (the logit bar), positive rows)."""
    rows = np.nonzero(g)[0]
    fn = band = differ = 0
    for a in range(0, rows.size, chunk):
        r = rows[a:a + chunk]
        z = mlp.forward(theta, in_dim, widths, q[r], bf16=bf16, act=act)
        sure = ~(np.abs(z) < 1e-4)
        d = L.decide(z)
        fn += int(((d == 0) & sure).sum())
        band += int((~sure).sum())
        if tol > 0:
            s = mlp.abs_forward(theta, in_dim, widths, q[r], bf16=bf16, act=act)
            sure = sure & (np.abs(z) > tol * np.maximum(np.abs(z), s))
        differ += int(((d != h[r]) & sure).sum())
    return fn, band, differ, int(rows.size)


def _check_schedule(res, sched):
    """The FN weights and learning rates the continuation trained with follow
    the oracle's schedule for the validation FN counts the run saw."""
    from oracle import train as T
    ref = T.continuation(res.val_fn_history, sched.alpha_max, sched.inc, sched.lr, sched.patience,
                         sched.max_iters, sched.lr_decay, sched.lr_min)
    assert res.alpha_history == ref["alpha"]
    assert np.allclose(res.lr_history, ref["lr"], rtol=1e-9)
    assert (res.iters, res.converged, res.alpha_final) == (ref["iters"], ref["converged"], ref["alpha_final"])


def test_trained_bound_gain_over_exact_test_alone(c2_grid):
    """What the learned part buys (Sec. 6): a bound trained on the device with
    Alg. 1 (ramp + step-wise schedule) is conservative on held-out queries, so
    the cascade returns exactly the exact test's answers while running the
    exact test on a small fraction of the queries; without the bound every
    query needs the exact test.  The oracle recounts the false negatives with
    the trained weights, and the schedule the run took is the oracle's."""
    from paper_2310_06822_amd import trainer
    _, _, grid = c2_grid
    ind = nb.Indicator.voxels(cuda(grid), 128)
    b = nb.Bound(3, 3, 64, nb.F32)
    b.set_params(synth.init_params(4001, 3, [64] * 3))
    sched = trainer.Schedule(steps=5000, batch=1 << 16, alpha_max=100.0, k=250, inc=50.0, max_iters=200,
                             val_n=1 << 22)
    res = trainer.train(b, ind, "point", 2001, sched, val_seed=5001)
    _check_schedule(res, sched)
    n = 1 << 22
    q = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    nb.nb_sample_queries(nb.POINT, 3, 3001, 0, q)
    g = ind.query("point", q)
    ans = torch.empty(n, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    nb.nb_cascade(b.handle, ind.handle, nb.POINT, q, ans, cnt)
    n_exact = int(host(cnt)[0])
    positives = int(host(g).sum())
    assert res.converged
    assert torch.equal(ans, g)                  # conservative: the cascade is the exact test
    assert n_exact < 0.25 * n                   # the exact test runs on under a quarter of the queries
    assert n_exact >= positives                 # (it still sees every true hit)
    _, h = b.forward(q)
    fn, band, differ, pos = _oracle_recount(host(b.params()), 3, [64] * 3, host(q), host(g), host(h))
    assert pos == positives and fn == 0 and differ == 0


def test_trained_bf16_bound_oracle_recount(c2_grid):
    """A bfloat16 bound trained on the device (ramp + step-wise schedule): the
    oracle (float64, hidden layers in bfloat16) recounts the held-out false
    negatives with the exported weights, and its decisions on the positives
    agree with the GPU's outside the band, so both count the same false
    negatives there.  The schedule stops after six FN-free validation draws of
    2^22, which bounds the held-out FN rate statistically, not at zero: at
    most 2 in 2^22 here."""
    from paper_2310_06822_amd import trainer
    _, _, grid = c2_grid
    ind = nb.Indicator.voxels(cuda(grid), 128)
    b = nb.Bound(3, 3, 64, nb.BF16)
    b.set_params(synth.init_params(4011, 3, [64] * 3))
    sched = trainer.Schedule(steps=4000, batch=1 << 16, alpha_max=100.0, k=250, inc=50.0, max_iters=200,
                             val_n=1 << 22, lr_decay=0.99)
    res = trainer.train(b, ind, "point", 2011, sched, val_seed=5011)
    _check_schedule(res, sched)
    assert res.converged
    n = 1 << 22
    q = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    nb.nb_sample_queries(nb.POINT, 3, 3011, 0, q)
    g = ind.query("point", q)
    _, h = b.forward(q)
    tp, fp, tn, fn_gpu = b.counts(q, g).tolist()
    fn, band, differ, pos = _oracle_recount(host(b.params()), 3, [64] * 3, host(q), host(g), host(h), bf16=True,
                                            tol=1e-3)
    assert differ == 0 and pos == tp + fn_gpu
    assert fn <= fn_gpu <= fn + band
    assert fn_gpu <= 2


def _with_nonfinite(q, seed, frac=0.03):
    """A copy of q with a non-finite value (NaN, +inf or -inf) in a random
    column of about frac of the rows; also the mask of those rows."""
    g = np.random.default_rng(seed)
    bad = g.random(q.shape[0]) < frac
    bad[0] = bad[-1] = True
    qb = q.copy()
    vals = np.array([np.nan, np.inf, -np.inf], np.float32)
    for r in np.nonzero(bad)[0]:
        qb[r, g.integers(q.shape[1])] = vals[g.integers(3)]
    return qb, bad


def _check_nonfinite(forward, q, seed):
    qb, bad = _with_nonfinite(q, seed)
    z, h = forward(cuda(qb))
    z0, h0 = forward(cuda(q))
    z, h, z0, h0 = host(z), host(h), host(z0), host(h0)
    assert np.all(np.isnan(z[bad])) and np.all(h[bad] == 1)
    assert np.array_equal(bits(z[~bad]), bits(z0[~bad])) and np.array_equal(h[~bad], h0[~bad])


@pytest.mark.parametrize("prec,act,d,w,nh", [(nb.F32, "relu", 3, 64, 3), (nb.F32, "relu", 5, 32, 2),
                                             (nb.F32, "sine", 3, 64, 2), (nb.BF16, "relu", 6, 128, 4),
                                             (nb.BF16, "relu", 4, 256, 3)])
def test_nonfinite_rows_decided_positive(prec, act, d, w, nh):
    """Boundary rule: a query row with a NaN or infinite value gets logit NaN
    and decision 1 (the conservative side); the other rows are untouched."""
    b = nb.Bound(d, nh, w, prec)
    if act == "sine":
        nb.nb_bound_set_activation(b.handle, nb.SINE)
    b.set_params(synth.init_params(150 + w, d, [w] * nh))
    _check_nonfinite(b.forward, synth.points(151, 3001, d), 152)


def test_nonfinite_rows_grouped_kdop_and_early_out():
    q = synth.points(160, 2001, 6)
    gr = nb.Group(6, [64, 128], 3)
    gr.set_params(np.concatenate([synth.init_params(161 + o, 6, [w] * 3) for o, w in enumerate([64, 128])]))
    qoff = cuda(np.array([0, 900, 2001], np.int64))
    _check_nonfinite(lambda x: gr.forward(x, qoff), q, 162)
    kd = nb.KDop(3, 4)
    kd.set_params(synth.kdop_init(3, 4, seed=163))
    q3 = synth.points(164, 2001, 3)
    _check_nonfinite(lambda x: kd.forward("point", x), q3, 165)
    first, second = nb.Bound(3, 1, 32), nb.Bound(3, 3, 64)
    first.set_params(synth.init_params(166, 3, [32]))
    second.set_params(synth.init_params(167, 3, [64] * 3))
    qb, bad = _with_nonfinite(q3, 168)
    h = torch.empty(q3.shape[0], dtype=torch.uint8, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    nb.nb_early_out(first.handle, second.handle, cuda(qb), h, cnt)
    assert np.all(host(h)[bad] == 1)


def test_nonfinite_training_is_reported_on_sync(c2_grid):
    """A training step that meets a non-finite loss or gradient is reported
    (NB_ERR_NONFINITE) by the next sync call, which then clears the flag; a
    healthy run reports nothing."""
    _, _, grid = c2_grid
    ind = nb.Indicator.voxels(cuda(grid), 128)
    for prec, d, w, nh, kind in ((nb.F32, 3, 64, 3, nb.POINT), (nb.BF16, 6, 128, 4, nb.RAY)):
        b = nb.Bound(d, nh, w, prec)
        b.set_params(synth.init_params(170 + w, d, [w] * nh))
        for t in range(3):
            nb.nb_bound_train_step(b.handle, ind.handle, kind, 171, t, 4096, 1.0)
        nb.nb_bound_sync(b.handle)
        b.set_params(np.full(b.n_params, 3e38, np.float32))   # the logits overflow
        nb.nb_bound_train_step(b.handle, ind.handle, kind, 171, 3, 4096, 1.0)
        with pytest.raises(nb.NBError) as e:
            nb.nb_bound_sync(b.handle)
        assert "non-finite" in str(e.value)
        nb.nb_bound_sync(b.handle)   # cleared
    gr = nb.Group(3, [32, 64], 2)
    gr.set_params(np.concatenate([synth.init_params(172 + o, 3, [w] * 2) for o, w in enumerate([32, 64])]))
    gs = [I.voxelize_metaballs(*synth.metaballs3d(173 + o, k=6), 32) for o in range(2)]
    gr.set_voxels(cuda(np.concatenate(gs)), [32, 32])
    nb.nb_group_train_step(gr.handle, 2, nb.POINT, 174, 0, 1024, 1.0)
    nb.nb_group_sync(gr.handle)
    th = host(gr.params())
    th[: gr.offsets[1]] = 3e38
    gr.set_params(th)
    nb.nb_group_train_step(gr.handle, 2, nb.POINT, 174, 1, 1024, 1.0)
    with pytest.raises(nb.NBError):
        nb.nb_group_sync(gr.handle)
    nb.nb_group_sync(gr.handle)
    kd = nb.KDop(3, 4)
    kd.set_params(np.full(3 * 4 + 2 * 4 + 1, 3e38, np.float32))
    nb.nb_kdop_train_step(kd.handle, ind.handle, nb.POINT, 176, 0, 4096, 1.0, 1.0, 1e-3)
    with pytest.raises(nb.NBError):
        nb.nb_kdop_sync(kd.handle)
    nb.nb_kdop_sync(kd.handle)
