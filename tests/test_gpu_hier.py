"""GPU parity of neural bounding hierarchies (Sec. 3.3) against the CPU
oracle through the C ABI: the (row, leaf) pairs of the level-by-level
descent equal the oracle's, leaf by leaf, for every row whose logits are
clear of the threshold at every node (|z - tau| above the bfloat16 forward's
tolerance 1e-3 max(|z|, s); such rows are few and are left out on both
sides).  Rows come out in increasing order inside each leaf's segment."""

import numpy as np
import pytest
import torch

import synth
from oracle import hierarchy as H, loss as L, mlp

pytestmark = pytest.mark.gpu

nb = pytest.importorskip("paper_2310_06822_amd")


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def complete(fan, depth):
    """Breadth-first child ranges of a complete tree."""
    cb, ce, nxt, level = [], [], 1, [0]
    for d in range(depth):
        nodes = fan ** d
        for _ in range(nodes):
            if d + 1 < depth:
                cb.append(nxt)
                ce.append(nxt + fan)
                nxt += fan
            else:
                cb.append(0)
                ce.append(0)
    return cb, ce


IRREGULAR = ([1, 4, 0, 6, 0, 0, 9, 0, 0, 0], [4, 6, 0, 9, 0, 0, 10, 0, 0, 0])
CHAIN = ([1, 2, 3, 0], [2, 3, 4, 0])

TREES = {
    "complete_4x3": (complete(4, 3), 3, 3, {0: 128, 1: 64, 2: 32}),
    "irregular": (IRREGULAR, 6, 2, None),
    "single": (([0], [0]), 3, 4, {0: 32}),
    "chain": (CHAIN, 4, 3, None),
}


def _setup(name, seed, q, accept=0.6):
    (cb, ce), in_dim, nh, wl = TREES[name]
    _, level, _ = H.structure(cb, ce)
    rng = np.random.default_rng(seed)
    widths = [wl[level[v]] if wl else int(rng.choice([32, 64, 128])) for v in range(len(cb))]
    thetas = []
    for v, w in enumerate(widths):
        th = synth.init_params(seed + v, in_dim, [w] * nh)
        z = mlp.forward(th, in_dim, [w] * nh, q, bf16=True)
        th[-1] -= np.float32(np.quantile(z, 1.0 - accept))   # about `accept` of the rows pass each node
        thetas.append(th)
    gr = nb.Group(in_dim, widths, nh)
    gr.set_params(np.concatenate(thetas).astype(np.float32))
    return cb, ce, in_dim, nh, widths, thetas, gr


def _oracle(cb, ce, in_dim, nh, widths, thetas, q):
    Z = [mlp.forward(th, in_dim, [w] * nh, q, bf16=True) for th, w in zip(thetas, widths)]
    S = [mlp.abs_forward(th, in_dim, [w] * nh, q, bf16=True) for th, w in zip(thetas, widths)]
    amb = np.zeros(q.shape[0], bool)
    for z, s in zip(Z, S):
        amb |= np.abs(z - L.tau()) <= 1e-3 * np.maximum(np.abs(z), s)
    out = H.traverse(lambda v, rows: L.decide(Z[v][rows]).astype(bool), cb, ce, q.shape[0])
    return out, amb


def _compare(leaf_off, qidx, out, amb, rows=None):
    """GPU pairs vs the oracle's, per leaf; rows: the oracle's row -> GPU row map."""
    assert leaf_off[0] == 0 and np.all(np.diff(leaf_off) >= 0) and leaf_off[-1] == qidx.size
    for r, ref in enumerate(out):
        got = qidx[leaf_off[r]:leaf_off[r + 1]].astype(np.int64)
        assert np.all(np.diff(got) > 0), r
        if rows is not None:
            got = np.nonzero(np.isin(rows, got))[0]
        keep_g = got[~amb[got]]
        keep_r = ref[~amb[ref]]
        assert np.array_equal(keep_g, keep_r), f"leaf {r}: {keep_g.size} vs {keep_r.size} rows"


@pytest.mark.parametrize("name", list(TREES))
@pytest.mark.parametrize("n", [1, 777, 20001])
def test_hier_query_parity(name, n):
    in_dim = TREES[name][1]
    q = synth.points(600 + n, n, in_dim)
    cb, ce, in_dim, nh, widths, thetas, gr = _setup(name, 610, q)
    hr = nb.Hierarchy(gr, cb, ce)
    leaf_off, qidx = hr.query(cuda(q))
    out, amb = _oracle(cb, ce, in_dim, nh, widths, thetas, q)
    if n > 1:
        assert amb.mean() < 0.5    # most rows are clear of the threshold at every node
    _compare(host(leaf_off), host(qidx), out, amb)
    if n > 1:
        assert 0 < qidx.numel()


def test_hier_query_large_sampled():
    """2^20 rows through 21 nodes (pairs per level in the millions: many scan
    blocks); the oracle checks a sample of 3000 rows."""
    n = 1 << 20
    q = synth.points(620, n, 3)
    sample = np.sort(np.random.default_rng(621).choice(n, 3000, replace=False))
    cb, ce, in_dim, nh, widths, thetas, gr = _setup("complete_4x3", 630, q[sample], accept=0.7)
    hr = nb.Hierarchy(gr, cb, ce)
    leaf_off, qidx = hr.query(cuda(q))
    out, amb = _oracle(cb, ce, in_dim, nh, widths, thetas, q[sample])
    _compare(host(leaf_off), host(qidx), out, amb, rows=sample)
    assert qidx.numel() > n // 10


def test_hier_accept_all_and_reuse():
    """Every node accepts everything: each leaf holds all rows, in order; a
    second query on the same handle (fewer rows) gives the same answer for
    its rows."""
    cb, ce = complete(3, 3)
    widths = [64] * len(cb)
    thetas = [synth.init_params(640 + v, 3, [w] * 2) for v, w in enumerate(widths)]
    for th in thetas:
        th[-1] = 1e3
    gr = nb.Group(3, widths, 2)
    gr.set_params(np.concatenate(thetas).astype(np.float32))
    hr = nb.Hierarchy(gr, cb, ce)
    for n in (5000, 123):
        q = cuda(synth.points(641 + n, n, 3))
        leaf_off, qidx = hr.query(q)
        assert np.array_equal(host(leaf_off), np.arange(hr.n_leaves + 1) * n)
        assert np.array_equal(host(qidx), np.tile(np.arange(n, dtype=np.int32), hr.n_leaves))
        assert hr.depth == 3 and list(hr.level_pairs()) == [n, 3 * n, 9 * n]


def test_hier_capacity_and_errors():
    q = synth.points(650, 777, 3)
    cb, ce, *_ , gr = _setup("complete_4x3", 651, q)
    hr = nb.Hierarchy(gr, cb, ce)
    leaf_off = torch.empty(hr.n_leaves + 1, dtype=torch.int64, device="cuda")
    small = torch.full((5,), -1, dtype=torch.int32, device="cuda")
    need = nb.nb_hier_query(hr.handle, 3, cuda(q), small, leaf_off, check=False)
    assert need > 5
    with pytest.raises(nb.NBError):
        nb.nb_hier_query(hr.handle, 3, cuda(q), small, leaf_off)
    full = torch.empty(need, dtype=torch.int32, device="cuda")
    assert nb.nb_hier_query(hr.handle, 3, cuda(q), full, leaf_off) == need
    assert torch.equal(full[:5], small)    # the prefix that fitted was written the same way
    # malformed trees are refused
    with pytest.raises(nb.NBError):
        nb.Hierarchy(gr, [2] + [0] * (len(cb) - 1), [3] + [0] * (len(cb) - 1))
    with pytest.raises(ValueError):
        nb.Hierarchy(gr, [1, 0], [2, 0])   # two nodes described for a 21-object group
    leaf_nodes = hr.leaf_nodes
    assert list(leaf_nodes) == H.structure(cb, ce)[2]
