"""The allocation-free cascade (nb_cascade_noalloc) against nb_cascade,
through the C ABI: identical answers and exact-test counts on two calls in a
row (the second with fewer queries, so stale entries of the shared index list
must not leak into it), for a float32 and a bfloat16 bound; sizes beyond the
array's limit are refused before any work."""

import numpy as np
import pytest
import torch

import synth
from oracle import indicators as I, mlp, sampling

pytestmark = pytest.mark.gpu

nb = pytest.importorskip("paper_2310_06822_amd")


@pytest.mark.parametrize("prec,kind,in_dim,width,nh", [(nb.F32, "point", 3, 64, 3), (nb.BF16, "ray", 6, 128, 4)])
def test_cascade_noalloc_equals_cascade(prec, kind, in_dim, width, nh):
    c, r = synth.metaballs3d(1001, k=16)
    grid = I.voxelize_metaballs(c, r, 128)
    ind = nb.Indicator.voxels(torch.from_numpy(grid).cuda(), 128)
    b = nb.Bound(in_dim, nh, width, prec)
    k = nb.KINDS[kind]
    th = synth.init_params(90 + width, in_dim, [width] * nh)
    # output bias at the median logit: the bound calls about half the queries positive
    probe = sampling.sample(kind, 93, 0, 4096, 3)
    th[-1] -= np.float32(np.median(mlp.forward(th, in_dim, [width] * nh, probe, bf16=prec == nb.BF16)))
    b.set_params(th)
    for n, seed in [((1 << 22) - 5, 91), (100_003, 92)]:
        q = torch.empty((n, in_dim), dtype=torch.float32, device="cuda")
        nb.nb_sample_queries(k, 3, seed, 0, q)
        a_ref = torch.empty(n, dtype=torch.uint8, device="cuda")
        c_ref = torch.empty(1, dtype=torch.int64, device="cuda")
        nb.nb_cascade(b.handle, ind.handle, k, q, a_ref, c_ref)
        a = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        nb.nb_cascade_noalloc(b.handle, ind.handle, k, q, a, cnt)
        torch.cuda.synchronize()
        assert torch.equal(a, a_ref), (n, kind)
        assert int(cnt.item()) == int(c_ref.item()) > 0
        assert 0 < int(cnt.item()) < n


def test_cascade_noalloc_size_limit():
    ind = nb.Indicator.discs2d(synth.discs2d(1000))
    b = nb.Bound(2, 3, 32)
    b.set_params(synth.init_params(1, 2, [32] * 3))
    n = nb.CASCADE_NOALLOC_MAX + 1
    q = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    with pytest.raises(nb.NBError) as e:
        nb.nb_cascade_noalloc(b.handle, ind.handle, nb.POINT, q, a, cnt)
    assert e.value.status == 1   # NB_ERR_INVALID_ARG
