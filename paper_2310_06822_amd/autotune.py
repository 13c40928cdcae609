"""Tile-shape tuner for the bound's forward kernels.

Every forward variant of a bound computes the same logits; they differ in how
many 16-query blocks a wave carries and how many waves share the weights a
workgroup holds in LDS.  The tuner times each variant on the caller's query
batch with HIP events, keeps the fastest, and remembers the choice per
(precision, in_dim, width, n_hidden, batch size class, device).
"""

from __future__ import annotations

import time

import torch

from . import Bound, nb_bound_forward, nb_bound_num_variants, nb_bound_set_variant

_CACHE: dict = {}


def _key(b: Bound, n: int):
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return (b.precision, b.in_dim, b.width, b.n_hidden, max(n, 1).bit_length(), props.name)


def time_variants(b: Bound, q: torch.Tensor, reps: int = 5) -> list:
    """Mean milliseconds per forward (decision only) for every variant."""
    n = q.shape[0]
    h = torch.empty(n, dtype=torch.uint8, device=q.device)
    out = []
    for v in range(nb_bound_num_variants(b.handle)):
        nb_bound_set_variant(b.handle, v)
        nb_bound_forward(b.handle, q, h=h)                  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            nb_bound_forward(b.handle, q, h=h)
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / reps)
    return out


def tune(b: Bound, q: torch.Tensor, reps: int = 5) -> int:
    """Select the fastest forward variant for this bound and batch; returns it."""
    k = _key(b, q.shape[0])
    if k not in _CACHE:
        ms = time_variants(b, q, reps)
        _CACHE[k] = (min(range(len(ms)), key=ms.__getitem__), ms)
    v = _CACHE[k][0]
    nb_bound_set_variant(b.handle, v)
    return v


def report() -> dict:
    return {str(k): {"variant": v, "ms": ms} for k, (v, ms) in _CACHE.items()}


def _time_group(group, q: torch.Tensor, qoff: torch.Tensor, h: torch.Tensor, reps: int) -> float:
    from . import nb_group_forward
    nb_group_forward(group.handle, group.n_obj, group.in_dim, q, qoff, h=h)   # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        nb_group_forward(group.handle, group.n_obj, group.in_dim, q, qoff, h=h)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def time_group_variants(group, q: torch.Tensor, qoff: torch.Tensor, reps: int = 5) -> list:
    """Mean milliseconds per grouped forward (decision only) for every tile
    shape, the same shape for every width class."""
    from . import nb_group_num_variants, nb_group_set_variant
    h = torch.empty(q.shape[0], dtype=torch.uint8, device=q.device)
    out = []
    for v in range(nb_group_num_variants(group.handle)):
        nb_group_set_variant(group.handle, v)
        out.append(_time_group(group, q, qoff, h, reps))
    return out


def tune_group(group, q: torch.Tensor, qoff: torch.Tensor, reps: int = 5) -> dict:
    """Select the fastest grouped-forward tile shape of every width class for
    this group and query layout (keyed by the width mix, depth and batch size
    class); returns {width: variant}.  The classes run as separate launches,
    so their times add and each class is tuned with the others held fixed."""
    from . import nb_group_num_variants, nb_group_set_width_variant
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    k = ("group", group.in_dim, group.n_hidden, tuple(sorted(group.widths)), max(q.shape[0], 1).bit_length(),
         props.name)
    if k not in _CACHE:
        h = torch.empty(q.shape[0], dtype=torch.uint8, device=q.device)
        nv = nb_group_num_variants(group.handle)
        best, ms_all = {}, {}
        for w in sorted(set(group.widths)):
            ms = []
            for v in range(nv):
                nb_group_set_width_variant(group.handle, w, v)
                ms.append(_time_group(group, q, qoff, h, reps))
            best[w] = min(range(nv), key=ms.__getitem__)
            ms_all[w] = ms
            nb_group_set_width_variant(group.handle, w, best[w])
        _CACHE[k] = (best, ms_all)
    best = _CACHE[k][0]
    for w, v in best.items():
        nb_group_set_width_variant(group.handle, w, v)
    return dict(best)


def tune_hierarchy(hier, q: torch.Tensor, reps: int = 3) -> dict:
    """Select the grouped-forward tile shape of every width class under which
    a whole hierarchy query (every level) runs fastest for these rows, one
    class at a time with the others held fixed; returns {width: variant}."""
    from . import nb_group_num_variants, nb_group_set_width_variant
    g = hier.group
    best = {}
    for w in sorted(set(g.widths)):
        best_v, best_ms = 0, float("inf")
        for v in range(nb_group_num_variants(g.handle)):
            nb_group_set_width_variant(g.handle, w, v)
            hier.query(q)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                hier.query(q)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            if ms < best_ms:
                best_v, best_ms = v, ms
        best[w] = best_v
        nb_group_set_width_variant(g.handle, w, best_v)
    return best
