"""Neural Bounding on MI355X: Python binding of libnbound (HIP, gfx950).

The functions below carry the names of the C ABI in include/nbound.h and do
argument marshalling only: every step of the hot path (sampling, exact
queries, MLP forward / backward, loss, Adam) runs in the library's kernels.
Tensors must be contiguous CUDA (HIP) tensors of the documented dtype; the
work is enqueued on torch's current stream unless a stream is given.

Higher-level helpers (Indicator, Bound) own the C handles.
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib

POINT, RAY, BOX, PLANE = 0, 1, 2, 3
KINDS = {"point": POINT, "ray": RAY, "box": BOX, "plane": PLANE}
F32, BF16 = 0, 1
EPS_OUT = 1e-5

STATUS = {0: "NB_OK", 1: "NB_ERR_INVALID_ARG", 2: "NB_ERR_NO_DEVICE", 3: "NB_ERR_HIP", 4: "NB_ERR_OOM",
          5: "NB_ERR_NONFINITE", 6: "NB_ERR_UNSUPPORTED"}


class NBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def lib():
    return _lib.load()


def _check(st: int):
    if st != 0:
        raise NBError(st, lib().nb_last_error().decode(errors="replace"))


def _dev(t, dtype, name, numel=None):
    """Device pointer of a contiguous CUDA tensor of the given dtype (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _host(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------------- C ABI

def nb_version():
    ma, mi = C.c_int(), C.c_int()
    _check(lib().nb_version(C.byref(ma), C.byref(mi)))
    return ma.value, mi.value


def nb_device_count() -> int:
    n = C.c_int()
    _check(lib().nb_device_count(C.byref(n)))
    return n.value


def nb_indicator_discs2d(discs) -> C.c_void_p:
    a, p = _host(discs)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("discs must be [k, 3]")
    h = C.c_void_p()
    _check(lib().nb_indicator_discs2d(p, a.shape[0], C.byref(h)))
    return h


def nb_indicator_voxels(grid: torch.Tensor, n: int) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().nb_indicator_voxels(_dev(grid, torch.uint8, "grid", n ** 3), int(n), C.byref(h)))
    return h


def nb_indicator_metaballs4d(a, b, radii, iso: float = 1.0) -> C.c_void_p:
    aa, pa = _host(a)
    bb, pb = _host(b)
    rr, pr = _host(radii)
    k = rr.shape[0]
    if aa.shape != (k, 3) or bb.shape != (k, 3):
        raise ValueError("a and b must be [k, 3], radii [k]")
    h = C.c_void_p()
    _check(lib().nb_indicator_metaballs4d(pa, pb, pr, k, float(iso), C.byref(h)))
    return h


def nb_indicator_dim(ind) -> int:
    d = C.c_int()
    _check(lib().nb_indicator_dim(ind, C.byref(d)))
    return d.value


def nb_indicator_destroy(ind):
    _check(lib().nb_indicator_destroy(ind))


def nb_voxelize_metaballs(centres, radii, iso: float, n: int, grid: torch.Tensor, stream=None):
    cc, pc = _host(centres)
    rr, pr = _host(radii)
    if cc.shape != (rr.shape[0], 3):
        raise ValueError("centres must be [k, 3], radii [k]")
    _check(lib().nb_voxelize_metaballs(pc, pr, rr.shape[0], float(iso), int(n),
                                       _dev(grid, torch.uint8, "grid", n ** 3), _stream(stream)))


def _rows(q, d=None):
    if q.dim() != 2 or (d is not None and q.shape[1] != d):
        raise ValueError(f"queries must be [n, {d if d is not None else 'd'}]")
    return q.shape[0]


def _query_cols(kind: int, point_dim: int) -> int:
    return point_dim if kind == POINT else 6


def nb_query_exact(ind, kind: int, q: torch.Tensor, g: torch.Tensor, stream=None):
    n = _rows(q, _query_cols(int(kind), nb_indicator_dim(ind)))
    _check(lib().nb_query_exact(ind, int(kind), _dev(q, torch.float32, "q"), n,
                                _dev(g, torch.uint8, "g", n), _stream(stream)))


def nb_sample_queries(kind: int, dim: int, seed: int, step: int, q: torch.Tensor, stream=None):
    n = _rows(q, _query_cols(int(kind), int(dim)))
    _check(lib().nb_sample_queries(int(kind), int(dim), int(seed), int(step), n,
                                   _dev(q, torch.float32, "q"), _stream(stream)))


def nb_bound_create(in_dim: int, n_hidden: int, width: int, precision: int = F32) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().nb_bound_create(int(in_dim), int(n_hidden), int(width), int(precision), C.byref(h)))
    return h


def nb_bound_destroy(b):
    _check(lib().nb_bound_destroy(b))


def nb_bound_num_params(b) -> int:
    n = C.c_int64()
    _check(lib().nb_bound_num_params(b, C.byref(n)))
    return n.value


def nb_bound_shape(b):
    """(in_dim, n_hidden, width, precision)."""
    v = [C.c_int() for _ in range(4)]
    _check(lib().nb_bound_shape(b, *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)


def nb_bound_num_variants(b) -> int:
    n = C.c_int()
    _check(lib().nb_bound_num_variants(b, C.byref(n)))
    return n.value


RELU, SINE = 0, 1


def nb_bound_set_activation(b, activation: int):
    _check(lib().nb_bound_set_activation(b, int(activation)))


def nb_bound_set_recompute(b, every: int):
    _check(lib().nb_bound_set_recompute(b, int(every)))


TRAIN_AUTO, TRAIN_LAYERWISE = 0, 1


def nb_bound_set_train_kernel(b, kernel: int, stream=None):
    _check(lib().nb_bound_set_train_kernel(b, int(kernel), _stream(stream)))


def nb_bound_set_variant(b, variant: int):
    _check(lib().nb_bound_set_variant(b, int(variant)))


def nb_bound_set_params(b, theta: torch.Tensor, stream=None):
    _check(lib().nb_bound_set_params(b, _dev(theta, torch.float32, "theta"), theta.numel(), _stream(stream)))


def nb_bound_get_params(b, theta: torch.Tensor, stream=None):
    _check(lib().nb_bound_get_params(b, _dev(theta, torch.float32, "theta"), theta.numel(), _stream(stream)))


def nb_bound_get_state(b, m: torch.Tensor, v: torch.Tensor, stream=None) -> int:
    t = C.c_int64()
    _check(lib().nb_bound_get_state(b, _dev(m, torch.float32, "m"), _dev(v, torch.float32, "v", m.numel()),
                                    m.numel(), C.byref(t), _stream(stream)))
    return t.value


def nb_bound_set_state(b, m: torch.Tensor, v: torch.Tensor, step: int, stream=None):
    _check(lib().nb_bound_set_state(b, _dev(m, torch.float32, "m"), _dev(v, torch.float32, "v", m.numel()),
                                    m.numel(), int(step), _stream(stream)))


def nb_bound_save(b, stream=None) -> bytes:
    """Checkpoint of the bound's training state (parameters, Adam moments
    and step) as bytes."""
    size = C.c_size_t(0)
    _check(lib().nb_bound_save(b, None, C.byref(size), _stream(stream)))
    buf = C.create_string_buffer(size.value)
    _check(lib().nb_bound_save(b, C.cast(buf, C.c_void_p), C.byref(size), _stream(stream)))
    return buf.raw[:size.value]


def nb_bound_load(b, data: bytes, stream=None):
    buf = C.create_string_buffer(bytes(data), len(data))
    _check(lib().nb_bound_load(b, C.cast(buf, C.c_void_p), len(data), _stream(stream)))


def nb_bound_forward(b, q: torch.Tensor, eps: float = EPS_OUT, logits=None, h=None, g=None, counts=None,
                     stream=None):
    n = _rows(q, nb_bound_shape(b)[0])
    _check(lib().nb_bound_forward(b, _dev(q, torch.float32, "q"), n, float(eps),
                                  _dev(logits, torch.float32, "logits", n), _dev(h, torch.uint8, "h", n),
                                  _dev(g, torch.uint8, "g", n), _dev(counts, torch.int64, "counts", 4),
                                  _stream(stream)))


def nb_bound_loss_grad(b, q: torch.Tensor, y: torch.Tensor, alpha: float, beta: float, grad: torch.Tensor,
                       loss=None, counts=None, stream=None):
    n = _rows(q, nb_bound_shape(b)[0])
    _check(lib().nb_bound_loss_grad(b, _dev(q, torch.float32, "q"), _dev(y, torch.uint8, "y", n), n,
                                    float(alpha), float(beta), _dev(grad, torch.float32, "grad", nb_bound_num_params(b)),
                                    _dev(loss, torch.float32, "loss", 1), _dev(counts, torch.int64, "counts", 4),
                                    _stream(stream)))


def nb_bound_adam_step(b, grad: torch.Tensor, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                       adam_eps: float = 1e-8, lam1: float = 0.0, lam2: float = 0.0, stream=None):
    _check(lib().nb_bound_adam_step(b, _dev(grad, torch.float32, "grad", nb_bound_num_params(b)), float(lr), float(beta1), float(beta2),
                                    float(adam_eps), float(lam1), float(lam2), _stream(stream)))


def nb_bound_train_step(b, ind, kind: int, seed: int, step: int, batch: int, alpha: float, beta: float = 1.0,
                        lr: float = 1e-3, lam1: float = 0.0, lam2: float = 0.0, loss=None, counts=None,
                        stream=None):
    _check(lib().nb_bound_train_step(b, ind, int(kind), int(seed), int(step), int(batch), float(alpha),
                                     float(beta), float(lr), float(lam1), float(lam2),
                                     _dev(loss, torch.float32, "loss", 1), _dev(counts, torch.int64, "counts", 4),
                                     _stream(stream)))


def nb_cascade(b, ind, kind: int, q: torch.Tensor, answer: torch.Tensor, n_exact: torch.Tensor,
               eps: float = EPS_OUT, stream=None):
    n = _rows(q, nb_bound_shape(b)[0])
    if _query_cols(int(kind), nb_indicator_dim(ind)) != q.shape[1]:
        raise ValueError("query width does not match the indicator and kind")
    _check(lib().nb_cascade(b, ind, int(kind), _dev(q, torch.float32, "q"), n, float(eps),
                            _dev(answer, torch.uint8, "answer", n), _dev(n_exact, torch.int64, "n_exact", 1),
                            _stream(stream)))


CASCADE_NOALLOC_MAX = 1 << 22


def nb_cascade_noalloc(b, ind, kind: int, q: torch.Tensor, answer: torch.Tensor, n_exact: torch.Tensor,
                       eps: float = EPS_OUT, stream=None):
    """nb_cascade with its index list in the library's per-GPU device array
    (no allocation; at most CASCADE_NOALLOC_MAX queries)."""
    n = _rows(q, nb_bound_shape(b)[0])
    if _query_cols(int(kind), nb_indicator_dim(ind)) != q.shape[1]:
        raise ValueError("query width does not match the indicator and kind")
    _check(lib().nb_cascade_noalloc(b, ind, int(kind), _dev(q, torch.float32, "q"), n, float(eps),
                                    _dev(answer, torch.uint8, "answer", n), _dev(n_exact, torch.int64, "n_exact", 1),
                                    _stream(stream)))


def nb_early_out(first, second, q: torch.Tensor, h: torch.Tensor, n_second: torch.Tensor, eps: float = EPS_OUT,
                 stream=None):
    n = _rows(q, nb_bound_shape(first)[0])
    _check(lib().nb_early_out(first, second, _dev(q, torch.float32, "q"), n, float(eps), _dev(h, torch.uint8, "h", n),
                              _dev(n_second, torch.int64, "n_second", 1), _stream(stream)))


# ------------------------------------------------------------------ k-DOPs

def nb_kdop_forward(b, kind: int, q: torch.Tensor, eps: float = EPS_OUT, logits=None, h=None, g=None, counts=None,
                    stream=None):
    n = q.shape[0]
    _check(lib().nb_kdop_forward(b, int(kind), _dev(q, torch.float32, "q"), n, float(eps),
                                 _dev(logits, torch.float32, "logits", n), _dev(h, torch.uint8, "h", n),
                                 _dev(g, torch.uint8, "g", n), _dev(counts, torch.int64, "counts", 4), _stream(stream)))


def nb_kdop_train_step(b, ind, kind: int, seed: int, step: int, batch: int, alpha: float, beta: float = 1.0,
                       lr: float = 1e-3, loss=None, counts=None, stream=None):
    _check(lib().nb_kdop_train_step(b, ind, int(kind), int(seed), int(step), int(batch), float(alpha), float(beta),
                                    float(lr), _dev(loss, torch.float32, "loss", 1),
                                    _dev(counts, torch.int64, "counts", 4), _stream(stream)))


class KDop:
    """Owns an nb_kdop handle: k slabs in `dim` dimensions."""

    def __init__(self, dim: int, k: int = 4):
        self.dim, self.k = dim, k
        h = C.c_void_p()
        _check(lib().nb_kdop_create(int(dim), int(k), C.byref(h)))
        self.handle = h
        n = C.c_int64()
        _check(lib().nb_kdop_num_params(h, C.byref(n)))
        self.n_params = n.value

    def set_params(self, theta):
        if isinstance(theta, np.ndarray):
            theta = torch.from_numpy(np.ascontiguousarray(theta, dtype=np.float32)).cuda()
        _check(lib().nb_kdop_set_params(self.handle, _dev(theta, torch.float32, "theta", self.n_params),
                                        self.n_params, None))

    def params(self) -> torch.Tensor:
        t = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(lib().nb_kdop_get_params(self.handle, _dev(t, torch.float32, "theta"), self.n_params, None))
        return t

    def forward(self, kind, q: torch.Tensor, eps: float = EPS_OUT):
        n = q.shape[0]
        z = torch.empty(n, dtype=torch.float32, device=q.device)
        h = torch.empty(n, dtype=torch.uint8, device=q.device)
        nb_kdop_forward(self.handle, KINDS.get(kind, kind), q, eps, logits=z, h=h)
        return z, h

    def counts(self, kind, q: torch.Tensor, g: torch.Tensor, eps: float = EPS_OUT) -> torch.Tensor:
        c = torch.empty(4, dtype=torch.int64, device=q.device)
        nb_kdop_forward(self.handle, KINDS.get(kind, kind), q, eps, g=g, counts=c)
        return c

    def close(self):
        if getattr(self, "handle", None):
            lib().nb_kdop_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ groups

def nb_group_create(in_dim: int, widths, n_hidden: int, precision: int = BF16) -> C.c_void_p:
    w = np.ascontiguousarray(widths, dtype=np.int32)
    h = C.c_void_p()
    _check(lib().nb_group_create(int(w.size), int(in_dim), w.ctypes.data_as(C.c_void_p), int(n_hidden),
                                 int(precision), C.byref(h)))
    return h


def nb_group_destroy(g):
    _check(lib().nb_group_destroy(g))


def nb_group_num_params(g) -> int:
    n = C.c_int64()
    _check(lib().nb_group_num_params(g, C.byref(n)))
    return n.value


def nb_group_param_offsets(g, n_obj: int) -> np.ndarray:
    off = np.zeros(n_obj + 1, dtype=np.int64)
    _check(lib().nb_group_param_offsets(g, off.ctypes.data_as(C.c_void_p)))
    return off


def nb_group_set_params(g, theta: torch.Tensor, stream=None):
    _check(lib().nb_group_set_params(g, _dev(theta, torch.float32, "theta"), theta.numel(), _stream(stream)))


def nb_group_get_params(g, theta: torch.Tensor, stream=None):
    _check(lib().nb_group_get_params(g, _dev(theta, torch.float32, "theta"), theta.numel(), _stream(stream)))


def nb_group_set_voxels(g, grids: torch.Tensor, sizes):
    n = np.ascontiguousarray(sizes, dtype=np.int32)
    if grids.numel() != int((n.astype(np.int64) ** 3).sum()):
        raise ValueError("grids must hold sum(n^3) bytes")
    _check(lib().nb_group_set_voxels(g, _dev(grids, torch.uint8, "grids"), n.ctypes.data_as(C.c_void_p)))


BOX_SCAN, BOX_TABLE = 0, 1


def nb_group_set_box_method(g, method: int):
    _check(lib().nb_group_set_box_method(g, int(method)))


def nb_group_set_active(g, active=None):
    a = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    _check(lib().nb_group_set_active(g, None if a is None else a.ctypes.data_as(C.c_void_p)))


def _qoff(qoff: torch.Tensor, n_obj: int, n: int):
    if qoff.numel() != n_obj + 1:
        raise ValueError("qoff must have n_obj + 1 entries")
    return _dev(qoff, torch.int64, "qoff")


def nb_group_query_exact(g, n_obj: int, kind: int, q: torch.Tensor, qoff: torch.Tensor, out: torch.Tensor,
                         stream=None):
    n = _rows(q)
    _check(lib().nb_group_query_exact(g, int(kind), _dev(q, torch.float32, "q"), _qoff(qoff, n_obj, n), n,
                                      _dev(out, torch.uint8, "g", n), _stream(stream)))


def nb_group_forward(g, n_obj: int, in_dim: int, q: torch.Tensor, qoff: torch.Tensor, eps: float = EPS_OUT,
                     logits=None, h=None, g_exact=None, counts=None, stream=None):
    n = _rows(q, in_dim)
    _check(lib().nb_group_forward(g, _dev(q, torch.float32, "q"), _qoff(qoff, n_obj, n), n, float(eps),
                                  _dev(logits, torch.float32, "logits", n), _dev(h, torch.uint8, "h", n),
                                  _dev(g_exact, torch.uint8, "g", n), _dev(counts, torch.int64, "counts", 4 * n_obj),
                                  _stream(stream)))


def nb_group_num_variants(g) -> int:
    c = C.c_int()
    _check(lib().nb_group_num_variants(g, C.byref(c)))
    return c.value


def nb_group_set_variant(g, variant: int):
    _check(lib().nb_group_set_variant(g, int(variant)))


def nb_group_set_width_variant(g, width: int, variant: int):
    _check(lib().nb_group_set_width_variant(g, int(width), int(variant)))


def nb_group_train_step(g, n_obj: int, kind: int, seed: int, step: int, per_obj: int, alpha: float,
                        beta: float = 1.0, lr: float = 1e-3, loss=None, counts=None, alpha_obj=None, lr_obj=None,
                        stream=None):
    _check(lib().nb_group_train_step(g, int(kind), int(seed), int(step), int(per_obj), float(alpha),
                                     _dev(alpha_obj, torch.float32, "alpha_obj", n_obj), float(beta),
                                     float(lr), _dev(lr_obj, torch.float32, "lr_obj", n_obj),
                                     _dev(loss, torch.float32, "loss", n_obj),
                                     _dev(counts, torch.int64, "counts", 4 * n_obj), _stream(stream)))


class Group:
    """Owns an nb_group handle: n_obj bfloat16 bounds in_dim -> w_o^n_hidden -> 1."""

    def __init__(self, in_dim: int, widths, n_hidden: int):
        self.in_dim, self.widths, self.n_hidden = in_dim, list(widths), n_hidden
        self.n_obj = len(self.widths)
        self.handle = nb_group_create(in_dim, self.widths, n_hidden)
        self.n_params = nb_group_num_params(self.handle)
        self.offsets = nb_group_param_offsets(self.handle, self.n_obj)

    def set_params(self, theta):
        if isinstance(theta, np.ndarray):
            theta = torch.from_numpy(np.ascontiguousarray(theta, dtype=np.float32)).cuda()
        nb_group_set_params(self.handle, theta)

    def params(self) -> torch.Tensor:
        t = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        nb_group_get_params(self.handle, t)
        return t

    def set_voxels(self, grids: torch.Tensor, sizes):
        nb_group_set_voxels(self.handle, grids, sizes)

    def forward(self, q: torch.Tensor, qoff: torch.Tensor, eps: float = EPS_OUT):
        n = q.shape[0]
        z = torch.empty(n, dtype=torch.float32, device=q.device)
        h = torch.empty(n, dtype=torch.uint8, device=q.device)
        nb_group_forward(self.handle, self.n_obj, self.in_dim, q, qoff, eps, logits=z, h=h)
        return z, h

    def counts(self, q: torch.Tensor, qoff: torch.Tensor, g: torch.Tensor, eps: float = EPS_OUT) -> torch.Tensor:
        """Per-object (TP, FP, TN, FN) of the bound's decisions against g: int64[n_obj, 4]."""
        c = torch.empty(4 * self.n_obj, dtype=torch.int64, device=q.device)
        nb_group_forward(self.handle, self.n_obj, self.in_dim, q, qoff, eps, g_exact=g, counts=c)
        return c.view(self.n_obj, 4)

    def query(self, kind, q: torch.Tensor, qoff: torch.Tensor) -> torch.Tensor:
        out = torch.zeros(q.shape[0], dtype=torch.uint8, device=q.device)
        nb_group_query_exact(self.handle, self.n_obj, KINDS.get(kind, kind), q, qoff, out)
        return out

    def close(self):
        if self.handle:
            nb_group_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------- training health

def nb_bound_sync(b, stream=None):
    """Raise NBError (NB_ERR_NONFINITE) if a training call since the last
    check met a non-finite loss or gradient; synchronises the stream."""
    _check(lib().nb_bound_sync(b, _stream(stream)))


def nb_group_sync(g, stream=None):
    _check(lib().nb_group_sync(g, _stream(stream)))


def nb_kdop_sync(b, stream=None):
    _check(lib().nb_kdop_sync(b, _stream(stream)))


# ------------------------------------------------------------ hierarchies

def nb_hier_create(g, child_begin, child_end) -> C.c_void_p:
    b = np.ascontiguousarray(child_begin, dtype=np.int32)
    e = np.ascontiguousarray(child_end, dtype=np.int32)
    h = C.c_void_p()
    _check(lib().nb_hier_create(g, b.ctypes.data_as(C.c_void_p), e.ctypes.data_as(C.c_void_p), C.byref(h)))
    return h


def nb_hier_destroy(h):
    _check(lib().nb_hier_destroy(h))


def nb_hier_num_leaves(h) -> int:
    n = C.c_int32()
    _check(lib().nb_hier_num_leaves(h, C.byref(n)))
    return n.value


def nb_hier_leaf_nodes(h, n_leaves: int) -> np.ndarray:
    out = np.zeros(n_leaves, dtype=np.int32)
    _check(lib().nb_hier_leaf_nodes(h, out.ctypes.data_as(C.c_void_p)))
    return out


def nb_hier_depth(h) -> int:
    d = C.c_int32()
    _check(lib().nb_hier_depth(h, C.byref(d)))
    return d.value


def nb_hier_level_pairs(h, depth: int) -> np.ndarray:
    out = np.zeros(depth, dtype=np.int64)
    _check(lib().nb_hier_level_pairs(h, out.ctypes.data_as(C.c_void_p)))
    return out


def nb_hier_query(h, in_dim: int, q: torch.Tensor, qidx_out: torch.Tensor | None, leaf_off: torch.Tensor,
                  eps: float = EPS_OUT, stream=None, check: bool = True) -> int:
    """Number of (row, leaf) pairs.  With check=False a too-small qidx_out
    (or None) does not raise: compare the returned count with its size."""
    n = _rows(q, in_dim)
    cap = 0 if qidx_out is None else qidx_out.numel()
    npairs = C.c_int64(-1)
    st = lib().nb_hier_query(h, _dev(q, torch.float32, "q"), n, float(eps), _dev(qidx_out, torch.int32, "qidx_out"),
                             cap, _dev(leaf_off, torch.int64, "leaf_off"), C.byref(npairs), _stream(stream))
    if st != 0 and (check or npairs.value <= cap):
        _check(st)
    return npairs.value


class Hierarchy:
    """A user-supplied tree over the objects of a Group (node i = object i,
    breadth-first order, node 0 the root, children of p = child_begin[p] ..
    child_end[p]-1)."""

    def __init__(self, group: Group, child_begin, child_end):
        if len(child_begin) != group.n_obj or len(child_end) != group.n_obj:
            raise ValueError(f"the tree needs one child range per object of the group ({group.n_obj})")
        self.group = group
        self.handle = nb_hier_create(group.handle, child_begin, child_end)
        self.n_leaves = nb_hier_num_leaves(self.handle)
        self.leaf_nodes = nb_hier_leaf_nodes(self.handle, self.n_leaves)
        self.depth = nb_hier_depth(self.handle)
        self._out = None

    def level_pairs(self) -> np.ndarray:
        """(row, node) pairs per level of the last query."""
        return nb_hier_level_pairs(self.handle, self.depth)

    def query(self, q: torch.Tensor, eps: float = EPS_OUT):
        """(leaf_off int64[n_leaves + 1], qidx int32[pairs]) on the device;
        the output buffer grows when the pairs do not fit."""
        leaf_off = torch.empty(self.n_leaves + 1, dtype=torch.int64, device=q.device)
        if self._out is None:
            self._out = torch.empty(max(q.shape[0], 1 << 16), dtype=torch.int32, device=q.device)
        n = nb_hier_query(self.handle, self.group.in_dim, q, self._out, leaf_off, eps, check=False)
        if n > self._out.numel():
            self._out = torch.empty(n + n // 4 + 1, dtype=torch.int32, device=q.device)
            n = nb_hier_query(self.handle, self.group.in_dim, q, self._out, leaf_off, eps)
        return leaf_off, self._out[:n]

    def close(self):
        if self.handle:
            nb_hier_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ conveniences

class Indicator:
    """Owns an nb_indicator handle."""

    def __init__(self, handle, dim: int, grid: torch.Tensor | None = None, n: int = 0):
        self.handle, self.dim, self.grid, self.n = handle, dim, grid, n

    @classmethod
    def discs2d(cls, discs):
        return cls(nb_indicator_discs2d(discs), 2)

    @classmethod
    def voxels(cls, grid: torch.Tensor, n: int):
        return cls(nb_indicator_voxels(grid, n), 3, grid, n)

    @classmethod
    def metaball_voxels(cls, centres, radii, n: int, iso: float = 1.0, device="cuda"):
        grid = torch.empty(n ** 3, dtype=torch.uint8, device=device)
        nb_voxelize_metaballs(centres, radii, iso, n, grid)
        return cls.voxels(grid, n)

    @classmethod
    def metaballs4d(cls, a, b, radii, iso: float = 1.0):
        return cls(nb_indicator_metaballs4d(a, b, radii, iso), 4)

    def query(self, kind, q: torch.Tensor, g: torch.Tensor | None = None) -> torch.Tensor:
        kind = KINDS.get(kind, kind)
        if g is None:
            g = torch.empty(q.shape[0], dtype=torch.uint8, device=q.device)
        nb_query_exact(self.handle, kind, q, g)
        return g

    def close(self):
        if self.handle:
            nb_indicator_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Bound:
    """Owns an nb_bound handle: in_dim -> width^n_hidden -> 1 logit."""

    def __init__(self, in_dim: int, n_hidden: int, width: int, precision: int = F32):
        self.in_dim, self.n_hidden, self.width, self.precision = in_dim, n_hidden, width, precision
        self.handle = nb_bound_create(in_dim, n_hidden, width, precision)
        self.n_params = nb_bound_num_params(self.handle)

    def set_params(self, theta):
        if isinstance(theta, np.ndarray):
            theta = torch.from_numpy(np.ascontiguousarray(theta, dtype=np.float32)).cuda()
        nb_bound_set_params(self.handle, theta)

    def params(self) -> torch.Tensor:
        t = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        nb_bound_get_params(self.handle, t)
        return t

    def forward(self, q: torch.Tensor, eps: float = EPS_OUT, want_logits=True, want_h=True):
        n = q.shape[0]
        z = torch.empty(n, dtype=torch.float32, device=q.device) if want_logits else None
        h = torch.empty(n, dtype=torch.uint8, device=q.device) if want_h else None
        nb_bound_forward(self.handle, q, eps, logits=z, h=h)
        return z, h

    def counts(self, q: torch.Tensor, g: torch.Tensor, eps: float = EPS_OUT) -> torch.Tensor:
        c = torch.zeros(4, dtype=torch.int64, device=q.device)
        nb_bound_forward(self.handle, q, eps, g=g, counts=c)
        return c

    def close(self):
        if self.handle:
            nb_bound_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
