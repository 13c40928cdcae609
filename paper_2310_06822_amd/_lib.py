"""ctypes loader for libnbound.so: signatures of every nbound.h entry point.

Loading fails loudly if the library has not been built: there is no
fallback implementation anywhere in the package.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbound.so")

vp, i32, i64, u64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_float
PP = C.POINTER(C.c_void_p)

# name -> (restype, argtypes); mirrors include/nbound.h
SIGNATURES = {
    "nb_last_error": (C.c_char_p, []),
    "nb_version": (i32, [C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "nb_device_count": (i32, [C.POINTER(C.c_int)]),
    "nb_indicator_discs2d": (i32, [vp, C.c_int, PP]),
    "nb_indicator_voxels": (i32, [vp, C.c_int, PP]),
    "nb_indicator_metaballs4d": (i32, [vp, vp, vp, C.c_int, f32, PP]),
    "nb_indicator_dim": (i32, [vp, C.POINTER(C.c_int)]),
    "nb_indicator_destroy": (i32, [vp]),
    "nb_voxelize_metaballs": (i32, [vp, vp, C.c_int, f32, C.c_int, vp, vp]),
    "nb_query_exact": (i32, [vp, C.c_int, vp, i64, vp, vp]),
    "nb_sample_queries": (i32, [C.c_int, C.c_int, u64, u64, i64, vp, vp]),
    "nb_bound_create": (i32, [C.c_int, C.c_int, C.c_int, C.c_int, PP]),
    "nb_bound_destroy": (i32, [vp]),
    "nb_bound_num_params": (i32, [vp, C.POINTER(i64)]),
    "nb_bound_shape": (i32, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "nb_bound_num_variants": (i32, [vp, C.POINTER(C.c_int)]),
    "nb_bound_set_variant": (i32, [vp, C.c_int]),
    "nb_bound_set_recompute": (i32, [vp, C.c_int]),
    "nb_bound_set_train_kernel": (i32, [vp, C.c_int, vp]),
    "nb_bound_set_activation": (i32, [vp, C.c_int]),
    "nb_bound_set_params": (i32, [vp, vp, i64, vp]),
    "nb_bound_save": (i32, [vp, vp, C.POINTER(C.c_size_t), vp]),
    "nb_bound_load": (i32, [vp, vp, C.c_size_t, vp]),
    "nb_bound_get_params": (i32, [vp, vp, i64, vp]),
    "nb_bound_get_state": (i32, [vp, vp, vp, i64, C.POINTER(i64), vp]),
    "nb_bound_set_state": (i32, [vp, vp, vp, i64, i64, vp]),
    "nb_bound_forward": (i32, [vp, vp, i64, f32, vp, vp, vp, vp, vp]),
    "nb_bound_loss_grad": (i32, [vp, vp, vp, i64, f32, f32, vp, vp, vp, vp]),
    "nb_bound_adam_step": (i32, [vp, vp, f32, f32, f32, f32, f32, f32, vp]),
    "nb_bound_train_step": (i32, [vp, vp, C.c_int, u64, u64, i64, f32, f32, f32, f32, f32, vp, vp, vp]),
    "nb_cascade": (i32, [vp, vp, C.c_int, vp, i64, f32, vp, vp, vp]),
    "nb_cascade_noalloc": (i32, [vp, vp, C.c_int, vp, i64, f32, vp, vp, vp]),
    "nb_early_out": (i32, [vp, vp, vp, i64, f32, vp, vp, vp]),
    "nb_kdop_create": (i32, [C.c_int, C.c_int, PP]),
    "nb_kdop_destroy": (i32, [vp]),
    "nb_kdop_num_params": (i32, [vp, C.POINTER(i64)]),
    "nb_kdop_set_params": (i32, [vp, vp, i64, vp]),
    "nb_kdop_get_params": (i32, [vp, vp, i64, vp]),
    "nb_kdop_forward": (i32, [vp, C.c_int, vp, i64, f32, vp, vp, vp, vp, vp]),
    "nb_kdop_train_step": (i32, [vp, vp, C.c_int, u64, u64, i64, f32, f32, f32, vp, vp, vp]),
    "nb_group_create": (i32, [C.c_int, C.c_int, vp, C.c_int, C.c_int, PP]),
    "nb_group_destroy": (i32, [vp]),
    "nb_group_num_params": (i32, [vp, C.POINTER(i64)]),
    "nb_group_param_offsets": (i32, [vp, vp]),
    "nb_group_set_params": (i32, [vp, vp, i64, vp]),
    "nb_group_get_params": (i32, [vp, vp, i64, vp]),
    "nb_group_set_voxels": (i32, [vp, vp, vp]),
    "nb_group_set_box_method": (i32, [vp, C.c_int]),
    "nb_group_set_active": (i32, [vp, vp]),
    "nb_group_query_exact": (i32, [vp, C.c_int, vp, vp, i64, vp, vp]),
    "nb_group_forward": (i32, [vp, vp, vp, i64, f32, vp, vp, vp, vp, vp]),
    "nb_group_num_variants": (i32, [vp, C.POINTER(C.c_int)]),
    "nb_group_set_variant": (i32, [vp, C.c_int]),
    "nb_group_set_width_variant": (i32, [vp, C.c_int, C.c_int]),
    "nb_group_train_step": (i32, [vp, C.c_int, u64, u64, i64, f32, vp, f32, f32, vp, vp, vp, vp]),
    "nb_bound_sync": (i32, [vp, vp]),
    "nb_group_sync": (i32, [vp, vp]),
    "nb_kdop_sync": (i32, [vp, vp]),
    "nb_hier_create": (i32, [vp, vp, vp, PP]),
    "nb_hier_destroy": (i32, [vp]),
    "nb_hier_num_leaves": (i32, [vp, C.POINTER(i32)]),
    "nb_hier_leaf_nodes": (i32, [vp, vp]),
    "nb_hier_depth": (i32, [vp, C.POINTER(i32)]),
    "nb_hier_level_pairs": (i32, [vp, vp]),
    "nb_hier_query": (i32, [vp, vp, i64, f32, vp, i64, vp, C.POINTER(i64), vp]),
}

_lib = None


def load() -> C.CDLL:
    """Load libnbound.so once; raise if it is missing (build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2310_06822_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
