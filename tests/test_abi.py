"""The C ABI on the CPU: the library loads, exports every function the header
declares, and rejects bad arguments with the documented status codes.  No
kernel is launched."""

import ctypes as C
import os
import re

import pytest

import paper_2310_06822_amd as nb
from paper_2310_06822_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "nbound.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nb_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_signatures():
    assert _declared() == sorted(_lib.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_version_and_device_count():
    assert nb.nb_version() == (0, 1)
    assert nb.nb_device_count() >= 0


def test_invalid_arguments():
    lib = _lib.load()
    h = C.c_void_p()
    assert lib.nb_bound_create(3, 3, 64, 0, None) == 1
    assert lib.nb_bound_create(0, 3, 64, 0, C.byref(h)) == 1
    assert lib.nb_bound_create(3, 0, 64, 0, C.byref(h)) == 1
    assert lib.nb_bound_create(3, 3, 40, 0, C.byref(h)) == 1
    assert lib.nb_bound_create(3, 3, 64, 7, C.byref(h)) == 1
    assert lib.nb_indicator_discs2d(None, 8, C.byref(h)) == 1
    assert lib.nb_indicator_voxels(None, 8, C.byref(h)) == 1
    assert lib.nb_query_exact(None, 0, None, 10, None, None) == 1
    assert lib.nb_sample_queries(9, 3, 1, 0, 10, C.c_void_p(16), None) == 1
    assert lib.nb_sample_queries(0, 5, 1, 0, 10, C.c_void_p(16), None) == 1
    assert lib.nb_sample_queries(0, 3, 1, 0, 0, C.c_void_p(16), None) == 1
    assert lib.nb_last_error().decode()
    with pytest.raises(nb.NBError) as e:
        nb._check(lib.nb_bound_create(3, 3, 40, 0, C.byref(h)))
    assert e.value.status == 1


def test_unsupported_shape_reported():
    lib = _lib.load()
    h = C.c_void_p()
    # shapes the library has no kernel for
    assert lib.nb_bound_create(3, 3, 48, 0, C.byref(h)) == 6
    assert lib.nb_bound_create(3, 5, 64, 0, C.byref(h)) == 6
    assert lib.nb_bound_create(3, 6, 128, 1, C.byref(h)) == 6
    assert lib.nb_bound_create(3, 1, 256, 1, C.byref(h)) == 6
    assert lib.nb_bound_create(3, 9, 64, 0, C.byref(h)) == 1


@pytest.mark.skipif(nb.nb_device_count() > 0, reason="a GPU is visible")
def test_no_device_status():
    lib = _lib.load()
    h = C.c_void_p()
    assert lib.nb_bound_create(3, 3, 64, 0, C.byref(h)) == 2
    import numpy as np
    d = np.zeros((8, 3), np.float32)
    assert lib.nb_indicator_discs2d(d.ctypes.data_as(C.c_void_p), 8, C.byref(h)) == 2


def test_group_arguments():
    import numpy as np
    lib = _lib.load()
    h = C.c_void_p()
    w = np.array([32, 64, 128], np.int32)
    wp = w.ctypes.data_as(C.c_void_p)
    assert lib.nb_group_create(3, 6, wp, 3, 1, None) == 1
    assert lib.nb_group_create(0, 6, wp, 3, 1, C.byref(h)) == 1
    assert lib.nb_group_create(3, 6, wp, 1, 1, C.byref(h)) == 1    # depth outside 2..4
    assert lib.nb_group_create(3, 6, wp, 3, 0, C.byref(h)) == 1    # float32 groups: none
    bad = np.array([32, 48, 128], np.int32)
    assert lib.nb_group_create(3, 6, bad.ctypes.data_as(C.c_void_p), 3, 1, C.byref(h)) == 1
    assert lib.nb_group_destroy(None) == 0
    assert lib.nb_group_forward(None, None, None, 10, 1e-5, None, None, None, None, None) == 1
    assert lib.nb_group_train_step(None, 2, 1, 0, 64, 1.0, None, 1.0, 1e-3, None, None, None, None) == 1
    assert lib.nb_group_set_variant(None, 0) == 1
    assert lib.nb_group_set_width_variant(None, 32, 0) == 1
    if nb.nb_device_count() == 0:
        assert lib.nb_group_create(3, 6, wp, 3, 1, C.byref(h)) == 2


def test_kdop_arguments():
    lib = _lib.load()
    h = C.c_void_p()
    assert lib.nb_kdop_create(3, 4, None) == 1
    assert lib.nb_kdop_create(1, 4, C.byref(h)) == 1
    assert lib.nb_kdop_create(3, 9, C.byref(h)) == 1
    assert lib.nb_kdop_destroy(None) == 0
    assert lib.nb_kdop_forward(None, 0, None, 10, 1e-5, None, None, None, None, None) == 1
    if nb.nb_device_count() == 0:
        assert lib.nb_kdop_create(3, 4, C.byref(h)) == 2
