"""CPU checks of the C ABI: libsfmm.so loads, exports every entry point that
include/sfmm.h declares, and rejects bad arguments without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "sfmm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfmm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2602_05804_amd as P

    return P.lib()


def test_every_declared_symbol_is_exported(L):
    import paper_2602_05804_amd as P

    names = declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(P.EXPORTED)


def test_strerror(L):
    assert L.sfmm_strerror(0) == b"ok"
    assert L.sfmm_strerror(-1) == b"invalid argument"
    assert L.sfmm_strerror(-5).startswith(b"non-finite")
    assert L.sfmm_strerror(7) == b"unknown status"


def test_null_arguments(L):
    import paper_2602_05804_amd as P

    assert L.sfmm_config_default(None) == -1
    c = P.Config()
    assert L.sfmm_config_default(C.byref(c)) == 0
    assert (c.G, c.leaf_size, c.r_kern, c.include_self_potential, c.check_inputs,
            c.walk_mode, c.fp64_top_depth, c.far_mode, c.far_kernel,
            c.near_kernel) == (1.0, 10, 2.0, 1, 1, 0, 8, 1, 0, 0)
    assert L.sfmm_create(None, 0, None, None) == -1
    assert L.sfmm_solve(None, 10, None, None, None, 0.5, 3, 0, None, None) == -1
    assert L.sfmm_build(None, 10, None, None, None, 3) == -1
    assert L.sfmm_get_stats(None, None) == -1
    assert L.sfmm_destroy(None) == 0
    assert L.sfmm_last_error(None) == b""


def test_bad_config_rejected(L):
    import paper_2602_05804_amd as P

    ctx = C.c_void_p(0)
    bad = P.Config(1.0, 0, 2.0, 1, 1, 0, 8, 0)  # leaf_size 0
    assert L.sfmm_create(C.byref(ctx), 0, None, C.byref(bad)) == -1
    bad = P.Config(1.0, 10, -1.0, 1, 1, 0, 8, 0)  # negative kernel radius
    assert L.sfmm_create(C.byref(ctx), 0, None, C.byref(bad)) == -1
    bad = P.Config(1.0, 10, 2.0, 1, 1, 7, 8, 0)  # unknown walk mode
    assert L.sfmm_create(C.byref(ctx), 0, None, C.byref(bad)) == -1
    bad = P.Config(1.0, 10, 2.0, 1, 1, 0, 8, 5)  # unknown far mode
    assert L.sfmm_create(C.byref(ctx), 0, None, C.byref(bad)) == -1
    bad = P.Config(1.0, 10, 2.0, 1, 1, 0, 8, 1, 9, 0)  # unknown far kernel shape
    assert L.sfmm_create(C.byref(ctx), 0, None, C.byref(bad)) == -1
    bad = P.Config(1.0, 10, 2.0, 1, 1, 0, 8, 1, 1, 0)  # far shapes other than 0 are gone
    assert L.sfmm_create(C.byref(ctx), 0, None, C.byref(bad)) == -1
    for shape in (2, 3, 4, 5, 8, 9, 10, 11, 12, 14, -1):  # P2P shapes that do not exist
        bad = P.Config(1.0, 10, 2.0, 1, 1, 0, 8, 1, 0, shape)
        assert L.sfmm_create(C.byref(ctx), 0, None, C.byref(bad)) == -1, shape


def test_no_device_is_an_error_not_a_fallback(L):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = C.c_void_p(0)
    assert L.sfmm_create(C.byref(ctx), 0, None, None) == -3
    import paper_2602_05804_amd as P

    with pytest.raises(P.SfmmError):
        P.Solver()
