"""The C-ABI library loads on a machine without a GPU and exports every
function that include/vp.h declares (no compute calls are made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:vp_status|size_t|int64_t|const char\*)\s+(vp_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libvp():
    from paper_1204_3853_amd import vp
    path = vp.LIB_PATH
    if not os.path.exists(path):
        from paper_1204_3853_amd import build
        build.build()
    return ctypes.CDLL(path)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ["vp_rhs", "vp_reduce_moment", "vp_inject_field", "vp_poisson_periodic",
                     "vp_rk4_step", "vp_adjoint_step", "vp_plan_create", "vp_plan_destroy",
                     "vp_workspace_bytes", "vp_last_error"]:
        assert required in names


def test_every_declared_symbol_is_exported(libvp):
    missing = [n for n in declared_functions() if not hasattr(libvp, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_1204_3853_amd import vp
    assert set(declared_functions()) <= set(vp.SIGNATURES)


def test_null_plan_is_rejected_without_gpu(libvp):
    libvp.vp_rhs.restype = ctypes.c_int
    libvp.vp_rhs.argtypes = [ctypes.c_void_p] * 5
    libvp.vp_last_error.restype = ctypes.c_char_p
    assert libvp.vp_rhs(None, None, None, None, None) == 1   # VP_EINVAL
    assert b"NULL" in libvp.vp_last_error()
