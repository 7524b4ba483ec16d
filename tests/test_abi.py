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
    names = re.findall(r"^\s*(?:vp_status|size_t|int64_t|int32_t|const char\*|const vp_plan\*)\s+(vp_\w+)\s*\(", src, flags=re.M)
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
    libvp.vp_amr_subcycle_step.restype = ctypes.c_int
    libvp.vp_amr_subcycle_step.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                           ctypes.c_void_p, ctypes.c_void_p]
    assert libvp.vp_amr_subcycle_step(None, None, None, 0.1, None, None) == 1


def test_amr_run_parameters_rejected_without_gpu(libvp):
    """vp_amr_run_create validates its parameters on the host before any HIP call."""
    from paper_1204_3853_amd import vp
    L = vp.lib()
    pb = vp.vp_problem()
    pb.ndim, pb.n_levels = 1, 2
    out = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    good = dict(tol=0.01, regrid_interval=2, efficiency=0.7, min_width=2, buffer=1, cfl=0.5, dt_growth=1.1,
                dt_initial=0.01)
    for bad in (dict(regrid_interval=0), dict(efficiency=0.0), dict(efficiency=1.5), dict(min_width=0),
                dict(buffer=-1), dict(cfl=0.0), dict(dt_growth=0.5), dict(dt_initial=0.0), dict(tol=-1.0),
                dict(tol=float("nan"))):
        prm = vp.vp_amr_params(**dict(good, **bad))
        assert L.vp_amr_run_create(ctypes.byref(pb), None, 0, dummy, ctypes.byref(prm), ctypes.byref(out), None) == 1
        assert b"bad parameters" in L.vp_last_error()
    prm = vp.vp_amr_params(**good)
    prm.max_size[1][0] = -1
    assert L.vp_amr_run_create(ctypes.byref(pb), None, 0, dummy, ctypes.byref(prm), ctypes.byref(out), None) == 1
    assert b"patch size" in L.vp_last_error()
    pb.n_levels = 1
    prm = vp.vp_amr_params(**good)
    assert L.vp_amr_run_create(ctypes.byref(pb), None, 0, dummy, ctypes.byref(prm), ctypes.byref(out), None) == 1
    assert b"two or more levels" in L.vp_last_error()
    assert L.vp_amr_run_create(None, None, 0, dummy, ctypes.byref(prm), ctypes.byref(out), None) == 1
    assert L.vp_amr_run_destroy(None) == 0


def test_species_group_arguments_rejected_without_gpu(libvp):
    """vp_species_group_create validates its arguments on the host."""
    from paper_1204_3853_amd import vp
    L = vp.lib()
    out = ctypes.c_void_p()
    ch = (ctypes.c_double * 2)(-1.0, 1.0)
    nulls = (ctypes.c_void_p * 2)(None, None)
    assert L.vp_species_group_create(None, ch, 2, 0.0, ctypes.byref(out)) == 1
    assert L.vp_species_group_create(nulls, ch, 0, 0.0, ctypes.byref(out)) == 1
    assert b"species" in L.vp_last_error()
    assert L.vp_species_group_create(nulls, ch, 5, 0.0, ctypes.byref(out)) == 1
    assert L.vp_species_group_create(nulls, ch, 2, float("inf"), ctypes.byref(out)) == 1
    assert b"finite" in L.vp_last_error()
    assert L.vp_species_group_create(nulls, ch, 2, 0.0, ctypes.byref(out)) == 1
    assert b"NULL plan" in L.vp_last_error()
    assert L.vp_species_group_destroy(None) == 0
    assert L.vp_species_workspace_bytes(None) == 0
    assert L.vp_species_rk4_step(None, None, None, ctypes.c_double(0.1), None, None, None) == 1
    assert L.vp_species_field(None, None, None, None, None, None) == 1
    run_out = ctypes.c_void_p()
    assert L.vp_amr_run_create_species(0, None, None, None, None, None, ctypes.c_double(0.0), None,
                                       ctypes.byref(run_out), None) == 1
    assert L.vp_amr_run_species_count(None) == 0
