"""Host-side validation of vp_plan_create for two-level problems: bad
boxes and unsupported requests are rejected before any HIP call, so these
run on a machine without a GPU."""
import ctypes
import math

import numpy as np
import pytest

import vp_inputs as I


@pytest.fixture(scope="module")
def V():
    from paper_1204_3853_amd import vp
    import os
    if not os.path.exists(vp.LIB_PATH):
        from paper_1204_3853_amd import build
        build.build()
    return vp


def make_problem(V, ncx=32, ncv=48, R=4, dtype=0, ndim=1):
    pb = V.vp_problem()
    pb.ndim = ndim
    pb.dtype = dtype
    pb.n_levels = 2
    pb.cells[0], pb.cells[1] = ncx, ncv
    pb.ratio[0][0], pb.ratio[0][1] = R, R
    pb.x_len[0] = 4 * math.pi
    pb.v_lo[0], pb.v_hi[0] = -8.0, 8.0
    pb.qm = -1.0
    vc = I.cell_average_1d(I.maxwellian, -8, 8, ncv, first=-2, count=ncv + 4)
    vf = I.cell_average_1d(I.maxwellian, -8, 8, ncv * R, first=-2, count=ncv * R + 4)
    keep = [(ctypes.c_double * len(vc))(*vc), (ctypes.c_double * len(vf))(*vf)]
    pb.veq[0][0] = ctypes.cast(keep[0], ctypes.POINTER(ctypes.c_double))
    pb.veq[1][0] = ctypes.cast(keep[1], ctypes.POINTER(ctypes.c_double))
    return pb, keep


def create(V, pb, boxes):
    arr = (V.vp_box * max(len(boxes), 1))()
    for q, (lo, hi) in enumerate(boxes):
        arr[q].level = 1
        arr[q].lo[0], arr[q].lo[1] = lo
        arr[q].hi[0], arr[q].hi[1] = hi
    h = ctypes.c_void_p()
    L = V.lib()
    code = L.vp_plan_create(ctypes.byref(pb), arr, len(boxes), ctypes.byref(h))
    msg = L.vp_last_error().decode()
    if code == 0:
        L.vp_plan_destroy(h)
    return code, msg


@pytest.mark.parametrize("boxes,code,word", [
    ([((16, 40), (38, 63))], 1, "aligned"),                             # hi + 1 not a multiple of R
    ([((18, 40), (39, 63))], 1, "aligned"),                             # lo not aligned
    ([((120, 40), (131, 63))], 1, "outside"),                           # past the x extent
    ([((16, 40), (39, 63)), ((32, 48), (47, 71))], 1, "overlap"),       # overlapping patches
])
def test_bad_boxes(V, boxes, code, word):
    pb, keep = make_problem(V)
    got, msg = create(V, pb, boxes)
    assert got == code, msg
    assert word in msg


@pytest.mark.parametrize("boxes", [
    [((16, 40), (39, 63)), ((40, 40), (55, 63))],                       # touching in x
    [((16, 40), (39, 63)), ((24, 64), (31, 79))],                       # touching in v
    [((0, 40), (15, 63)), ((112, 40), (127, 63))],                      # touching across x = 0
    [((0, 40), (127, 63))],                                             # the whole x range
])
def test_touching_boxes_pass_validation(V, boxes):
    """Touching patches are valid: creation gets past the box checks (it
    then succeeds on a GPU, or stops at the first HIP call without one)."""
    pb, keep = make_problem(V)
    got, msg = create(V, pb, boxes)
    assert got in (0, 5), msg


def test_unsupported_requests(V):
    pb, keep = make_problem(V, dtype=1)
    assert create(V, pb, [((16, 40), (39, 63))])[0] == 4          # FP32 two-level
    pb, keep = make_problem(V, R=3)
    assert create(V, pb, [((15, 39), (38, 62))])[0] == 4          # ratio 3
    pb, keep = make_problem(V)
    pb.veq[1][0] = None
    assert create(V, pb, [((16, 40), (39, 63))])[0] == 1          # no level-1 equilibrium
    pb, keep = make_problem(V)
    arr = (V.vp_box * 1)()
    arr[0].level = 0
    h = ctypes.c_void_p()
    assert V.lib().vp_plan_create(ctypes.byref(pb), arr, 1, ctypes.byref(h)) == 1   # level-0 box


def test_single_level_rejects_boxes(V):
    pb, keep = make_problem(V)
    pb.n_levels = 1
    assert create(V, pb, [((16, 40), (39, 63))])[0] == 1


def make_problem_4d(V, nx=8, ny=8, nvx=16, nvy=16, dtype=0):
    pb = V.vp_problem()
    pb.ndim, pb.dtype, pb.n_levels = 2, dtype, 1
    for d, c in enumerate((nx, ny, nvx, nvy)):
        pb.cells[d] = c
    for d in range(2):
        pb.x_len[d] = 4 * math.pi
        pb.v_lo[d], pb.v_hi[d] = -6.0, 6.0
    pb.qm = -1.0
    gx = I.cell_average_1d(I.maxwellian, -6, 6, nvx, first=-2, count=nvx + 4)
    gy = I.cell_average_1d(I.maxwellian, -6, 6, nvy, first=-2, count=nvy + 4)
    keep = [(ctypes.c_double * len(gx))(*gx), (ctypes.c_double * len(gy))(*gy)]
    pb.veq[0][0] = ctypes.cast(keep[0], ctypes.POINTER(ctypes.c_double))
    pb.veq[0][1] = ctypes.cast(keep[1], ctypes.POINTER(ctypes.c_double))
    return pb, keep


@pytest.mark.parametrize("kw,code", [(dict(nx=257), 4), (dict(ny=300), 4), (dict(nvx=1025), 4), (dict(dtype=1), 4),
                                     (dict(nx=256, ny=256, nvx=1024, nvy=32), 4)])
def test_4d_limits(V, kw, code):
    pb, keep = make_problem_4d(V, **kw)
    assert create(V, pb, [])[0] == code


def test_4d_needs_vy_equilibrium(V):
    pb, keep = make_problem_4d(V)
    pb.veq[0][1] = None
    assert create(V, pb, [])[0] == 1
