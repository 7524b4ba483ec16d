"""GPU parity of the two-level path with limited face averages (section 2,
eq. limitedFace on both levels; the coarse fluxes on coarse-fine faces
limited too) against the limited two-level oracle: the right-hand side,
synchronous steps on every layout of the centred tests, every tile shape,
a subcycled step, and one step of the 512 x 512 ratio-4 hierarchy with 40
seeded patches.  Tolerance 1e-12 of max|f| per step."""
import math

import numpy as np
import pytest

import vp_inputs as I
from test_gpu_amr import LAYOUTS, Case, cmp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vp():
    from paper_1204_3853_amd import vp as V
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return V


def limited_case(vp, oracle, L, **kw):
    c = Case(vp, oracle, L["boxes"], L["ncx"], L["ncv"], L["R"], **kw)
    c.plan.set_face_scheme(vp.FACE_LIMITED)
    c.o.set_limited()
    return c


@pytest.fixture(scope="module", params=list(LAYOUTS))
def case(request, vp, oracle):
    print(f"layout {request.param}", flush=True)
    return limited_case(vp, oracle, LAYOUTS[request.param])


def test_rhs(vp, case):
    a_o, _ = case.o.constraints(case.f0)
    k = vp.rhs(case.plan, case.gpu(case.f0), case.gpu(a_o))
    cmp(k, case.o.rhs(case.f0, a_o), 1e-12, "rhs")


def test_steps(vp, case):
    f = case.gpu(case.f0)
    a = vp.field_of(case.plan, f)
    want = case.f0
    for s in range(3):
        vp.rk4_step(case.plan, f, a, case.dt)
        want = case.o.step(want, case.dt)
        cmp(f, want, 1e-12 * (s + 1), f"step {s + 1}")
    assert np.abs(f.cpu().numpy() - case.f0).max() > 1e-9


def test_every_tile_shape(vp, case):
    """Every valid tile shape, in both launch structures, gives the oracle's step."""
    want = case.o.step(case.f0, case.dt)
    shapes = case.plan.tile_shapes()
    tried = 0
    for q, shp in enumerate(shapes):
        try:
            case.plan.set_tile_shape(q)
        except vp.VPError:
            assert shp[1] == 2       # two cells per thread need even widths
            continue
        for mode in (vp.LAUNCH_PERSISTENT, vp.LAUNCH_PER_PATCH):
            case.plan.set_launch_mode(mode)
            f = case.gpu(case.f0)
            a = vp.field_of(case.plan, f)
            vp.rk4_step(case.plan, f, a, case.dt)
            cmp(f, want, 1e-12, f"shape {shp} mode {mode}")
        tried += 1
    case.plan.set_launch_mode(vp.LAUNCH_PERSISTENT)
    assert tried >= 8


def test_subcycled_step(vp, oracle):
    c = limited_case(vp, oracle, LAYOUTS["small"])
    f = c.gpu(c.f0)
    a = vp.field_of(c.plan, f)
    vp.amr_subcycle_step(c.plan, f, a, 2 * c.dt)
    cmp(f, c.o.subcycle_step(c.f0, 2 * c.dt), 1e-12, "subcycled step")


def test_full_config_one_step(vp, oracle):
    print("layout 512 x 512, 40 patches", flush=True)
    c = limited_case(vp, oracle, dict(boxes=I.amr_boxes(0), ncx=512, ncv=512, R=4), eps=0.01, k=0.5, noise=0.0)
    f = c.gpu(c.f0)
    a = vp.field_of(c.plan, f)
    vp.rk4_step(c.plan, f, a, c.dt)
    cmp(f, c.o.step(c.f0, c.dt), 1e-12, "step")
