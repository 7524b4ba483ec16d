"""GPU test of vp_rk4_step_noalloc, the RK4 step whose workspace is the
library's static device scratch array: two calls in a row through the C ABI
(the second on a smaller mesh, so that it runs on what the first left in
the array) each agree with vp_rk4_step on the same input, to the parity bar
of the single-level path (max |diff| / max |f| <= 1e-12 in FP64, 1e-5 in
FP32; the two entry points run the same kernels, so they are expected to
agree bit for bit).  Size and plan-kind rejections are checked too."""
import math

import numpy as np
import pytest
import torch

import vp_inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    from paper_1204_3853_amd import vp
    vp.lib()
    return vp


def prob(nx, nv):
    return I.Problem1D(nx, nv, 0.0, 4.0 * math.pi, -8.0, 8.0, profile="maxwellian", eps=0.01, k=0.5)


def rel(x, y):
    return (x - y).abs().max().item() / max(y.abs().max().item(), 1e-300)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_step_matches_rk4_step(V, dtype):
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    dt = 0.01
    for call, (nx, nv) in enumerate([(1030, 517), (37, 45)]):      # larger, then smaller
        print(f"noalloc call {call}: {nx}x{nv} {dtype}", flush=True)
        p = prob(nx, nv)
        plan = V.Plan(p, dtype=dtype)
        f0, _ = I.random_state(nx, nv, seed=1234 + call)
        f_ref = torch.tensor(f0, dtype=dtype, device="cuda")
        a_ref = V.field_of(plan, f_ref)
        f_na = f_ref.clone()
        a_na = a_ref.clone()
        for _ in range(2):                                            # two steps each
            V.rk4_step(plan, f_ref, a_ref, dt)
            V.rk4_step_noalloc(plan, f_na, a_na, dt)
        torch.cuda.synchronize()
        assert rel(f_na.double(), f_ref.double()) <= tol
        assert rel(a_na, a_ref) <= 1e-12
        print(f"  bitwise equal: {bool(torch.equal(f_na, f_ref) and torch.equal(a_na, a_ref))}", flush=True)


def test_noalloc_rejects_what_it_cannot_hold(V):
    big = V.Plan(prob(2048, 2048), dtype=torch.float64)        # 3 states of 32 MiB: beyond the array
    f = torch.zeros(big.state_elems, dtype=torch.float64, device="cuda")
    a = torch.zeros(big.field_elems, dtype=torch.float64, device="cuda")
    with pytest.raises(V.VPError) as e:
        V.rk4_step_noalloc(big, f, a, 0.01)
    assert e.value.code == 2                                     # VP_ESHAPE
    boxes = [{"level": 1, "lo": [16, 40], "hi": [39, 63]}]
    _, veq_c, veq_f = I.amr_landau(boxes, coarse=(32, 48), ratio=4)
    two = V.Plan(V.two_level_spec(32, 48, 4 * math.pi, -8.0, 8.0, -1.0, 4, veq_c, veq_f), boxes=boxes)
    f2 = torch.zeros(two.state_elems, dtype=torch.float64, device="cuda")
    a2 = torch.zeros(two.field_elems, dtype=torch.float64, device="cuda")
    with pytest.raises(V.VPError) as e:
        V.rk4_step_noalloc(two, f2, a2, 0.01)
    assert e.value.code == 4                                     # VP_ENOTSUP
