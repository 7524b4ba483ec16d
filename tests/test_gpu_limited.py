"""GPU parity of the limited face averages (section 2, eq. limitedFace) on
the single-level 1D+1V path against the oracle's limited scheme: the
right-hand side on random data (weights far from ideal) for FP64 and FP32,
RK4 steps with the field re-solved at every stage, a two-stream step at
1024 x 1024, every tile shape, and the unsupported combinations."""
import math

import numpy as np
import pytest
import torch

import vp_inputs as I

pytestmark = pytest.mark.gpu

SIZES = [(8, 8), (5, 12), (37, 45), (64, 64), (300, 517), (130, 1030)]


@pytest.fixture(scope="module")
def V():
    from paper_1204_3853_amd import vp
    vp.lib()
    return vp


def prob(nx, nv):
    return I.Problem1D(nx, nv, 0.0, 4.0 * math.pi, -8.0, 8.0, profile="maxwellian", eps=0.01, k=0.5)


def dev(x, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def rel(x, y):
    return np.abs(x - y).max() / max(np.abs(y).max(), 1e-300)


def limited_plan(V, p, dtype=torch.float64):
    plan = V.Plan(p, dtype=dtype)
    plan.set_face_scheme(V.FACE_LIMITED)
    return plan


@pytest.mark.parametrize("nx,nv", SIZES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rhs_limited(V, oracle, nx, nv, dtype):
    p = prob(nx, nv)
    f, a = I.random_state(nx, nv, seed=4321)
    plan = limited_plan(V, p, dtype)
    fg = dev(f, dtype)
    k = V.rhs(plan, fg, dev(a))
    ko = oracle.rhs_limited(host(fg), a, p.dx, p.dv, p.v_lo, p.vghost)
    assert rel(host(k), ko) <= (1e-12 if dtype == torch.float64 else 1e-5)
    kc = oracle.rhs(host(fg), a, p.dx, p.dv, p.v_lo, p.vghost)
    assert rel(kc, ko) > 1e-3             # the limiter is active on this data


@pytest.mark.parametrize("nx,nv", SIZES)
def test_rk4_limited(V, oracle, nx, nv):
    p = prob(nx, nv)
    rng = np.random.default_rng(7)
    f0 = p.initial_state() * (1.0 + 0.2 * rng.random((nx, nv)))
    o = oracle.Oracle1D.from_problem(p)
    plan = limited_plan(V, p)
    f = dev(f0)
    a = V.field_of(plan, f)
    dt = 0.5 / (8.0 / p.dx + 0.1 / p.dv)
    want = f0
    for s in range(3):
        V.rk4_step(plan, f, a, dt)
        want = o.step_limited(want, dt)
        assert rel(host(f), want) <= 1e-12 * (s + 1), f"step {s + 1}"


def test_two_stream_1024_limited(V, oracle):
    p = I.two_stream(1024, 1024)
    o = oracle.Oracle1D.from_problem(p)
    plan = limited_plan(V, p)
    f0 = p.initial_state()
    f = dev(f0)
    a = V.field_of(plan, f)
    dt = 4 * 4.788e-4
    V.rk4_step(plan, f, a, dt)
    assert rel(host(f), o.step_limited(f0, dt)) <= 1e-12


def test_every_tile_shape_limited(V, oracle):
    p = prob(130, 1030)
    f, a = I.random_state(130, 1030, seed=3)
    plan = limited_plan(V, p)
    ref = host(V.rhs(plan, dev(f), dev(a)))
    for q in range(len(plan.tile_shapes())):
        plan.set_tile_shape(q)
        np.testing.assert_allclose(host(V.rhs(plan, dev(f), dev(a))), ref, rtol=0, atol=1e-15 * np.abs(ref).max())


def test_limited_unsupported(V):
    p = prob(16, 16)
    plan = limited_plan(V, p)
    f = dev(p.initial_state())
    a = V.field_of(plan, f)
    with pytest.raises(V.VPError, match="ENOTSUP"):
        V.adjoint_step(plan, f, a, f.clone(), 0.01)
    with pytest.raises(V.VPError, match="ENOTSUP"):
        V.rk4_step_record(plan, f, a, 0.01)
    p2 = I.Problem2D(4, 4, 8, 8)
    plan2 = V.Plan(p2)
    with pytest.raises(V.VPError, match="ENOTSUP"):
        plan2.set_face_scheme(V.FACE_LIMITED)
