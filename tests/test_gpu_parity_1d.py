"""GPU parity of the 1D+1V single-level path against the CPU oracle.

Every call goes through the C ABI (include/vp.h) via the ctypes binding.
Inputs are seeded; sizes span several tiles of the stage kernel with
ragged tails in both directions, odd velocity counts (the scalar path) and
the full 4096 x 4096 two-stream configuration.

Tolerances: FP64 per step max|f_gpu - f_oracle| / max|f_oracle| <= 1e-12;
FP32 (FP32 input rounded from FP64, oracle run in FP64 on the rounded
input) <= 1e-5.  Moments are compared relatively at 1e-13, fields at 1e-10
of their maximum.
"""
import math

import numpy as np
import pytest
import torch

import vp_inputs as I

pytestmark = pytest.mark.gpu

SIZES = [(8, 8), (5, 12), (37, 45), (64, 64), (300, 517), (130, 1030), (257, 256)]
# configuration meshes that take the chunked field solve (ragged last chunk included)
SPLIT_SIZES = [(1024, 12), (1030, 16), (2051, 8), (8192, 6)]


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


@pytest.mark.parametrize("nx,nv", SIZES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rhs(V, oracle, nx, nv, dtype):
    print(f"rhs nx={nx} nv={nv} {dtype}", flush=True)
    p = prob(nx, nv)
    f, a = I.random_state(nx, nv, seed=1234)
    plan = V.Plan(p, dtype=dtype)
    fg = dev(f, dtype)
    k = V.rhs(plan, fg, dev(a))
    f_in = host(fg)                                   # the (possibly rounded) input the GPU saw
    ko = oracle.rhs(f_in, a, p.dx, p.dv, p.v_lo, p.vghost)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert rel(host(k), ko) <= tol


@pytest.mark.parametrize("nx,nv", SIZES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_reduce_moment(V, oracle, nx, nv, dtype):
    p = prob(nx, nv)
    f, _ = I.random_state(nx, nv, seed=99)
    plan = V.Plan(p, dtype=dtype)
    fg = dev(f, dtype)
    n = V.reduce_moment(plan, fg)
    no = oracle.moment(host(fg), p.dv)
    np.testing.assert_allclose(host(n), no, rtol=1e-13, atol=0)


@pytest.mark.parametrize("nx", [1, 2, 3, 5, 8, 41, 42, 64, 1000, 4096, 8192])
def test_poisson_field(V, oracle, nx):
    print(f"poisson nx={nx}", flush=True)
    p = prob(nx, 4)
    rng = np.random.default_rng(nx)
    n = 1.0 + 0.01 * rng.normal(size=nx)
    plan = V.Plan(p)
    phi, E = V.poisson_periodic(plan, dev(n))
    rho = 1.0 - n
    phio = oracle.poisson_solve(rho, p.dx)
    Eo = oracle.field(phio, p.dx)
    scale_phi = max(np.abs(phio).max(), 1e-30)
    scale_E = max(np.abs(Eo).max(), 1e-30)
    assert np.abs(host(phi) - phio).max() <= 1e-10 * scale_phi + 1e-300
    assert np.abs(host(E) - Eo).max() <= 1e-10 * scale_E + 1e-300
    a = V.inject_field(plan, E)
    np.testing.assert_array_equal(host(a), -host(E))


@pytest.mark.parametrize("nx,nv", SIZES + SPLIT_SIZES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("init", ["landau", "random"])
def test_rk4_step(V, oracle, nx, nv, dtype, init):
    print(f"rk4 nx={nx} nv={nv} {dtype} {init}", flush=True)
    p = prob(nx, nv)
    if init == "landau":
        f = p.initial_state()
    else:
        f = I.random_state(nx, nv, seed=7)[0] * p.veq[None, 2:-2] * 10
    plan = V.Plan(p, dtype=dtype)
    fg = dev(f, dtype)
    f_in = host(fg)
    o = oracle.Oracle1D.from_problem(p)
    a0 = o.constraints(f_in)[0]
    ag = V.field_of(plan, fg)
    # the split solve keeps its mesh-wide sums in double-double and the
    # oracle refines its LU solve, so a stays near rounding at every size
    atol_a = 1e-12
    assert np.abs(host(ag) - a0).max() <= atol_a * max(np.abs(a0).max(), 1e-12) + 1e-15
    dt = 0.5 / (8.0 / p.dx + 0.1 / p.dv)
    V.rk4_step(plan, fg, ag, dt)
    fo = o.step(f_in, dt)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert rel(host(fg), fo) <= tol
    a1 = o.constraints(fo)[0]
    assert np.abs(host(ag) - a1).max() <= (1e-12 if dtype == torch.float64 else 1e-4) * \
        max(np.abs(a1).max(), 1e-12) + 1e-15


def test_rk4_landau_100_steps(V, oracle):
    """Landau 64 x 64, 100 steps at the CFL 0.5 step: drift reported, bounded."""
    p = I.landau_64()
    plan = V.Plan(p)
    o = oracle.Oracle1D.from_problem(p)
    f = p.initial_state()
    fg = dev(f)
    ag = V.field_of(plan, fg)
    dt = 0.012248
    fo = f.copy()
    for _ in range(100):
        V.rk4_step(plan, fg, ag, dt)
        fo = o.step(fo, dt)
    d = rel(host(fg), fo)
    print(f"landau 64x64 100-step drift {d:.3e}")
    assert d <= 1e-11


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rk4_step_two_stream_4096(V, oracle, dtype):
    """Full-size two-stream 4096 x 4096: one step in the launch
    configuration the benchmark times, compared element by element."""
    print(f"two-stream 4096^2 {dtype}", flush=True)
    p = I.two_stream(4096, 4096)
    f = p.initial_state()
    plan = V.Plan(p, dtype=dtype)
    fg = dev(f, dtype)
    f_in = host(fg)
    ag = V.field_of(plan, fg)
    dt = 4.788e-4
    V.rk4_step(plan, fg, ag, dt)
    o = oracle.Oracle1D.from_problem(p)
    fo = o.step(f_in, dt)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    d = rel(host(fg), fo)
    print(f"two-stream 4096^2 {dtype} rel diff {d:.3e}")
    assert d <= tol


def test_rhs_rejects_bad_arguments(V):
    p = prob(16, 16)
    plan = V.Plan(p)
    f = torch.zeros(16 * 16, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        V.rhs(plan, torch.zeros(15 * 16, dtype=torch.float64, device="cuda"),
              torch.zeros(16, dtype=torch.float64, device="cuda"))
    code = V.lib().vp_rhs(plan.h, V._ptr(f), None, V._ptr(f), V._stream())
    assert code == 1                                    # VP_EINVAL, nothing enqueued
    assert b"NULL" in V.lib().vp_last_error() or b"alias" in V.lib().vp_last_error()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rk4_step_every_tile_shape(V, oracle, dtype):
    """Every compiled tile shape of the stage kernel gives the oracle's step
    (the autotuner may pick any of them); ragged in x and v for every shape."""
    nx, nv = 37, 1040
    p = prob(nx, nv)
    f = I.random_state(nx, nv, seed=11)[0] * p.veq[None, 2:-2] * 10
    plan = V.Plan(p, dtype=dtype)
    f_in = host(dev(f, dtype))
    o = oracle.Oracle1D.from_problem(p)
    dt = 0.5 / (8.0 / p.dx + 0.1 / p.dv)
    want = o.step(f_in, dt)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    shapes = plan.tile_shapes()
    assert len(shapes) >= 10
    for q, shp in enumerate(shapes):
        print(f"shape {shp} {dtype}", flush=True)
        plan.set_tile_shape(q)
        fg = dev(f, dtype)
        ag = V.field_of(plan, fg)
        V.rk4_step(plan, fg, ag, dt)
        assert rel(host(fg), want) <= tol, shp
