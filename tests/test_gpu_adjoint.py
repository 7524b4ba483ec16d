"""GPU discrete adjoint against the CPU oracle's adjoint, finite differences
and the dot-product identity.  All calls go through the C ABI.

Tolerances: one adjoint step <= 1e-11 of max|lam_n| against the oracle;
rollout gradients against central finite differences <= 1e-6 relative
and against the oracle's chained adjoint <= 1e-10 relative.
"""
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


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("nx,nv", [(8, 8), (5, 12), (37, 46), (33, 45), (64, 64), (130, 1030), (257, 256)])
@pytest.mark.parametrize("use_record", [False, True])
def test_adjoint_step_vs_oracle(V, oracle, nx, nv, use_record):
    print(f"adjoint step nx={nx} nv={nv} record={use_record}", flush=True)
    p = I.Problem1D(nx, nv, 0.0, 4.0 * math.pi, -8.0, 8.0, eps=0.05, k=0.5)
    rng = np.random.default_rng(nx * 1000 + nv)
    f = p.initial_state() * (1 + 0.3 * rng.random((nx, nv)))
    lam = rng.normal(size=(nx, nv))
    dt = 0.5 / (8.0 / p.dx + 0.1 / p.dv)
    plan = V.Plan(p)
    fg = dev(f)
    a = V.field_of(plan, fg)
    rec = None
    if use_record:
        f2, a2 = fg.clone(), a.clone()
        _, _, rec = V.rk4_step_record(plan, f2, a2, dt)
    mu = V.adjoint_step(plan, fg, a, dev(lam), dt, stages=rec)
    o = oracle.Oracle1D.from_problem(p)
    mo = o.adjoint_step(f, lam, dt)
    d = np.abs(host(mu) - mo).max() / np.abs(mo).max()
    assert d <= 1e-11, d


def test_adjoint_record_path_is_bitwise_recompute(V):
    p = I.landau(40, 64)
    plan = V.Plan(p)
    rng = np.random.default_rng(3)
    fg = dev(p.initial_state())
    a = V.field_of(plan, fg)
    lam = dev(rng.normal(size=(40, 64)))
    dt = 0.01
    f2, a2 = fg.clone(), a.clone()
    _, _, rec = V.rk4_step_record(plan, f2, a2, dt)
    m1 = V.adjoint_step(plan, fg, a, lam, dt, stages=rec)
    m2 = V.adjoint_step(plan, fg, a, lam, dt)
    assert torch.equal(m1, m2)


@pytest.mark.parametrize("nx", [1, 2, 5, 64, 512, 4096])
def test_field_adjoint_vs_oracle(V, oracle, nx):
    p = I.landau(nx, 16)
    plan = V.Plan(p)
    rng = np.random.default_rng(nx)
    abar = rng.normal(size=nx)
    fb = V.field_adjoint(plan, dev(abar))
    o = oracle.Oracle1D.from_problem(p)
    fo = o.constraints_adjoint(abar, np.zeros((nx, 16)))
    scale = max(np.abs(fo).max(), 1e-300)
    assert np.abs(host(fb).reshape(nx, 16) - fo).max() <= 1e-11 * scale + 1e-300


def test_adjoint_dot_product_vs_gpu_forward(V):
    """<lam, (f(x + h u) - f(x - h u)) / 2h> = <u, J^T lam> with the GPU
    forward step on both sides."""
    p = I.landau(48, 64)
    plan = V.Plan(p)
    rng = np.random.default_rng(9)
    f = p.initial_state() * (1 + 0.2 * rng.random((48, 64)))
    lam = rng.normal(size=(48, 64))
    dt = 0.01
    fg = dev(f)
    a = V.field_of(plan, fg)
    mu = host(V.adjoint_step(plan, fg, a, dev(lam), dt))
    for trial in range(3):
        u = rng.normal(size=f.shape)
        h = 1e-5
        outs = []
        for sgn in (1, -1):
            x = dev(f + sgn * h * u)
            ax = V.field_of(plan, x)
            V.rk4_step(plan, x, ax, dt)
            outs.append(host(x))
        fd = ((outs[0] - outs[1]) / (2 * h) * lam).sum()
        ad = (u * mu).sum()
        assert abs(fd - ad) <= 1e-7 * abs(ad), (fd, ad)


def gradient_gpu(V, prob, c, pvec, g, dt, nsteps, every):
    from paper_1204_3853_amd import autograd as AG
    plan = V.Plan(prob)
    pt = torch.tensor(pvec, dtype=torch.float64, device="cuda", requires_grad=True)
    ct = dev(c)
    gt = dev(g)
    f0 = ((1.0 + ct + pt)[:, None] * gt[None, :]).contiguous()
    fT = AG.rollout(f0, plan, dt, nsteps, every)
    W = AG.field_energy(fT, plan)
    W.backward()
    return float(W), host(pt.grad)


def energy_gpu(V, plan, prob, c, pvec, g, dt, nsteps):
    f = dev((1.0 + c + pvec)[:, None] * g[None, :])
    a = V.field_of(plan, f)
    for _ in range(nsteps):
        V.rk4_step(plan, f, a, dt)
    E = host(a) / prob.qm
    return 0.5 * (E * E).sum()


def oracle_gradient(oracle, prob, c, pvec, g, dt, nsteps):
    o = oracle.Oracle1D.from_problem(prob)
    f = (1.0 + c + pvec)[:, None] * g[None, :]
    states = []
    for _ in range(nsteps):
        states.append(f)
        f = o.step(f, dt)
    a, n, phi, E = o.constraints(f)
    lam = o.constraints_adjoint(E / prob.qm, np.zeros_like(f))
    for fs in reversed(states):
        lam = o.adjoint_step(fs, lam, dt)
    return (lam * g[None, :]).sum(axis=1)


def test_rollout_gradient_small(V, oracle):
    """64 x 64, 40 steps, checkpoint every 10: gradient of the final field
    energy w.r.t. the initial profile against finite differences and the
    oracle's chained discrete adjoint."""
    prob, c, pvec = I.adjoint_setup(64, 64, seed=0)
    g = prob.veq[2:-2]
    dt = 0.5 / (8.0 / prob.dx + 0.02 / prob.dv)
    W, grad = gradient_gpu(V, prob, c, pvec, g, dt, 40, 10)
    go = oracle_gradient(oracle, prob, c, pvec, g, dt, 40)
    assert np.abs(grad - go).max() <= 1e-10 * np.abs(go).max()
    plan = V.Plan(prob)
    for d in I.adjoint_directions(64, 4, seed=1):
        h = 1e-6
        fd = (energy_gpu(V, plan, prob, c, pvec + h * d, g, dt, 40)
              - energy_gpu(V, plan, prob, c, pvec - h * d, g, dt, 40)) / (2 * h)
        assert abs(fd - grad @ d) <= 1e-6 * abs(grad @ d), (fd, grad @ d)


def test_rollout_gradient_adj_config(V, oracle):
    """Adjoint workload: Landau 512 x 512, 400 steps, checkpoint every 20;
    8 random unit directions, central differences h = 1e-6; and the
    oracle's chained discrete adjoint."""
    prob, c, pvec = I.adjoint_setup(512, 512, seed=0)
    g = prob.veq[2:-2]
    dt = 1.531e-3
    W, grad = gradient_gpu(V, prob, c, pvec, g, dt, 400, 20)
    plan = V.Plan(prob)
    worst = 0.0
    for d in I.adjoint_directions(512, 8, seed=1):
        h = 1e-6
        fd = (energy_gpu(V, plan, prob, c, pvec + h * d, g, dt, 400)
              - energy_gpu(V, plan, prob, c, pvec - h * d, g, dt, 400)) / (2 * h)
        worst = max(worst, abs(fd - grad @ d) / abs(grad @ d))
    print(f"ADJ 512^2 x 400: W={W:.6e}, worst FD rel diff {worst:.2e}")
    assert worst <= 1e-6
    go = oracle_gradient(oracle, prob, c, pvec, g, dt, 400)
    d = np.abs(grad - go).max() / np.abs(go).max()
    print(f"ADJ gradient vs oracle rel diff {d:.2e}")
    assert d <= 1e-10
