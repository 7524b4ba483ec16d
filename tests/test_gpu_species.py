"""GPU parity of several species on one configuration mesh
(vp_species_field, vp_species_rk4_step) against the several-species oracle.

Electron-ion plasmas (mass ratio 100, ions on their own narrower velocity
mesh with another cell count), three species, the small-mesh and the split
(nx >= 1024) field solves, FP32 states, and the argument errors.  FP64:
1e-12 relative per step; FP32: 1e-5 against the FP64 oracle started from the
FP32-rounded states.
"""
import math

import numpy as np
import pytest

import vp_inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vp():
    from paper_1204_3853_amd import vp as V
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return V


def ion_problem(nx, nv, x_len, mass=100.0, eps=0.02, k=0.5):
    vth = 1.0 / math.sqrt(mass)
    veq = I.cell_average_1d(lambda u: I.maxwellian(u / vth) / vth, -8 * vth, 8 * vth, nv, first=-2, count=nv + 4)
    return I.Problem1D(nx=nx, nv=nv, x_lo=0.0, x_len=x_len, v_lo=-8 * vth, v_hi=8 * vth, qm=1.0 / mass, eps=eps,
                       k=k, veq=veq)


def species_of(p):
    return {"dv": p.dv, "v_lo": p.v_lo, "vghost": p.vghost, "qm": p.qm}


def run_case(vp, oracle, probs, charges, background, steps, dt, dtype=torch.float64, noise=0.0):
    plans = [vp.Plan(p, dtype=dtype) for p in probs]
    rng = np.random.default_rng(7)
    f0 = [p.initial_state() * (1.0 + noise * rng.random((p.nx, p.nv))) for p in probs]
    fs = [torch.tensor(f, dtype=dtype, device="cuda").reshape(-1) for f in f0]
    g = vp.SpeciesGroup(plans, charges, background)
    a = g.field(fs)
    sp = [species_of(p) for p in probs]
    start = [f.double().cpu().numpy().reshape(p.nx, p.nv) for f, p in zip(fs, probs)]
    want_a, _ = oracle.species_field(start, sp, charges, background, probs[0].dx)
    tol_a = 1e-12
    for ag, aw in zip(a, want_a):
        assert np.abs(ag.cpu().numpy() - aw).max() <= tol_a * max(np.abs(aw).max(), 1e-300)
    want = start
    for _ in range(steps):
        g.rk4_step(fs, a, dt)
        want = oracle.species_rk4_step(want, sp, charges, background, probs[0].dx, dt)
    tol = 1e-12 * steps if dtype == torch.float64 else 1e-5 * steps
    for f, w in zip(fs, want):
        got = f.double().cpu().numpy().reshape(w.shape)
        assert np.abs(got - w).max() <= tol * np.abs(w).max()
    # the accelerations after the step are the field of the new states
    want_a, _ = oracle.species_field(want, sp, charges, background, probs[0].dx)
    tol_a = 1e-11 * steps if dtype == torch.float64 else 1e-4
    for ag, aw in zip(a, want_a):
        assert np.abs(ag.cpu().numpy() - aw).max() <= tol_a * np.abs(aw).max()


@pytest.mark.parametrize("nx,nve,nvi", [(37, 45, 30), (64, 128, 64)])
def test_electrons_and_ions(vp, oracle, nx, nve, nvi):
    pe = I.landau(nx, nve, eps=0.05)
    pi_ = ion_problem(nx, nvi, pe.x_len)
    run_case(vp, oracle, [pe, pi_], [-1.0, 1.0], 0.0, 3, 0.05, noise=0.01)


def test_three_species_split_field(vp, oracle):
    nx = 1024
    pe = I.landau(nx, 64, eps=0.02)
    pi_ = ion_problem(nx, 33, pe.x_len, mass=25.0)
    pp = I.Problem1D(nx=nx, nv=40, x_lo=0.0, x_len=pe.x_len, v_lo=-6.0, v_hi=6.0, qm=+1.0, eps=0.01, k=1.0)
    # neutral on average: -1 + 1 + 0.5 - 0.5
    run_case(vp, oracle, [pe, pi_, pp], [-1.0, 1.0, 0.5], -0.5, 2, 0.01, noise=0.01)


def test_single_species_matches_the_plan_step(vp, oracle):
    """One species of charge -1 over a unit background: the group step equals
    the plan's own step to rounding."""
    p = I.two_stream(256, 512)
    plan = vp.Plan(p)
    f = torch.tensor(p.initial_state().ravel(), device="cuda")
    f2 = f.clone()
    a = vp.field_of(plan, f)
    g = vp.SpeciesGroup([plan], [-1.0], 1.0)
    a2 = g.field([f2])[0]
    assert torch.allclose(a, a2, rtol=0, atol=1e-13 * float(a.abs().max()))
    for _ in range(3):
        vp.rk4_step(plan, f, a, 1e-3)
        g.rk4_step([f2], [a2], 1e-3)
    assert float((f - f2).abs().max()) <= 1e-12 * float(f.abs().max())


def test_fp32_species(vp, oracle):
    pe = I.landau(96, 128, eps=0.05)
    pi_ = ion_problem(96, 64, pe.x_len)
    run_case(vp, oracle, [pe, pi_], [-1.0, 1.0], 0.0, 2, 0.05, dtype=torch.float32, noise=0.01)


def test_group_errors(vp):
    pe = I.landau(32, 48)
    plan = vp.Plan(pe)
    with pytest.raises(vp.VPError, match="configuration mesh"):
        vp.SpeciesGroup([plan, vp.Plan(I.landau(16, 48))], [-1.0, 1.0])
    with pytest.raises(vp.VPError, match="dtype"):
        vp.SpeciesGroup([plan, vp.Plan(pe, dtype=torch.float32)], [-1.0, 1.0])
    with pytest.raises(vp.VPError, match="species"):
        vp.SpeciesGroup([plan] * 5, [-1.0] * 5)
    with pytest.raises(vp.VPError, match="finite"):
        vp.SpeciesGroup([plan], [float("inf")])
    boxes = [{"level": 1, "lo": [0, 0], "hi": [7, 7]}]
    f, vc, vf = I.amr_landau(boxes, coarse=(32, 48), ratio=4)
    two = vp.Plan(vp.two_level_spec(32, 48, 4 * math.pi, -8.0, 8.0, -1.0, 4, vc, vf), boxes=boxes)
    with pytest.raises(vp.VPError, match="configuration mesh"):     # finest meshes of 32 and 128 cells
        vp.SpeciesGroup([plan, two], [-1.0, 1.0])
    with pytest.raises(vp.VPError, match="1D"):
        vp.SpeciesGroup([vp.Plan(I.Problem2D(8, 8, 16, 16))], [-1.0])


# ---- one two-level hierarchy per species

E_BOXES = [{"level": 1, "lo": [8, 64], "hi": [39, 127]}, {"level": 1, "lo": [64, 80], "hi": [99, 111]}]
I_BOXES = [{"level": 1, "lo": [0, 32], "hi": [27, 63]}, {"level": 1, "lo": [48, 40], "hi": [119, 55]}]


def amr_species(vp, oracle, ncx, ncv, R, qm, v_lo, v_hi, profile, boxes, eps, noise, seed):
    f, vc, vf = I._amr_state(profile, 0.0, 4 * math.pi, v_lo, v_hi, eps, 0.5, boxes, (ncx, ncv), R)
    f = f * (1.0 + noise * np.random.default_rng(seed).random(f.size))
    spec = vp.two_level_spec(ncx, ncv, 4 * math.pi, v_lo, v_hi, qm, R, vc, vf)
    plan = vp.Plan(spec, boxes=boxes)
    o = oracle.OracleAMR(ncx, ncv, 4 * math.pi, v_lo, v_hi, qm, R, boxes, vc, vf)
    return plan, o, f


def test_two_level_electrons_and_ions(vp, oracle):
    ncx, R = 32, 4
    vth = 0.1
    ion = lambda u: I.maxwellian(u / vth) / vth
    pe, oe, fe = amr_species(vp, oracle, ncx, 48, R, -1.0, -8.0, 8.0, I.maxwellian, E_BOXES, 0.05, 0.01, 1)
    pi_, oi, fi = amr_species(vp, oracle, ncx, 24, R, 0.01, -8 * vth, 8 * vth, ion, I_BOXES, 0.02, 0.01, 2)
    g = vp.SpeciesGroup([pe, pi_], [-1.0, 1.0], 0.0)
    fs = [torch.tensor(fe, device="cuda"), torch.tensor(fi, device="cuda")]
    a = g.field(fs)
    want_a = oracle.amr_species_field([oe, oi], [fe, fi], [-1.0, 1.0], 0.0)
    for ag, aw in zip(a, want_a):
        assert np.abs(ag.cpu().numpy() - aw).max() <= 1e-11 * np.abs(aw).max()
    want = [fe, fi]
    dt = 0.5 * (4 * math.pi / (ncx * R)) / 8.0
    for _ in range(3):
        g.rk4_step(fs, a, dt)
        want = oracle.amr_species_rk4_step([oe, oi], want, [-1.0, 1.0], 0.0, dt)
    for f, w in zip(fs, want):
        assert np.abs(f.cpu().numpy() - w).max() <= 3e-12 * np.abs(w).max()
    want_a = oracle.amr_species_field([oe, oi], want, [-1.0, 1.0], 0.0)
    for ag, aw in zip(a, want_a):
        assert np.abs(ag.cpu().numpy() - aw).max() <= 1e-9 * np.abs(aw).max()


def test_two_level_single_species_matches_the_plan_step(vp, oracle):
    pe, oe, fe = amr_species(vp, oracle, 32, 48, 4, -1.0, -8.0, 8.0, I.maxwellian, E_BOXES, 0.05, 0.0, 1)
    f = torch.tensor(fe, device="cuda")
    f2 = f.clone()
    a = vp.field_of(pe, f)
    g = vp.SpeciesGroup([pe], [-1.0], 1.0)
    a2 = g.field([f2])[0]
    assert float((a - a2).abs().max()) <= 1e-12 * float(a.abs().max())
    for _ in range(2):
        vp.rk4_step(pe, f, a, 0.01)
        g.rk4_step([f2], [a2], 0.01)
    assert float((f - f2).abs().max()) <= 1e-12 * float(f.abs().max())
