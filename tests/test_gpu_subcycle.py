"""GPU parity of the subcycled two-level step (vp_amr_subcycle_step) against
the FP64 oracle: the coarse level takes dt with the field of its own moment,
the patches R substeps of dt / R whose coarse data come from the continuous
extension of the coarse RK4 step, then refluxing and the average-down
(asynchronous stepping, future work of section 5).

Layouts: the small ratio-4 hierarchy (three patches, one across the periodic
x boundary), the ratio-2 hierarchy with an odd coarse velocity count, no
patches at all, the 512 x 512 ratio-4 hierarchy with 40 patches and one with
a single large patch over a high-velocity band; graph replay, the Mask
reduction, and the Landau damping rate of a GPU run.
"""
import math

import numpy as np
import pytest

import vp_inputs as I
from test_gpu_amr import LAYOUTS, Case, cmp, rel_tol

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vp():
    from paper_1204_3853_amd import vp as V
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return V


@pytest.fixture(scope="module", params=list(LAYOUTS))
def case(request, vp, oracle):
    L = LAYOUTS[request.param]
    return Case(vp, oracle, L["boxes"], L["ncx"], L["ncv"], L["R"])


def test_one_subcycled_step(vp, case):
    f = case.gpu(case.f0)
    a = torch.zeros(case.plan.field_elems, dtype=torch.float64, device="cuda")
    vp.amr_subcycle_step(case.plan, f, a, case.dt * case.R)
    torch.cuda.synchronize()
    want = case.o.subcycle_step(case.f0, case.dt * case.R)
    cmp(f, want, rel_tol(), "subcycled step")
    cmp(a, case.o.constraints(want)[0], rel_tol(), "field after the step")
    # the subcycled step is not the synchronous one
    assert np.abs(want - case.o.step(case.f0, case.dt * case.R)).max() > 1e-10


def test_several_subcycled_steps(vp, case):
    f = case.gpu(case.f0)
    a = torch.zeros(case.plan.field_elems, dtype=torch.float64, device="cuda")
    want = case.f0
    for _ in range(3):
        vp.amr_subcycle_step(case.plan, f, a, case.dt * case.R)
        want = case.o.subcycle_step(want, case.dt * case.R)
    torch.cuda.synchronize()
    cmp(f, want, 3 * rel_tol(), "three subcycled steps")


def test_subcycle_interleaves_with_synchronous_steps(vp, case):
    """The subcycled step leaves the workspace in a state the synchronous
    step does not depend on (and the other way round)."""
    f = case.gpu(case.f0)
    a = vp.field_of(case.plan, f)
    vp.rk4_step(case.plan, f, a, case.dt)
    vp.amr_subcycle_step(case.plan, f, a, case.dt * case.R)
    vp.rk4_step(case.plan, f, a, case.dt)
    torch.cuda.synchronize()
    want = case.o.step(case.o.subcycle_step(case.o.step(case.f0, case.dt), case.dt * case.R), case.dt)
    cmp(f, want, 3 * rel_tol(), "sync, subcycled, sync")


def test_no_patches(vp, oracle):
    ncx, ncv, R = 40, 36, 2
    f0, veq_c, veq_f = I.amr_landau([], coarse=(ncx, ncv), ratio=R, eps=0.2)
    plan = vp.Plan(vp.two_level_spec(ncx, ncv, 4 * math.pi, -8.0, 8.0, -1.0, R, veq_c, veq_f), boxes=[])
    o = oracle.OracleAMR(ncx, ncv, 4 * math.pi, -8.0, 8.0, -1.0, R, [], veq_c, veq_f)
    f = torch.tensor(f0, dtype=torch.float64, device="cuda")
    a = torch.zeros(plan.field_elems, dtype=torch.float64, device="cuda")
    dt = 0.05
    vp.amr_subcycle_step(plan, f, a, dt)
    torch.cuda.synchronize()
    cmp(f, o.subcycle_step(f0, dt), rel_tol(), "subcycled step without patches")


def test_full_config_subcycled_step(vp, oracle):
    boxes = I.amr_boxes(0)
    c = Case(vp, oracle, boxes, 512, 512, 4, eps=0.01, k=0.5, noise=0.0)
    f = c.gpu(c.f0)
    a = torch.zeros(c.plan.field_elems, dtype=torch.float64, device="cuda")
    vp.amr_subcycle_step(c.plan, f, a, 4 * c.dt)
    torch.cuda.synchronize()
    cmp(f, c.o.subcycle_step(c.f0, 4 * c.dt), rel_tol(), "512 x 512 subcycled step")


def test_errors(vp):
    p = I.landau(32, 32)
    plan = vp.Plan(p)
    f = torch.tensor(p.initial_state().ravel(), device="cuda")
    a = vp.field_of(plan, f)
    with pytest.raises(vp.VPError, match="two-level"):
        vp.amr_subcycle_step(plan, f, a, 0.01)
    L = LAYOUTS["small"]
    f0, veq_c, veq_f = I.amr_landau(L["boxes"], coarse=(L["ncx"], L["ncv"]), ratio=L["R"])
    plan2 = vp.Plan(vp.two_level_spec(L["ncx"], L["ncv"], 4 * math.pi, -8.0, 8.0, -1.0, L["R"], veq_c, veq_f),
                    boxes=L["boxes"])
    f2 = torch.tensor(f0, dtype=torch.float64, device="cuda")
    a2 = torch.zeros(plan2.field_elems, dtype=torch.float64, device="cuda")
    with pytest.raises(vp.VPError, match="finite"):
        vp.amr_subcycle_step(plan2, f2, a2, float("nan"))


def test_high_velocity_band_layout(vp, oracle):
    """One patch of 2044 x 448 fine cells over v in [4, 7.5) (the layout the
    subcycling benchmark also times): synchronous and subcycled steps."""
    R = 4
    boxes = [{"level": 1, "lo": [0, 12 * 32 * R], "hi": [511 * R - 1, 496 * R - 1]}]
    c = Case(vp, oracle, boxes, 512, 512, R, eps=0.01, k=0.5, noise=0.0)
    f = c.gpu(c.f0)
    a = vp.field_of(c.plan, f)
    vp.rk4_step(c.plan, f, a, c.dt)
    torch.cuda.synchronize()
    cmp(f, c.o.step(c.f0, c.dt), rel_tol(), "synchronous step, band layout")
    f = c.gpu(c.f0)
    vp.amr_subcycle_step(c.plan, f, a, 2 * c.dt)
    torch.cuda.synchronize()
    cmp(f, c.o.subcycle_step(c.f0, 2 * c.dt), rel_tol(), "subcycled step, band layout")


def test_graph_replay_matches_eager(vp, oracle):
    """The subcycled step captured in a HIP graph and replayed gives the
    eager results, replay after replay (with eager work in between)."""
    L = LAYOUTS["small"]
    c = Case(vp, oracle, L["boxes"], L["ncx"], L["ncv"], L["R"])
    f_e = c.gpu(c.f0)
    a_e = vp.field_of(c.plan, f_e)
    f_g, a_g = f_e.clone(), a_e.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        vp.amr_subcycle_step(c.plan, f_g, a_g, 4 * c.dt)
    torch.cuda.current_stream().wait_stream(s)
    vp.amr_subcycle_step(c.plan, f_e, a_e, 4 * c.dt)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        vp.amr_subcycle_step(c.plan, f_g, a_g, 4 * c.dt)
    for r in range(3):
        g.replay()
        vp.amr_subcycle_step(c.plan, f_e, a_e, 4 * c.dt)
        torch.cuda.synchronize()
        assert torch.equal(f_g, f_e), f"replay {r}"
        assert torch.equal(a_g, a_e), f"replay {r}"


def test_subcycle_with_mask_reduction(vp, oracle):
    """The fine stages' composite moment by the Mask reduction gives the
    same step (both reductions are exact sums of the same cells)."""
    L = LAYOUTS["ratio2_odd"]
    c = Case(vp, oracle, L["boxes"], L["ncx"], L["ncv"], L["R"])
    c.plan.set_reduction(vp.REDUCE_MASK)
    try:
        f = c.gpu(c.f0)
        a = torch.zeros(c.plan.field_elems, dtype=torch.float64, device="cuda")
        vp.amr_subcycle_step(c.plan, f, a, 2 * c.dt)
        torch.cuda.synchronize()
        cmp(f, c.o.subcycle_step(c.f0, 2 * c.dt), rel_tol(), "subcycled step, Mask reduction")
    finally:
        c.plan.set_reduction(vp.REDUCE_FUSED)


def test_subcycled_landau_damping_rate_on_gpu(vp):
    """Physics of the GPU path alone: 64 x 128 coarse cells with a ratio-2
    patch over v in [1, 3.625) (every coarse column but the last), subcycled
    to t = 30: the field decays at the Landau rate (the root of the
    dispersion relation for k = 0.5)."""
    from test_oracle_pins import landau_fit, landau_root
    w = landau_root()
    ncx, ncv, R = 64, 128, 2
    boxes = [{"level": 1, "lo": [0, 72 * R], "hi": [63 * R - 1, 93 * R - 1]}]
    f0, veq_c, veq_f = I._amr_state(I.maxwellian, 0.0, 4 * math.pi, -8.0, 8.0, 0.01, 0.5, boxes, (ncx, ncv), R)
    plan = vp.Plan(vp.two_level_spec(ncx, ncv, 4 * math.pi, -8.0, 8.0, -1.0, R, veq_c, veq_f), boxes=boxes)
    a = torch.zeros(plan.field_elems, dtype=torch.float64, device="cuda")

    class P:
        dx = 4 * math.pi / (ncx * R)

        @staticmethod
        def initial_state():
            return torch.tensor(f0, dtype=torch.float64, device="cuda")

    def step(g, dt):
        vp.amr_subcycle_step(plan, g, a, dt)
        return g

    def field(g):
        return -vp.field_of(plan, g)[ncx:].cpu().numpy()          # E = a / (q/m), q/m = -1

    dt = 0.5 / (8.0 / (4 * math.pi / ncx) + 0.01 / (16.0 / ncv))
    gamma, omega = landau_fit(step, field, P, dt)
    assert abs(gamma - w.imag) < 0.003, gamma
    assert abs(omega - w.real) < 0.006, omega
