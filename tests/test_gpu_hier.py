"""GPU parity of the multi-level path (L <= 4 levels, a refinement ratio per
level and direction, touching patches) against the FP64 multi-level oracle
(oracle/vp_oracle_hier.c): ghost frames (same-level copy, equilibrium,
parent interpolation), Sub-Patch reduction vs the oracle's Mask reduction,
field and injection on every level, right-hand side, RK4 steps with the
coarse-fine correction and the average-down of every level pair.

Layouts (all with touching patches, some across the periodic x boundary):
  three levels, ratios [2,4], [4,2] on 32 x 24;
  two levels with the anisotropic ratio [2,4];
  four levels with the section-4 ratios [2,4], [4,2], [2,2] on the
  section-4 level-0 mesh of 16 x 32 cells;
  three levels that each cover the whole domain.
Tolerances: f per step 1e-12 of max|f| (FP64), n 1e-13, a 1e-11.
"""
import math

import numpy as np
import pytest

import vp_inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

X_LEN, V_LO, V_HI = 4 * math.pi, -8.0, 8.0


def box(level, x0, v0, x1, v1):
    return {"level": level, "lo": [x0, v0], "hi": [x1, v1]}


LAYOUTS = {
    "three_levels": dict(coarse=(32, 24), ratios=[(2, 4), (4, 2)], boxes=[
        box(1, 8, 24, 31, 71), box(1, 32, 24, 43, 71), box(1, 0, 32, 7, 55), box(1, 56, 40, 63, 55),
        box(2, 56, 64, 119, 119), box(2, 120, 64, 143, 119), box(2, 240, 88, 255, 95)]),
    "two_levels_2x4": dict(coarse=(24, 20), ratios=[(2, 4)], boxes=[
        box(1, 6, 20, 17, 39), box(1, 18, 24, 27, 35), box(1, 0, 60, 9, 79), box(1, 38, 64, 47, 75),
        box(1, 20, 0, 25, 7)]),
    "four_levels": dict(coarse=(16, 32), ratios=[(2, 4), (4, 2), (2, 2)], boxes=[
        box(1, 0, 32, 15, 95), box(1, 16, 32, 31, 95),
        box(2, 0, 80, 63, 175), box(2, 64, 96, 127, 159),
        box(3, 16, 176, 111, 335), box(3, 140, 200, 241, 311)]),
    "full_cover": dict(coarse=(8, 8), ratios=[(2, 2), (2, 4)], boxes=[
        box(1, 0, 0, 5, 15), box(1, 6, 0, 15, 7), box(1, 6, 8, 15, 15),
        box(2, 0, 0, 11, 63), box(2, 12, 0, 31, 31), box(2, 12, 32, 31, 63)]),
}


@pytest.fixture(scope="module")
def vp():
    from paper_1204_3853_amd import vp as V
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    V.lib()
    return V


class Case:
    def __init__(self, vp, oracle, coarse, ratios, boxes, seed=0):
        ncx, ncv = coarse
        self.boxes, self.ratios = boxes, ratios
        f, veqs = I.hier_state(I.maxwellian, 0.0, X_LEN, V_LO, V_HI, 0.05, 0.5, coarse, ratios, boxes)
        f = f * (1 + 0.02 * np.random.default_rng(seed).random(f.size))
        self.f0 = f
        self.o = oracle.OracleHier(len(ratios) + 1, ncx, ncv, X_LEN, V_LO, V_HI, -1.0, ratios, boxes, veqs)
        self.spec = vp.hierarchy_spec(ncx, ncv, X_LEN, V_LO, V_HI, -1.0, ratios, veqs)
        self.plan = vp.Plan(self.spec, boxes=boxes)
        dxf = X_LEN / self.o.nfx
        dvf = 16.0 / self.o.nv[-1]
        self.dt = 0.4 / (V_HI / dxf + 0.2 / dvf)

    def gpu(self, x):
        return torch.tensor(x, dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module", params=list(LAYOUTS))
def case(request, vp, oracle):
    print(f"hierarchy layout {request.param}", flush=True)
    return Case(vp, oracle, **LAYOUTS[request.param])


def cmp(got, want, tol, what):
    got = got.detach().cpu().numpy() if hasattr(got, "detach") else got
    scale = max(np.abs(want).max(), 1e-300)
    err = np.abs(got - want).max()
    assert err <= tol * scale, f"{what}: max err {err:.3e} (rel {err / scale:.3e}) > {tol:.1e}"


def test_sizes(case):
    assert case.plan.state_elems == case.o.size
    for p in range(len(case.boxes)):
        assert case.plan.patch_offset(p) == case.o.offset(p)
    assert case.plan.config_elems == case.o.nfx
    assert case.plan.field_elems == case.o.field_elems


def test_reduce(vp, case):
    n = vp.reduce_moment(case.plan, case.gpu(case.f0))
    cmp(n, case.o.reduce_mask(case.f0), 1e-13, "n")


def test_constraints(vp, case):
    a = vp.field_of(case.plan, case.gpu(case.f0))
    a_o, _ = case.o.constraints(case.f0)
    cmp(a, a_o, 1e-11, "a")


def test_rhs(vp, case):
    a_o, _ = case.o.constraints(case.f0)
    k = vp.rhs(case.plan, case.gpu(case.f0), case.gpu(a_o))
    cmp(k, case.o.rhs(case.f0, a_o), 1e-12, "rhs")


def test_one_step(vp, case):
    f = case.gpu(case.f0)
    a = vp.field_of(case.plan, f)
    vp.rk4_step(case.plan, f, a, case.dt)
    want = case.o.step(case.f0, case.dt)
    cmp(f, want, 1e-12, "step")
    a_o, _ = case.o.constraints(want)
    cmp(a, a_o, 1e-11, "a after the step")


def test_several_steps(vp, case):
    f = case.gpu(case.f0)
    a = vp.field_of(case.plan, f)
    want = case.f0
    for s in range(4):
        vp.rk4_step(case.plan, f, a, case.dt)
        want = case.o.step(want, case.dt)
        cmp(f, want, 1e-12 * (s + 1), f"step {s + 1}")


def test_every_tile_shape(vp, case):
    ref = case.gpu(case.f0)
    a_ref = vp.field_of(case.plan, ref)
    vp.rk4_step(case.plan, ref, a_ref, case.dt)
    shapes = case.plan.tile_shapes()
    tried = 0
    for q, shp in enumerate(shapes):
        try:
            case.plan.set_tile_shape(q)
        except vp.VPError:
            assert shp[1] == 2
            continue
        f = case.gpu(case.f0)
        a = vp.field_of(case.plan, f)
        vp.rk4_step(case.plan, f, a, case.dt)
        cmp(f, ref.cpu().numpy(), 1e-14, f"shape {shp}")
        tried += 1
    case.plan.set_tile_shape(shapes.index((64, 1, 8)))
    assert tried >= 8


def test_graph_replay_matches_eager(vp, case):
    f_e = case.gpu(case.f0)
    a_e = vp.field_of(case.plan, f_e)
    f_g, a_g = f_e.clone(), a_e.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        vp.rk4_step(case.plan, f_g, a_g, case.dt)
    torch.cuda.current_stream().wait_stream(s)
    vp.rk4_step(case.plan, f_e, a_e, case.dt)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        vp.rk4_step(case.plan, f_g, a_g, case.dt)
    for r in range(3):
        g.replay()
        vp.rk4_step(case.plan, f_e, a_e, case.dt)
        torch.cuda.synchronize()
        assert torch.equal(f_g, f_e), f"replay {r}"
        assert torch.equal(a_g, a_e), f"replay {r}"


def test_unsupported_calls(vp, case):
    f = case.gpu(case.f0)
    a = vp.field_of(case.plan, f)
    with pytest.raises(vp.VPError, match="ENOTSUP"):
        vp.adjoint_step(case.plan, f, a, f.clone(), case.dt)
    with pytest.raises(vp.VPError, match="ENOTSUP"):
        case.plan.set_reduction(vp.REDUCE_MASK)
