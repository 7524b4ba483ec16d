"""GPU parity of the regridding of a multi-level hierarchy (criterion on
every level, clustering nested in the level below, level-by-level state
transfer; section 3) and of an adaptive run on four levels with the
section-4 ratios [2,4], [4,2], [2,2] followed step by step by the oracle.

Tolerances: criterion values 1e-13 relative (tags compared where the value
is more than 1e-9 tol away from tol: the ghost interpolation rounds
differently), transferred states 1e-12, the run's state 1e-10 of max|f|
after every block of steps (errors of 1e-12 per step accumulate), time and
step 1e-12.
"""
import math

import numpy as np
import pytest

import vp_inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

X_LEN, V_LO, V_HI = 4 * math.pi, -8.0, 8.0
RATIOS3 = [(2, 4), (4, 2)]


def box(level, x0, v0, x1, v1):
    return {"level": level, "lo": [x0, v0], "hi": [x1, v1]}


HIER3 = [box(1, 8, 24, 31, 71), box(1, 32, 24, 43, 71), box(1, 0, 32, 7, 55), box(1, 56, 40, 63, 55),
         box(2, 56, 64, 119, 119), box(2, 120, 64, 143, 119), box(2, 240, 88, 255, 95)]


@pytest.fixture(scope="module")
def vp():
    from paper_1204_3853_amd import vp as V
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    V.lib()
    return V


def setup(vp, oracle, boxes, seed=5, coarse=(32, 24), ratios=RATIOS3):
    f, veqs = I.hier_state(I.maxwellian, 0.0, X_LEN, V_LO, V_HI, 0.05, 0.5, coarse, ratios, boxes)
    f = f * (1 + 0.02 * np.random.default_rng(seed).random(f.size))
    o = oracle.OracleHier(len(ratios) + 1, coarse[0], coarse[1], X_LEN, V_LO, V_HI, -1.0, ratios, boxes, veqs)
    spec = vp.hierarchy_spec(coarse[0], coarse[1], X_LEN, V_LO, V_HI, -1.0, ratios, veqs)
    plan = vp.Plan(spec, boxes=boxes)
    return o, plan, f, veqs, spec


@pytest.mark.parametrize("level", [0, 1, 2])
def test_tag_level(vp, oracle, level):
    o, plan, f, _, _ = setup(vp, oracle, HIER3)
    want = o.tag_values(f, level)
    held = ~np.isnan(want)
    tol = float(np.median(want[held]))
    tags, vals = vp.tag_level(plan, torch.tensor(f, device="cuda"), level, tol, values=True)
    got = vals.cpu().numpy()
    assert np.array_equal(np.isnan(got), ~held)
    assert np.abs(got[held] - want[held]).max() <= 1e-13 * np.abs(want[held]).max()
    t = tags.cpu().numpy().astype(bool)
    sure = held & (np.abs(want - tol) > 1e-9 * tol)
    assert np.array_equal(t[sure], (want > tol)[sure])
    assert not t[~held].any()


def test_transfer(vp, oracle):
    o, plan, f, veqs, spec = setup(vp, oracle, HIER3, seed=3)
    new_boxes = [box(1, 8, 24, 43, 71), box(1, 0, 32, 7, 55), box(1, 56, 32, 63, 63),
                 box(2, 60, 60, 131, 119), box(2, 240, 88, 255, 95)]
    n = oracle.OracleHier(3, 32, 24, X_LEN, V_LO, V_HI, -1.0, RATIOS3, new_boxes, veqs)
    want = oracle.hier_regrid_transfer(o, f, n)
    new_plan = vp.Plan(spec, boxes=new_boxes)
    got = vp.regrid_transfer(plan, torch.tensor(f, device="cuda"), new_plan)
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    assert np.abs(g - want).max() <= 1e-12 * np.abs(want).max()


def test_cluster_level_nests_and_covers(vp, oracle):
    o, plan, f, veqs, spec = setup(vp, oracle, HIER3, seed=6)
    vals = o.tag_values(f, 1)
    held = ~np.isnan(vals)
    tol = float(np.quantile(vals[held], 0.7))
    tags = np.nan_to_num(vals, nan=0.0) > tol
    boxes2 = vp.cluster_level(plan, 1, tags.astype(np.uint8), RATIOS3[1], efficiency=0.7, min_width=2, buffer=1,
                              max_size=(64, 64))
    assert boxes2
    # nested with room for ghost interpolation: the oracle accepts the hierarchy
    lvl1 = [b for b in HIER3 if b["level"] == 1]
    oracle.OracleHier(3, 32, 24, X_LEN, V_LO, V_HI, -1.0, RATIOS3, lvl1 + boxes2, veqs)
    cov = np.zeros(tags.shape, bool)
    for b in boxes2:
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        assert x0 % 4 == 0 and v0 % 2 == 0 and (x1 + 1) % 4 == 0 and (v1 + 1) % 2 == 0
        assert x1 - x0 + 1 <= 64 and v1 - v0 + 1 <= 64
        c = (slice(x0 // 4, (x1 + 1) // 4), slice(v0 // 2, (v1 + 1) // 2))
        assert not cov[c].any()
        cov[c] = True
    # every tagged cell that nesting allows is covered (allowed: held with every cell within 3 held)
    nx, nv = tags.shape
    allowed = np.zeros_like(held)
    for i in range(nx):
        for j in range(nv):
            ok = True
            for a in range(-3, 4):
                for c in range(-3, 4):
                    jj = j + c
                    if 0 <= jj < nv and not held[(i + a) % nx, jj]:
                        ok = False
            allowed[i, j] = ok
    assert not (tags & allowed & ~cov).any()


BUMP_RATIOS = [(2, 4), (4, 2), (2, 2)]


def test_adaptive_four_level_run_followed_by_oracle(vp, oracle):
    """Bump-on-tail (section 4): level 0 16 x 32, ratios [2,4], [4,2],
    [2,2], the initial refinement [(0,8),(15,24)] on level 1, tol 0.01,
    AMR1's regrid interval 2, tag buffer 1 and patch size limits; six
    blocks of two steps.  After every block the GPU state equals the
    oracle's, which steps with its own time step and takes the run's new
    boxes (checked: level 1 covers every tagged level-0 cell, and the
    hierarchy is nested)."""
    coarse = (16, 32)
    b0 = [box(1, 0, 32, 31, 99)]
    f0, veqs = I.hier_state(I.bump_on_tail_profile, I.BUMP_X_LO, I.BUMP_X_LEN, I.BUMP_V_LO, I.BUMP_V_HI, 0.04, 0.3,
                            coarse, BUMP_RATIOS, b0)
    spec = vp.hierarchy_spec(coarse[0], coarse[1], I.BUMP_X_LEN, I.BUMP_V_LO, I.BUMP_V_HI, -1.0, BUMP_RATIOS, veqs,
                             x_lo=I.BUMP_X_LO)
    tol = 0.01
    run = vp.AmrRun(spec, b0, torch.tensor(f0, device="cuda"), tol, 2, efficiency=0.7, min_width=2, buffer=1,
                    cfl=0.5, dt_growth=1.1, dt_initial=0.01, max_size=[(32, 32), (64, 64), (64, 64), (64, 64)])

    def mk(boxes):
        return oracle.OracleHier(4, coarse[0], coarse[1], I.BUMP_X_LEN, I.BUMP_V_LO, I.BUMP_V_HI, -1.0, BUMP_RATIOS,
                                 boxes, veqs)

    o, f, boxes = mk(b0), f0, b0
    t, dt, steps = 0.0, None, 0
    deepest = 1
    for blk in range(6):
        print(f"block {blk}: {len(boxes)} boxes", flush=True)
        for _ in range(2):
            a, _ = o.constraints(f)
            lim = oracle.hier_stability_limit(o, a, I.BUMP_V_LO, I.BUMP_V_HI)
            dt = min(0.01 if dt is None else 1.1 * dt, 0.5 * lim)
            f = o.step(f, dt)
            t += dt
            steps += 1
        vals0 = o.tag_values(f, 0)
        run.advance(2)
        info = run.info()
        assert info["steps"] == steps
        assert abs(info["t"] - t) <= 1e-12 * t
        new_boxes = run.boxes()
        deepest = max([deepest] + [b["level"] for b in new_boxes])
        n = mk(new_boxes)                                  # raises unless nested
        cov = np.zeros(vals0.shape, bool)
        for b in new_boxes:
            if b["level"] == 1:
                cov[b["lo"][0] // 2:(b["hi"][0] + 1) // 2, b["lo"][1] // 4:(b["hi"][1] + 1) // 4] = True
        sure = (vals0 > tol) & (np.abs(vals0 - tol) > 1e-9 * tol)
        assert not (sure & ~cov).any()
        f = oracle.hier_regrid_transfer(o, f, n)
        o, boxes = n, new_boxes
        got = run.state().cpu().numpy()
        assert got.size == f.size
        assert np.abs(got - f).max() <= 1e-10 * np.abs(f).max(), f"block {blk}"
    assert deepest >= 2
