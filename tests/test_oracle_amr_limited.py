"""Pins of the two-level oracle with limited face averages (section 2, eq.
limitedFace, on every patch of both levels; the paper's AMR runs of section
4 use them).

- Without patches the right-hand side is the single-level limited one
  (vpo_rhs_limited, which assembles the fluxes cell by cell and shares no
  code with the patch fluxes).
- Full coverage: patches tiling the fine domain (touching in x and v and
  across the periodic boundary) advance exactly like the single-level
  limited step on the fine mesh; the coarse level becomes the mean of the
  fine cells.
- Splitting a patch into two touching patches leaves the step unchanged;
  the composite mass is conserved over three steps.
- The limited and the centred hierarchies differ (the flag is honoured).
"""
import math

import numpy as np
import pytest

import vp_inputs as I
from test_oracle_amr_exchange import V_HI, V_LO, X_LEN, box, coarse_of, fine_field, make, pack, unpack


def test_no_patches_is_the_single_level_limited_operator(oracle):
    ncx, ncv = 16, 24
    o, veq_c, _ = make(oracle, [], ncx, ncv, 2)
    o.set_limited()
    rng = np.random.default_rng(1)
    fc = (1 + 0.3 * rng.random((ncx, ncv))) * veq_c[None, 2:-2]
    a = rng.normal(0.0, 0.2, ncx + 2 * ncx)
    k = o.rhs(fc.ravel(), a)
    vg = np.array([veq_c[0], veq_c[1], veq_c[-2], veq_c[-1]])
    want = oracle.rhs_limited(fc, a[:ncx], X_LEN / ncx, (V_HI - V_LO) / ncv, V_LO, vg)
    assert np.abs(k - want.ravel()).max() <= 1e-14 * np.abs(want).max()


@pytest.mark.parametrize("R", [2, 4])
def test_full_coverage_equals_single_level_limited_fine(oracle, R):
    ncx, ncv = 8, 12
    nfx, nfv = ncx * R, ncv * R
    xs = [0, 3 * R, 5 * R, nfx]
    vs = [0, 7 * R, nfv]
    boxes = [box(xs[i], vs[j], xs[i + 1] - 1, vs[j + 1] - 1) for i in range(3) for j in range(2)]
    o, _, veq_f = make(oracle, boxes, ncx, ncv, R)
    o.set_limited()
    F = fine_field(ncx, ncv, R, seed=13)
    f = pack(o, coarse_of(F, R), F, boxes)
    dt = 0.5 / (V_HI / (X_LEN / nfx) + 0.1 / (16.0 / nfv))
    g = o.step(f, dt)
    uni = oracle.Oracle1D(nfx, nfv, X_LEN, V_LO, V_HI, -1.0, np.array([veq_f[0], veq_f[1], veq_f[-2], veq_f[-1]]))
    Fu = uni.step_limited(F, dt)
    Fg = unpack(o, g, boxes, (nfx, nfv))
    assert np.abs(Fg - Fu).max() <= 1e-13 * np.abs(Fu).max()
    np.testing.assert_allclose(g[: ncx * ncv].reshape(ncx, ncv), coarse_of(Fg, R), rtol=1e-14, atol=0)
    # the centred step is a different one
    o2, _, _ = make(oracle, boxes, ncx, ncv, R)
    assert np.abs(unpack(o2, o2.step(f, dt), boxes, (nfx, nfv)) - Fg).max() > 1e-9


def test_split_invariance_and_composite_mass(oracle):
    ncx, ncv, R = 16, 24, 4
    whole = [box(16, 32, 47, 63), box(52, 20, 59, 27)]
    parts = [box(16, 32, 27, 63), box(28, 32, 47, 63), whole[1]]
    o1, _, _ = make(oracle, whole, ncx, ncv, R)
    o2, _, _ = make(oracle, parts, ncx, ncv, R)
    o1.set_limited()
    o2.set_limited()
    F = fine_field(ncx, ncv, R, seed=17)
    fc = coarse_of(F, R) * (1 + 0.01 * np.random.default_rng(9).random((ncx, ncv)))
    dt = 0.004
    f1 = pack(o1, fc, F, whole)
    g1 = o1.step(f1, dt)
    g2 = o2.step(pack(o2, fc, F, parts), dt)
    shape = (ncx * R, ncv * R)
    F1, F2 = unpack(o1, g1, whole, shape), unpack(o2, g2, parts, shape)
    cov = ~np.isnan(F1)
    scale = np.abs(g1).max()
    assert np.abs(F1[cov] - F2[cov]).max() <= 1e-14 * scale
    np.testing.assert_allclose(g2[: ncx * ncv], g1[: ncx * ncv], rtol=0, atol=1e-14 * scale)

    dxc, dvc = X_LEN / ncx, (V_HI - V_LO) / ncv

    def mass(f):
        fcm = f[: ncx * ncv].reshape(ncx, ncv)
        c = np.zeros((ncx, ncv), bool)
        m = 0.0
        for p, b in enumerate(whole):
            (x0, v0), (x1, v1) = b["lo"], b["hi"]
            c[x0 // R:(x1 + 1) // R, v0 // R:(v1 + 1) // R] = True
            m += f[o1.offset(p): o1.offset(p) + (x1 - x0 + 1) * (v1 - v0 + 1)].sum() * dxc * dvc / R / R
        return m + fcm[~c].sum() * dxc * dvc

    g = f1
    for _ in range(3):
        g = o1.step(g, dt)
    assert abs(mass(g) - mass(f1)) <= 1e-13 * mass(f1)
    assert np.abs(g - f1).max() > 1e-6
