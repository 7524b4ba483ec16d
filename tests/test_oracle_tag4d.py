"""Pins of the oracle's refinement criterion on 2D+2V meshes (section 3,
mesh refinement criteria: delta1 f + delta2 f, here summed over the four
directions x, y, vx, vy).

- a state that depends on (x, vx) only gives, at cells whose vy neighbours
  are interior, the 1D+1V criterion of that (x, vx) slice (an independent
  code path);
- on cell averages of a quadratic with a different curvature per direction
  the value has a closed form (first differences 4 c_d h_d (x_d - a_d),
  second differences 2 c_d h_d^2), which fixes each direction's weights;
- tags are the cells whose value exceeds the tolerance.
"""
import math

import numpy as np


def make(oracle, nx=6, ny=7, nvx=8, nvy=9, x_len=3.0, y_len=5.0, v_lo=-2.0, v_hi=2.5, veq_x=None, veq_y=None):
    veq_x = np.linspace(0.5, 1.5, nvx + 4) if veq_x is None else veq_x
    veq_y = np.linspace(0.7, 1.3, nvy + 4) if veq_y is None else veq_y
    return oracle.Oracle4D(nx, ny, nvx, nvy, x_len, y_len, v_lo, v_hi, -1.0, veq_x, veq_y)


def test_reduces_to_the_1d1v_criterion(oracle):
    nx, ny, nvx, nvy = 8, 5, 12, 7
    rng = np.random.default_rng(3)
    A = 1.0 + 0.3 * rng.random(nx)
    Bg = 0.2 + rng.random(nvx + 4)                   # equilibrium in vx with ghosts
    o = make(oracle, nx, ny, nvx, nvy, x_len=2.0, veq_x=Bg, veq_y=np.ones(nvy + 4))
    f2 = A[:, None] * Bg[None, 2:-2]
    f4 = np.broadcast_to(f2[:, None, :, None], (nx, ny, nvx, nvy)).copy()
    dx, dvx = 2.0 / nx, 4.5 / nvx
    want = oracle.tag_values(f2, dx, dvx, np.array([Bg[0], Bg[1], Bg[-2], Bg[-1]]))
    _, vals = o.tag(f4, 0.0)
    for l in range(1, nvy - 1):
        for j in range(ny):
            np.testing.assert_allclose(vals[:, j, :, l], want, rtol=1e-15, atol=0)


def test_closed_form_on_a_quadratic(oracle):
    nx, ny, nvx, nvy = 7, 6, 9, 8
    lens = (3.0, 5.0, 4.5, 4.5)
    lo = (0.0, 0.0, -2.0, -2.0)
    n = (nx, ny, nvx, nvy)
    h = [lens[d] / n[d] for d in range(4)]
    c = (1.0, 2.0, 3.0, 5.0)
    a = (1.1, 2.3, 0.4, -0.6)
    centres = [lo[d] + (np.arange(n[d]) + 0.5) * h[d] for d in range(4)]
    # cell averages of c_d (x_d - a_d)^2 summed over d
    parts = [c[d] * ((centres[d] - a[d]) ** 2 + h[d] ** 2 / 12.0) for d in range(4)]
    f = (parts[0][:, None, None, None] + parts[1][None, :, None, None] + parts[2][None, None, :, None]
         + parts[3][None, None, None, :])
    o = make(oracle, nx, ny, nvx, nvy)
    _, vals = o.tag(f, 0.0)
    for (i, j, k, l) in [(1, 1, 1, 1), (3, 2, 4, 5), (5, 4, 7, 6), (2, 3, 3, 2)]:
        idx = (i, j, k, l)
        g = [4.0 * c[d] * h[d] * (centres[d][idx[d]] - a[d]) for d in range(4)]
        d1 = math.sqrt(0.5 * sum(h[d] * g[d] ** 2 for d in range(4)))
        d2 = 0.5 * sum(h[d] ** 2 * 2.0 * c[d] * h[d] ** 2 for d in range(4))
        assert abs(vals[idx] - (d1 + d2)) < 1e-13 * (d1 + d2), (idx, vals[idx], d1 + d2)
        assert abs(o.tag_value(f, *idx) - vals[idx]) == 0.0


def test_tags_are_the_cells_above_tolerance(oracle):
    o = make(oracle)
    f = 1.0 + np.random.default_rng(4).random((6, 7, 8, 9))
    _, vals = o.tag(f, 0.0)
    for tol in np.quantile(vals, [0.2, 0.7]):
        tags, _ = o.tag(f, float(tol))
        assert np.array_equal(tags, (vals > tol).astype(np.uint8))
