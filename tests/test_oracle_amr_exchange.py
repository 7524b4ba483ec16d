"""Pins of the two-level oracle with touching patches (ghost cells for
inter-patch communication on a level, section 3; Alg. mspsc exchanges ghost
cells on each level before the right-hand side).

- Full coverage: level-1 patches that tile the whole fine domain (touching
  in x and v, and across the periodic x boundary) advance exactly like the
  uniform fine mesh, since every fine ghost is then a copy or a velocity
  ghost; the coarse level becomes the mean of the fine cells.
- Decomposition invariance: splitting a patch into two touching patches
  (in x or in v) leaves the step unchanged to rounding.
- Translation across the seam: shifting the data by a whole number of
  coarse cells so that a patch is cut by the periodic x boundary into two
  patches touching across it gives the shifted result.
Each fails if the ghost cells held by a neighbouring patch are interpolated
from the coarse level instead of copied.
"""
import math

import numpy as np
import pytest

import vp_inputs as I

X_LEN, V_LO, V_HI = 4 * math.pi, -8.0, 8.0


def make(oracle, boxes, ncx, ncv, R):
    veq_c = I.cell_average_1d(I.maxwellian, V_LO, V_HI, ncv, first=-2, count=ncv + 4)
    veq_f = I.cell_average_1d(I.maxwellian, V_LO, V_HI, ncv * R, first=-2, count=ncv * R + 4)
    o = oracle.OracleAMR(ncx, ncv, X_LEN, V_LO, V_HI, -1.0, R, boxes, veq_c, veq_f)
    return o, veq_c, veq_f


def box(x0, v0, x1, v1):
    return {"level": 1, "lo": [x0, v0], "hi": [x1, v1]}


def fine_field(ncx, ncv, R, seed, eps=0.05):
    """Exact cell averages of a perturbed Maxwellian on the fine mesh, times
    seeded noise (non-smooth content, so interpolation is never exact)."""
    nfx, nfv = ncx * R, ncv * R
    veq_f = I.cell_average_1d(I.maxwellian, V_LO, V_HI, nfv, first=-2, count=nfv + 4)
    xf = 1 + eps * I.cos_cell_average(0.0, X_LEN, nfx, 0.5)
    rng = np.random.default_rng(seed)
    return xf[:, None] * veq_f[None, 2:-2] * (1 + 0.02 * rng.random((nfx, nfv)))


def coarse_of(F, R):
    nfx, nfv = F.shape
    return F.reshape(nfx // R, R, nfv // R, R).mean(axis=(1, 3))


def pack(o, fc, F, boxes):
    parts = [fc.ravel()]
    for b in boxes:
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        parts.append(F[x0:x1 + 1, v0:v1 + 1].ravel())
    return np.concatenate(parts)


def unpack(o, f, boxes, shape):
    F = np.full(shape, np.nan)
    for p, b in enumerate(boxes):
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        nx, nv = x1 - x0 + 1, v1 - v0 + 1
        F[x0:x1 + 1, v0:v1 + 1] = f[o.offset(p): o.offset(p) + nx * nv].reshape(nx, nv)
    return F


@pytest.mark.parametrize("R", [2, 4])
def test_full_coverage_equals_uniform_fine(oracle, R):
    ncx, ncv = 8, 12
    nfx, nfv = ncx * R, ncv * R
    xs = [0, 3 * R, 5 * R, nfx]          # three columns of patches, two rows
    vs = [0, 7 * R, nfv]
    boxes = [box(xs[i], vs[j], xs[i + 1] - 1, vs[j + 1] - 1) for i in range(3) for j in range(2)]
    o, _, veq_f = make(oracle, boxes, ncx, ncv, R)
    F = fine_field(ncx, ncv, R, seed=3)
    f = pack(o, coarse_of(F, R), F, boxes)
    dt = 0.5 / (V_HI / (X_LEN / nfx) + 0.1 / (16.0 / nfv))
    g = o.step(f, dt)
    uni = oracle.Oracle1D(nfx, nfv, X_LEN, V_LO, V_HI, -1.0, np.array([veq_f[0], veq_f[1], veq_f[-2], veq_f[-1]]))
    Fu = uni.step(F, dt)
    Fg = unpack(o, g, boxes, (nfx, nfv))
    assert np.abs(Fg - Fu).max() <= 1e-13 * np.abs(Fu).max()
    gc = g[: ncx * ncv].reshape(ncx, ncv)
    np.testing.assert_allclose(gc, coarse_of(Fg, R), rtol=1e-14, atol=0)


@pytest.mark.parametrize("split", ["x", "v"])
def test_touching_split_is_invariant(oracle, split):
    ncx, ncv, R = 16, 24, 4
    whole = [box(16, 32, 47, 63), box(52, 20, 59, 27)]
    if split == "x":
        parts = [box(16, 32, 27, 63), box(28, 32, 47, 63), whole[1]]
    else:
        parts = [box(16, 32, 47, 43), box(16, 44, 47, 63), whole[1]]
    o1, _, _ = make(oracle, whole, ncx, ncv, R)
    o2, _, _ = make(oracle, parts, ncx, ncv, R)
    F = fine_field(ncx, ncv, R, seed=11)
    fc = coarse_of(F, R) * (1 + 0.01 * np.random.default_rng(4).random((ncx, ncv)))
    dt = 0.004
    g1 = o1.step(pack(o1, fc, F, whole), dt)
    g2 = o2.step(pack(o2, fc, F, parts), dt)
    shape = (ncx * R, ncv * R)
    F1, F2 = unpack(o1, g1, whole, shape), unpack(o2, g2, parts, shape)
    cov = ~np.isnan(F1)
    scale = np.abs(g1).max()
    assert np.abs(F1[cov] - F2[cov]).max() <= 1e-14 * scale
    np.testing.assert_allclose(g2[: ncx * ncv], g1[: ncx * ncv], rtol=0, atol=1e-14 * scale)
    assert np.abs(g1 - pack(o1, fc, F, whole)).max() > 1e-6       # the step did change the state


def test_translation_across_the_periodic_boundary(oracle):
    ncx, ncv, R = 16, 24, 2
    nfx = ncx * R
    boxes = [box(10, 12, 21, 33)]
    shift = 7                                    # coarse cells; the patch moves to fine [24, 35] -> wraps
    sf = shift * R
    cut = [box(24, 12, nfx - 1, 33), box(0, 12, 35 - nfx, 33)]
    o1, _, _ = make(oracle, boxes, ncx, ncv, R)
    o2, _, _ = make(oracle, cut, ncx, ncv, R)
    F = fine_field(ncx, ncv, R, seed=21)
    fc = coarse_of(F, R) * (1 + 0.01 * np.random.default_rng(6).random((ncx, ncv)))
    dt = 0.01
    g1 = o1.step(pack(o1, fc, F, boxes), dt)
    Fs, fcs = np.roll(F, sf, axis=0), np.roll(fc, shift, axis=0)
    g2 = o2.step(pack(o2, fcs, Fs, cut), dt)
    shape = (nfx, ncv * R)
    F1 = unpack(o1, g1, boxes, shape)
    F2 = np.roll(unpack(o2, g2, cut, shape), -sf, axis=0)
    cov = ~np.isnan(F1)
    scale = np.abs(g1).max()
    assert np.array_equal(cov, ~np.isnan(F2))
    assert np.abs(F1[cov] - F2[cov]).max() <= 1e-14 * scale
    c2 = np.roll(g2[: ncx * ncv].reshape(ncx, -1), -shift, axis=0).ravel()
    np.testing.assert_allclose(c2, g1[: ncx * ncv], rtol=0, atol=1e-14 * scale)
