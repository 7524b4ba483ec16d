"""Pins of the two-level 2D+2V oracle (oracle/vp_oracle_amr4d.c).

- Without patches its right-hand side is the single-level 2D+2V one and
  its charge density the refined single-level moment.
- Full coverage: patches tiling the whole fine domain (touching, across
  the periodic boundaries) advance exactly like the single-level oracle on
  the fine mesh; level 0 becomes the mean of its fine cells.
- Ghost cells: with exact cell averages of a product of quartics in x, y,
  vx and vy, every ghost cell the tensor sub-cell interpolation fills is
  the exact fine cell average.
- Reduction: a patch holding the tensor interpolation of level 0 leaves the
  charge density unchanged.
- Splitting a patch into two touching patches leaves the step unchanged;
  composite mass is conserved.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import Polynomial

import vp_inputs as I

X_LEN = Y_LEN = 4 * math.pi
V_LO, V_HI = -6.0, 6.0


def box(lo, hi):
    return {"level": 1, "lo": list(lo), "hi": list(hi)}


def make(oracle, ncells, R, boxes, noise=0.02, seed=0, v=(V_LO, V_HI)):
    f, gxc, gyc, gxf, gyf = I.amr4d_state(ncells, R, boxes, eps=0.05, v_lo=v[0], v_hi=v[1])
    f = f * (1 + noise * np.random.default_rng(seed).random(f.size))
    o = oracle.OracleAMR4D(ncells, X_LEN, Y_LEN, v[0], v[1], -1.0, R, boxes, gxc, gyc, gxf, gyf)
    return o, f, (gxc, gyc, gxf, gyf)


def test_no_patches_is_the_single_level_operator(oracle):
    """Without patches the right-hand side is the single-level 2D+2V one, and
    the charge density on the fine configuration mesh is the tensor sub-cell
    refinement of the single-level moment (the field itself is solved on the
    fine mesh, so the step is not the single-level step)."""
    n, R = (4, 4, 6, 6), 2
    o, f, (gxc, gyc, _, _) = make(oracle, n, R, [])
    s = oracle.Oracle4D(*n, X_LEN, Y_LEN, V_LO, V_HI, -1.0, gxc, gyc)
    a = np.random.default_rng(2).normal(0.0, 0.1, 2 * (16 + 64))
    k = o.rhs(f, a)
    want = s.rhs(f.reshape(n), a[: 2 * 16]).ravel()
    assert np.abs(k - want).max() <= 1e-14 * np.abs(want).max()
    nc = s.moment(f.reshape(n)).reshape(n[0], n[1])
    B = oracle.interp_weights(R)
    nf = np.empty((n[0] * R, n[1] * R))
    for I in range(n[0] * R):
        for J in range(n[1] * R):
            i, si, j, sj = I // R, I % R, J // R, J % R
            nf[I, J] = sum(B[sj, b + 2] * sum(B[si, a2 + 2] * nc[(i + a2) % n[0], (j + b) % n[1]] for a2 in range(-2, 3))
                           for b in range(-2, 3))
    np.testing.assert_allclose(o.reduce_mask(f), nf.ravel(), rtol=1e-13, atol=0)


def test_full_coverage_is_the_fine_single_level_oracle(oracle):
    n, R = (4, 4, 6, 6), 2
    nf = tuple(c * R for c in n)
    cuts = [(0, 4, 8), (0, 8), (0, 6, 12), (0, 12)]          # x and vx split: four touching patches
    boxes = []
    for a in range(len(cuts[0]) - 1):
        for c in range(len(cuts[2]) - 1):
            boxes.append(box((cuts[0][a], 0, cuts[2][c], 0),
                             (cuts[0][a + 1] - 1, nf[1] - 1, cuts[2][c + 1] - 1, nf[3] - 1)))
    fine = I.Problem2D(*nf, eps=0.05).initial_state()
    fine = fine * (1 + 0.02 * np.random.default_rng(3).random(fine.shape))
    coarse = fine.reshape(n[0], R, n[1], R, n[2], R, n[3], R).mean(axis=(1, 3, 5, 7))
    parts = [coarse.ravel()]
    for b in boxes:
        parts.append(fine[tuple(slice(b["lo"][d], b["hi"][d] + 1) for d in range(4))].ravel())
    f = np.concatenate(parts)
    _, gxc, gyc, gxf, gyf = I.amr4d_state(n, R, [], eps=0.05)
    o = oracle.OracleAMR4D(n, X_LEN, Y_LEN, V_LO, V_HI, -1.0, R, boxes, gxc, gyc, gxf, gyf)
    s = oracle.Oracle4D(*nf, X_LEN, Y_LEN, V_LO, V_HI, -1.0, gxf, gyf)
    dt = 0.03
    g = o.step(f, dt)
    want = s.step(fine, dt)
    got = np.empty(nf)
    for p, b in enumerate(boxes):
        got[tuple(slice(b["lo"][d], b["hi"][d] + 1) for d in range(4))] = o.patch(g, p)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    np.testing.assert_allclose(o.patch(g, -1), got.reshape(n[0], R, n[1], R, n[2], R, n[3], R).mean(axis=(1, 3, 5, 7)),
                               rtol=1e-13, atol=0)


PX = [Polynomial([1.0, 0.2, -0.03, 0.002, -0.0001]), Polynomial([2.0, -0.1, 0.04, -0.003, 0.0002]),
      Polynomial([1.5, 0.3, 0.05, -0.004, 0.0003]), Polynomial([0.7, -0.2, 0.06, 0.005, -0.0004])]


def poly_avgs(shape, lo_edges, h):
    vals = []
    for d in range(4):
        P = PX[d].integ()
        e = lo_edges[d] + np.arange(shape[d] + 1) * h[d]
        vals.append((P(e[1:]) - P(e[:-1])) / h[d])
    return np.einsum("i,j,k,l->ijkl", *vals)


def test_ghost_cells_exact_for_quartics(oracle):
    """Level 0 of 10^4 unit cells on [0, 10)^2 x [-5, 5)^2, R = 2, one patch
    over coarse cells 4..5 in every direction: every ghost cell (all are
    interpolated: no other patch, inside the velocity box) is the exact
    fine average of the product of quartics."""
    n, R = (10, 10, 10, 10), 2
    b = box((8, 8, 8, 8), (11, 11, 11, 11))
    coarse = poly_avgs(n, (0.0, 0.0, -5.0, -5.0), (1.0, 1.0, 1.0, 1.0))
    fine = poly_avgs(tuple(c * R for c in n), (0.0, 0.0, -5.0, -5.0), (0.5, 0.5, 0.5, 0.5))
    f = np.concatenate([coarse.ravel(), fine[8:12, 8:12, 8:12, 8:12].ravel()])
    z = [np.zeros(n[2] + 4), np.zeros(n[3] + 4), np.zeros(2 * n[2] + 4), np.zeros(2 * n[3] + 4)]
    o = oracle.OracleAMR4D(n, 10.0, 10.0, -5.0, 5.0, -1.0, R, [b], *z)
    g = o.ghosted(f, 0)
    want = fine[6:14, 6:14, 6:14, 6:14]
    assert np.abs(g - want).max() <= 1e-12 * np.abs(want).max()


def interp4(oracle, coarse, R, lo, hi):
    """The tensor sub-cell interpolation of a (periodic in x, y) coarse array
    onto the fine box [lo, hi] (velocity stencils stay inside)."""
    B = oracle.interp_weights(R)
    n = coarse.shape
    out = np.empty(tuple(hi[d] - lo[d] + 1 for d in range(4)))
    for idx in np.ndindex(out.shape):
        X = [lo[d] + idx[d] for d in range(4)]
        c = [x // R for x in X]
        s = [x % R for x in X]
        acc = 0.0
        for dd in range(-2, 3):
            av = 0.0
            for e in range(-2, 3):
                ay = 0.0
                for bb in range(-2, 3):
                    ax = sum(B[s[0], a + 2] * coarse[(c[0] + a) % n[0], (c[1] + bb) % n[1], c[2] + e, c[3] + dd]
                             for a in range(-2, 3))
                    ay += B[s[1], bb + 2] * ax
                av += B[s[2], e + 2] * ay
            acc += B[s[3], dd + 2] * av
        out[idx] = acc
    return out


def test_reduction_invariant_under_interpolated_refinement(oracle):
    n, R = (4, 4, 8, 8), 2
    o0, f0, gs = make(oracle, n, R, [], seed=4)
    b = box((2, 0, 4, 6), (5, 7, 11, 9))
    d = interp4(oracle, f0.reshape(n), R, b["lo"], b["hi"])
    o1 = oracle.OracleAMR4D(n, X_LEN, Y_LEN, V_LO, V_HI, -1.0, R, [b], *gs)
    np.testing.assert_allclose(o1.reduce_mask(np.concatenate([f0, d.ravel()])), o0.reduce_mask(f0),
                               rtol=1e-13, atol=1e-15)


def composite_mass(o, f, vspan):
    n, R = o.n, o.R
    hc = [X_LEN / n[0], Y_LEN / n[1], vspan / n[2], vspan / n[3]]
    vol_c = np.prod(hc)
    cov = np.zeros(n, bool)
    m = 0.0
    for p, b in enumerate(o.boxes):
        cov[tuple(slice(b["lo"][d] // R, (b["hi"][d] + 1) // R) for d in range(4))] = True
        m += o.patch(f, p).sum() * vol_c / R ** 4
    return m + o.patch(f, -1)[~cov].sum() * vol_c


SPLIT = [box((2, 2, 4, 4), (5, 5, 9, 7))]
SPLIT2 = [box((2, 2, 4, 4), (5, 3, 9, 7)), box((2, 4, 4, 4), (5, 5, 9, 7))]


def test_split_invariance_and_mass(oracle):
    n, R = (4, 4, 6, 6), 2
    o1, f1, gs = make(oracle, n, R, SPLIT, seed=7)
    o2 = oracle.OracleAMR4D(n, X_LEN, Y_LEN, V_LO, V_HI, -1.0, R, SPLIT2, *gs)
    whole = o1.patch(f1, 0)
    f2 = np.concatenate([f1[: o1.offset(0)], whole[:, 0:2].ravel(), whole[:, 2:4].ravel()])
    dt = 0.03
    g1, g2 = o1.step(f1, dt), o2.step(f2, dt)
    scale = np.abs(g1).max()
    assert np.abs(g1[: o1.offset(0)] - g2[: o2.offset(0)]).max() <= 1e-14 * scale
    w2 = np.concatenate([o2.patch(g2, 0), o2.patch(g2, 1)], axis=1)
    assert np.abs(o1.patch(g1, 0) - w2).max() <= 1e-14 * scale
    assert np.abs(g1 - f1).max() > 1e-6


def test_composite_mass_is_conserved(oracle):
    """Velocity box [-14, 14]^2 on 12 cells: the face averages next to the
    velocity boundary read f at |v| > 9, so no mass crosses it to within
    rounding; two steps with a patch and with it split in two."""
    n, R = (4, 4, 12, 12), 2
    for boxes in ([box((2, 2, 8, 8), (5, 5, 15, 13))],
                  [box((2, 2, 8, 8), (5, 3, 15, 13)), box((2, 4, 8, 8), (5, 5, 15, 13))]):
        o, f, _ = make(oracle, n, R, boxes, seed=8, v=(-14.0, 14.0))
        m0 = composite_mass(o, f, 28.0)
        g = o.step(o.step(f, 0.02), 0.02)
        assert abs(composite_mass(o, g, 28.0) - m0) <= 1e-13 * m0
        assert np.abs(g - f).max() > 1e-4
