"""Pins of the two-level AMR oracle.

- The sub-cell interpolation weights b_j(s) of section 3 (with the
  corrected p_k and gamma_1 readings) conserve the coarse average, form a
  partition of unity, and reproduce exact fine averages of quartics; the
  formulas as printed do not (shown, so the readings are pinned).
- Reduction bookkeeping: a hierarchy whose patches carry the conservative
  interpolation of the coarse data reduces to the same charge density as
  the coarse level alone (Mask Reduction invariance).
- Composite mass is conserved by the multi-level step (flux coarsening
  and restriction), to round-off.
- Fine patches converge to a uniform fine-mesh computation at high order
  when the whole hierarchy is refined.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from numpy.polynomial import Polynomial

import vp_inputs as I


@pytest.mark.parametrize("R", [2, 4])
def test_interp_weights_conservation_and_partition(oracle, R):
    B = oracle.interp_weights(R)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(B.sum(axis=0) / R, [0, 0, 1, 0, 0], atol=1e-15)


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_interp_weights_quartic_exactness(oracle, deg):
    """Coarse cell averages of x^deg on cells [i, i+1] -> the weights give the
    exact averages over the R sub-cells."""
    R = 4
    B = oracle.interp_weights(R)
    P = Polynomial([0] * deg + [1]).integ()
    i = 3
    cavg = np.array([P(i + j + 1) - P(i + j) for j in range(-2, 3)])
    for s in range(R):
        lo, hi = i + s / R, i + (s + 1) / R
        exact = (P(hi) - P(lo)) * R
        assert abs(B[s] @ cavg - exact) <= 1e-12 * max(1.0, abs(exact))


def test_printed_formulas_break_conservation():
    """p_k(s) = sum_j C(k, j) s^j as printed gives sum_s b_0(s)/R != 1."""
    R = 4

    def b0(p):
        return (6 * p[4] - 15 * p[3] - 40 * p[2] + 75 * p[1] + 94) / Fraction(120)

    printed = []
    for s in range(R):
        p = [Fraction(1)] + [sum(Fraction(math.comb(k, j)) * s ** j for j in range(k + 1)) for k in range(1, 5)]
        printed.append(b0(p))
    assert sum(printed) / R != 1


def small_layout():
    boxes = [{"level": 1, "lo": [16, 40], "hi": [39, 63]}, {"level": 1, "lo": [60, 68], "hi": [83, 87]},
             {"level": 1, "lo": [0, 96], "hi": [15, 111]}]
    return boxes


def make_oracle(oracle, boxes, ncx=32, ncv=48, R=4):
    veq_c = I.cell_average_1d(I.maxwellian, -8.0, 8.0, ncv, first=-2, count=ncv + 4)
    veq_f = I.cell_average_1d(I.maxwellian, -8.0, 8.0, ncv * R, first=-2, count=ncv * R + 4)
    return oracle.OracleAMR(ncx, ncv, 4 * math.pi, -8.0, 8.0, -1.0, R, boxes, veq_c, veq_f), veq_c, veq_f


def test_reduction_invariant_under_interpolated_refinement(oracle):
    boxes = small_layout()
    o, veq_c, veq_f = make_oracle(oracle, boxes)
    o0, _, _ = make_oracle(oracle, [])
    rng = np.random.default_rng(2)
    fc = (1 + 0.1 * rng.random((32, 48))) * veq_c[None, 2:-2]
    # patch interiors hold the x-then-v sub-cell interpolation of the coarse level
    B = oracle.interp_weights(4)
    parts = [fc.ravel()]
    for b in boxes:
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        vals = np.empty((x1 - x0 + 1, v1 - v0 + 1))
        for X in range(x0, x1 + 1):
            ci, s = divmod(X, 4)
            gx = np.array([sum(B[s, a + 2] * fc[(ci + a) % 32, cj] for a in range(-2, 3)) for cj in range(48)])
            for V in range(v0, v1 + 1):
                cj, t = divmod(V, 4)
                vals[X - x0, V - v0] = sum(B[t, bb + 2] * gx[cj + bb] for bb in range(-2, 3))
        parts.append(vals.ravel())
    f = np.concatenate(parts)
    n_h = o.reduce_mask(f)
    n_0 = o0.reduce_mask(fc.ravel())
    np.testing.assert_allclose(n_h, n_0, rtol=1e-14, atol=1e-15)


def test_ghost_fill_matches_interpolation(oracle):
    """Ghost cells of a patch hold the sub-cell interpolation of the coarse
    level (x periodic): equal to the values a patch covering them would get."""
    boxes = small_layout()
    o, veq_c, _ = make_oracle(oracle, boxes)
    rng = np.random.default_rng(5)
    fc = rng.random((32, 48))
    f = np.concatenate([fc.ravel()] + [rng.random((b["hi"][0] - b["lo"][0] + 1) * (b["hi"][1] - b["lo"][1] + 1))
                                       for b in boxes])
    g = o.ghosted_patch(f, 2)        # the patch at x = 0: its lower ghosts wrap around
    B = oracle.interp_weights(4)
    X, V = -1, 96 - 2                # ghost cell (row -1, column -2) in global fine indices
    ci, s = divmod(X, 4)
    cj, t = divmod(V, 4)
    val = sum(B[t, bb + 2] * sum(B[s, a + 2] * fc[(ci + a) % 32, cj + bb] for a in range(-2, 3))
              for bb in range(-2, 3))
    assert abs(g[X + 2, V - 96 + 2] - val) < 1e-14


def composite_mass(o, f, boxes, dxc, dvc, R=4):
    ncx, ncv = o.ncx, o.ncv
    fc = f[: ncx * ncv].reshape(ncx, ncv)
    cov = np.zeros((ncx, ncv), bool)
    m = 0.0
    for p, b in enumerate(boxes):
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        cov[x0 // R:(x1 + 1) // R, v0 // R:(v1 + 1) // R] = True
        m += f[o.offset(p): o.offset(p) + (x1 - x0 + 1) * (v1 - v0 + 1)].sum() * dxc * dvc / R / R
    return m + fc[~cov].sum() * dxc * dvc


def test_amr_step_conserves_composite_mass(oracle):
    boxes = small_layout()
    o, veq_c, veq_f = make_oracle(oracle, boxes)
    rng = np.random.default_rng(8)
    ncx, ncv = 32, 48
    dxc, dvc = 4 * math.pi / ncx, 16.0 / ncv
    xc = 1 + 0.05 * I.cos_cell_average(0, 4 * math.pi, ncx, 0.5)
    xf = 1 + 0.05 * I.cos_cell_average(0, 4 * math.pi, ncx * 4, 0.5)
    parts = [(xc[:, None] * veq_c[None, 2:-2]).ravel()]
    for b in boxes:
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        parts.append((xf[x0:x1 + 1, None] * veq_f[None, 2 + v0:2 + v1 + 1] * (1 + 0.01 * rng.random((x1 - x0 + 1, v1 - v0 + 1)))).ravel())
    f = np.concatenate(parts)
    m0 = composite_mass(o, f, boxes, dxc, dvc)
    g = f
    for _ in range(3):
        g = o.step(g, 0.02)
    m1 = composite_mass(o, g, boxes, dxc, dvc)
    assert abs(m1 - m0) < 1e-13 * m0, (m0, m1)
    assert np.abs(g - f).max() > 1e-6      # the state did change


def amr_vs_uniform_error(oracle, scale, T=0.4):
    """max |AMR fine patch - uniform fine run| after time T for the small
    layout refined by `scale` (coarse 32 scale x 48 scale, ratio 4)."""
    boxes = [{"level": 1, "lo": [b["lo"][0] * scale, b["lo"][1] * scale],
              "hi": [b["hi"][0] * scale + scale - 1, b["hi"][1] * scale + scale - 1]} for b in small_layout()]
    ncx, ncv, R = 32 * scale, 48 * scale, 4
    o, veq_c, veq_f = make_oracle(oracle, boxes, ncx, ncv, R)
    xc = 1 + 0.05 * I.cos_cell_average(0, 4 * math.pi, ncx, 0.5)
    xf = 1 + 0.05 * I.cos_cell_average(0, 4 * math.pi, ncx * R, 0.5)
    parts = [(xc[:, None] * veq_c[None, 2:-2]).ravel()]
    for b in boxes:
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        parts.append((xf[x0:x1 + 1, None] * veq_f[None, 2 + v0:2 + v1 + 1]).ravel())
    f = np.concatenate(parts)
    pf = I.Problem1D(ncx * R, ncv * R, 0.0, 4 * math.pi, -8.0, 8.0, eps=0.05, k=0.5)
    of = oracle.Oracle1D.from_problem(pf)
    ff = pf.initial_state()
    nsteps = int(math.ceil(T / (0.5 / (8.0 / pf.dx + 0.05 / pf.dv))))
    dt = T / nsteps
    for _ in range(nsteps):
        f = o.step(f, dt)
        ff = of.step(ff, dt)
    err = 0.0
    for p, b in enumerate(boxes):
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        nxp, nvp = x1 - x0 + 1, v1 - v0 + 1
        fp = f[o.offset(p): o.offset(p) + nxp * nvp].reshape(nxp, nvp)
        err = max(err, np.abs(fp - ff[x0:x1 + 1, v0:v1 + 1]).max())
    return err


@pytest.mark.slow
def test_amr_converges_to_uniform_fine(oracle):
    """Refining the whole hierarchy by 2 reduces the AMR-vs-uniform-fine
    difference on the patches at high order (it is set by the coarse-fine
    ghost interpolation and the coarse truncation error)."""
    e1 = amr_vs_uniform_error(oracle, 1)
    e2 = amr_vs_uniform_error(oracle, 2)
    assert e1 / e2 > 12.0, (e1, e2)
