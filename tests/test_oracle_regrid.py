"""Pins of the regridding pieces of section 3 in the oracle.

Conservative, limited, high-order interpolation (eqs. aux1, aux2,
interp_r_avg, renormalisation):
- fine averages agree with a derivation from the definitions: for each of
  the three candidates, the quadratic with the given cell averages on its
  three-cell stencil averaged over the sub-cells; Jiang-Shu smoothness as
  the integral of p'^2 + p''^2 over the coarse cell; weights
  d_r / (eps + beta_r)^2 normalised.  This fixes the reading of the
  printed B^(0) (the printed 2 D_i - D_{i-1} fails it);
- exact conservation of every coarse cell average (1D and the 2D tensor
  form), exactness for quadratics (every candidate is quadratic);
- next to a step the interpolation takes the smooth stencil (no
  overshoot), where fixed ideal weights overshoot.

Refinement criterion delta1 f + delta2 f > tol:
- closed forms for linear and quadratic data and the powers of the mesh
  spacing the estimates carry (delta1 ~ h^(3/2) for fixed slopes, delta2
  ~ h^4 for fixed curvature), translation covariance in periodic x,
  reflection symmetry, zero for a constant field with matching ghosts.
"""
import numpy as np
import pytest
from numpy.polynomial import Polynomial


def definition_prolong(u, R, eps=1e-6):
    d = [0.3, 0.6, 0.1]
    fine = np.zeros(R)
    alphas, cands = [], []
    for r in range(3):
        cells = [(k - r, k - r + 1) for k in range(3)]           # xi intervals, cell i = [0, 1]
        avgs = [u[2 - r + k] for k in range(3)]
        A = np.array([[1.0, (b * b - a * a) / 2.0, (b ** 3 - a ** 3) / 3.0] for a, b in cells])
        p = Polynomial(np.linalg.solve(A, avgs))
        P = p.integ()
        cands.append(np.array([(P((s + 1) / R) - P(s / R)) * R for s in range(R)]))
        s1 = (p.deriv() ** 2).integ()
        s2 = (p.deriv(2) ** 2).integ()
        beta = (s1(1) - s1(0)) + (s2(1) - s2(0))
        alphas.append(d[r] / (eps + beta) ** 2)
    w = np.array(alphas) / sum(alphas)
    for r in range(3):
        fine += w[r] * cands[r]
    return fine


@pytest.mark.parametrize("R", [2, 4])
def test_prolong_matches_definition(oracle, R):
    rng = np.random.default_rng(21)
    for _ in range(200):
        u = rng.standard_normal(5) * rng.choice([1e-2, 1.0, 10.0])
        got = oracle.prolong1d(u, R)
        want = definition_prolong(u, R)
        assert np.abs(got - want).max() <= 1e-11 * max(1.0, np.abs(u).max()), (u, got, want)


def test_printed_b0_fails_the_definition(oracle):
    """The printed B^(0) = 2 D_i - D_{i-1} is not the quadratic's slope on cells i, i+1, i+2."""
    u = np.array([0.0, 1.0, 0.5, 3.0, 2.0])
    D = np.diff(u)
    b_printed = 2 * D[2] - D[1]
    b_def = 2 * D[2] - D[3]
    assert abs(b_printed - b_def) > 0.1


@pytest.mark.parametrize("R", [2, 3, 4, 8])
def test_prolong_conserves(oracle, R):
    rng = np.random.default_rng(5)
    for _ in range(100):
        u = rng.random(5) * 10.0
        f = oracle.prolong1d(u, R)
        assert abs(f.mean() - u[2]) <= 4e-15 * abs(u[2])


@pytest.mark.parametrize("R", [2, 4])
def test_prolong_exact_for_quadratics(oracle, R):
    c0, c1, c2 = 0.3, -1.2, 0.7
    P = Polynomial([c0, c1, c2]).integ()
    u = np.array([P(k + 1) - P(k) for k in range(-2, 3)])     # cells [-2,-1] .. [2,3], cell i = [0,1]
    want = np.array([(P((s + 1) / R) - P(s / R)) * R for s in range(R)])
    assert np.abs(oracle.prolong1d(u, R) - want).max() <= 1e-14


def test_prolong_takes_the_smooth_side_of_a_step(oracle):
    R = 4
    u = np.array([0.0, 0.0, 1.0, 1.0, 1.0])
    f = oracle.prolong1d(u, R)
    assert np.abs(f - 1.0).max() <= 1e-9
    # fixed ideal weights (d_r) would put a new extremum in the cell
    ideal = definition_prolong(u, R, eps=1e30)
    assert ideal.max() > 1.0 + 1e-2 or ideal.min() < 1.0 - 1e-2


def test_prolong_box_conserves_and_is_exact_for_quadratics(oracle):
    R, ncx, ncv = 4, 16, 12
    rng = np.random.default_rng(9)
    fc = rng.random((ncx, ncv)) + 0.5
    vg = rng.random(4) + 0.5
    box = (8, 12, 31, 35)                                     # level-1 indices, aligned to R
    f = oracle.prolong_box(fc, vg, R, box)
    assert f.shape == (24, 24)
    for cx in range(box[0] // R, box[2] // R + 1):
        for cv in range(box[1] // R, box[3] // R + 1):
            blk = f[(cx * R - box[0]):(cx * R - box[0] + R), (cv * R - box[1]):(cv * R - box[1] + R)]
            assert abs(blk.mean() - fc[cx, cv]) <= 1e-14 * fc[cx, cv]
    # tensor quadratic away from the periodic seam and the v ghosts
    Px = Polynomial([0.2, 0.05, -0.01]).integ()
    Pv = Polynomial([1.0, -0.03, 0.02]).integ()
    cx_avg = np.array([Px(k + 1) - Px(k) for k in range(ncx)])
    cv_avg = np.array([Pv(k + 1) - Pv(k) for k in range(ncv)])
    fq = cx_avg[:, None] * cv_avg[None, :]
    fine = oracle.prolong_box(fq, vg, R, (12, 12, 27, 27))
    fx = np.array([(Px((k + 1) / R) - Px(k / R)) * R for k in range(12, 28)])
    fv = np.array([(Pv((k + 1) / R) - Pv(k / R)) * R for k in range(12, 28)])
    assert np.abs(fine - fx[:, None] * fv[None, :]).max() <= 1e-13


def test_tag_closed_forms_and_scaling(oracle):
    a, b = 0.7, -0.4
    for n, h in ((32, 0.1), (64, 0.05)):
        x = (np.arange(n) + 0.5) * h
        v = (np.arange(n) + 0.5) * h
        f = a * x[:, None] + b * v[None, :]                    # cell averages of a linear field
        t = oracle.tag_values(f, h, h, np.zeros(4))
        d1 = np.sqrt(0.5 * (h * (2 * a * h) ** 2 + h * (2 * b * h) ** 2))
        assert np.abs(t[2:-2, 2:-2] - d1).max() <= 1e-13
    # delta1 carries h^(3/2) for a fixed slope, delta2 h^4 for a fixed curvature
    vals1, vals2 = [], []
    for h in (0.1, 0.05):
        n = 40
        x = (np.arange(n) + 0.5) * h
        f1 = 2.0 * x[:, None] + 0 * x[None, :]
        vals1.append(oracle.tag_values(f1, h, h, np.zeros(4))[10, 10])
        P = Polynomial([0, 0, 3.0]).integ()                    # 3 (x - xc)^2 centred on cell 10: delta1 = 0 there
        avg = np.array([(P((k + 1 - 10.5) * h) - P((k - 10.5) * h)) / h for k in range(n)])
        f2 = avg[:, None] + 0 * x[None, :]
        vals2.append(oracle.tag_values(f2, h, h, np.zeros(4))[10, 10])
    assert abs(np.log2(vals1[0] / vals1[1]) - 1.5) < 1e-9
    assert abs(np.log2(vals2[0] / vals2[1]) - 4.0) < 1e-9


def test_tag_covariance_and_constant(oracle):
    rng = np.random.default_rng(3)
    f = rng.random((24, 20))
    vg = rng.random(4)
    t = oracle.tag_values(f, 0.3, 0.2, vg)
    ts = oracle.tag_values(np.roll(f, 5, axis=0), 0.3, 0.2, vg)
    assert np.array_equal(np.roll(t, 5, axis=0), ts)
    tr = oracle.tag_values(f[::-1].copy(), 0.3, 0.2, vg)
    assert np.abs(tr[::-1] - t).max() <= 1e-15 * np.abs(t).max()
    c = np.full((24, 20), 0.7)
    assert np.all(oracle.tag_values(c, 0.3, 0.2, np.full(4, 0.7)) == 0.0)
    tags = oracle.tag(f, 0.3, 0.2, vg, float(np.median(t)))
    assert np.array_equal(tags, (t > np.median(t)).astype(np.uint8))


def test_regrid_transfer_keeps_old_values_and_conserves(oracle):
    """State transfer at a regrid: level 0 unchanged, fine values kept where an
    old patch covered the cell, every new patch's coarse averages equal to
    level 0 where it interpolates."""
    rng = np.random.default_rng(4)
    ncx, ncv, R = 16, 20, 2
    f0 = rng.random((ncx, ncv)) + 0.5
    vg = rng.random(4) + 0.5
    old_boxes = [{"level": 1, "lo": [4, 8], "hi": [11, 19]}]
    new_boxes = [{"level": 1, "lo": [8, 4], "hi": [15, 15]}, {"level": 1, "lo": [20, 20], "hi": [27, 39]}]
    old_fine = rng.random((8, 12)) + 0.5
    f_old = np.concatenate([f0.ravel(), old_fine.ravel()])
    fn = oracle.regrid_transfer(f_old, old_boxes, new_boxes, ncx, ncv, R, vg)
    assert np.array_equal(fn[:ncx * ncv], f0.ravel())
    p0 = fn[ncx * ncv:ncx * ncv + 8 * 12].reshape(8, 12)
    p1 = fn[ncx * ncv + 8 * 12:].reshape(8, 20)
    # overlap of the first new box with the old one: fine x 8..11, v 8..15
    assert np.array_equal(p0[0:4, 4:12], old_fine[4:8, 0:8])
    # the second new box touches no old patch: conservative
    for cx in range(4):
        for cv in range(10):
            assert abs(p1[2 * cx:2 * cx + 2, 2 * cv:2 * cv + 2].mean() - f0[10 + cx, 10 + cv]) <= 1e-14
    # coarse cells of the first box outside the overlap are conserved too
    for cx, cv in ((4, 2), (5, 3), (7, 2), (6, 7)):
        blk = p0[2 * (cx - 4):2 * (cx - 4) + 2, 2 * (cv - 2):2 * (cv - 2) + 2]
        if cx >= 6 or cv < 4:
            assert abs(blk.mean() - f0[cx, cv]) <= 1e-14


def test_linear_stability_courant(oracle):
    """The Courant limit of the time step control (section 4: a fraction of
    the linear stability limit of the fourth-order scheme) is 2 sqrt 2 over
    the largest modulus of the flux-divergence symbol.  Pinned three ways:
    the oracle's x-advection operator has the eigenvalues i s(theta_m)/dx on
    every Fourier mode; RK4's amplification on the imaginary axis crosses 1
    at 2 sqrt 2; and oracle RK4 steps of a Fourier-rich state stay bounded
    just below the limit and grow just above it."""
    nu = oracle.linear_stability_courant()
    assert nu == pytest.approx(2.0612, abs=5e-5)
    # symbol of the oracle's operator: one velocity row with v = 1, zero ghosts, a = 0
    nx, dx = 16, 0.25
    L = np.empty((nx, nx))
    for q in range(nx):
        e = np.zeros((nx, 1))
        e[q, 0] = 1.0
        L[:, q] = oracle.rhs(e, np.zeros(nx), dx, 1.0, 0.5, np.zeros(4))[:, 0]
    th = 2.0 * np.pi * np.arange(nx) / nx
    s = (8.0 * np.sin(th) - np.sin(2.0 * th)) / 6.0
    modes = np.exp(1j * np.outer(np.arange(nx), th))
    np.testing.assert_allclose(L @ modes, modes * (-1j * s / dx)[None, :], atol=1e-12)
    dense = np.linspace(0.0, np.pi, 200001)
    s_max = ((8.0 * np.sin(dense) - np.sin(2.0 * dense)) / 6.0).max()
    assert 2.0 * np.sqrt(2.0) / s_max == pytest.approx(nu, rel=1e-9)

    def amp(y):
        z = 1j * y
        return abs(1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24)

    y0 = 2.0 * np.sqrt(2.0)
    assert amp(0.999 * y0) <= 1.0 < amp(1.001 * y0)
    # oracle RK4 steps, a mesh with a mode at theta = 2 pi 2/7 (near the symbol's maximum)
    nx = 7
    f0 = np.random.default_rng(3).random((nx, 1))
    o = oracle.Oracle1D(nx, 1, nx * dx, 0.5, 1.5, 0.0, np.zeros(4))
    growth = {}
    for frac in (0.98, 1.05):
        f = f0.copy()
        for _ in range(200):
            f = o.step_fixed_a(f, np.zeros(nx), frac * nu * dx)
        growth[frac] = np.abs(f - f0.mean()).max() / np.abs(f0 - f0.mean()).max()
    assert growth[0.98] < 1.0 and growth[1.05] > 1e3, growth


def test_stability_limit_closed_forms(oracle):
    ncx, ncv, R, x_len, v_lo, v_hi = 8, 16, 4, 2.0, -8.0, 10.0
    dxc, dvc = x_len / ncx, (v_hi - v_lo) / ncv
    nu = oracle.linear_stability_courant()
    a = np.zeros(ncx + ncx * R)
    assert oracle.amr_stability_limit(a, ncx, ncv, R, x_len, v_lo, v_hi, []) == pytest.approx(nu * dxc / 10.0,
                                                                                              rel=1e-15)
    a[:ncx] = 0.5
    a[ncx:] = np.linspace(-2.0, 1.0, ncx * R)
    want0 = nu / (10.0 / dxc + 0.5 / dvc)
    assert oracle.amr_stability_limit(a, ncx, ncv, R, x_len, v_lo, v_hi, []) == pytest.approx(want0, rel=1e-15)
    # a patch over fine v cells 8..15 (faces at v = -5.75 and -3.5) and fine x 0..3 (a in [-2, -1.71])
    box = {"level": 1, "lo": [0, 8], "hi": [3, 15]}
    dxf, dvf = dxc / R, dvc / R
    want1 = nu / (5.75 / dxf + 2.0 / dvf)
    got = oracle.amr_stability_limit(a, ncx, ncv, R, x_len, v_lo, v_hi, [box])
    assert got == pytest.approx(min(want0, want1), rel=1e-15)
    assert got == oracle.amr_stability_limit(-a, ncx, ncv, R, x_len, v_lo, v_hi, [box])
