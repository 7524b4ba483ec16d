"""Pins of the limited face averages of section 2 (eqs. limitedFace,
thirdLeft, thirdRight) in the oracle.

- Face values agree with a derivation from the definitions (quadratics
  matching the cell averages, smoothness as the integral of squared
  derivatives over the cell left of the face), independent of the closed
  forms in the oracle.
- Upwind assignment on a step: with flow to the right the face value
  leans to the left-biased candidate, with flow to the left to the
  right-biased one.
- On smooth data the limited face approaches the centred fourth-order
  face at fifth order (the weights tend to 1/2).
- The limited x-advection dissipates: sum_i g_i k_i < 0 on rough data in
  every interior velocity column, where the centred scheme gives zero
  (skew-symmetric); a downwind assignment would make it positive.
- Free streaming of smooth data still converges at about fourth order; a
  step is advected with clearly smaller overshoots than by the centred
  scheme; mass is conserved.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import Polynomial

import vp_inputs as I


def centered(um1, u0, u1, u2):
    return (7.0 * (u0 + u1) - (um1 + u2)) / 12.0


def definition_face(u, upwind_left, eps=1e-6):
    """The limited face from the definitions: the two quadratics with the
    given cell averages on cells [-1,0],[0,1],[1,2] and [0,1],[1,2],[2,3]
    evaluated at the face x = 1; smoothness = integral over cell [0, 1]
    (the cell left of the face, unit width) of p'^2 + p''^2; provisional
    weights (1/2) / (eps + beta)^2 normalised; the larger to the upwind side."""
    def quad(avgs, cells):
        # coefficients c of p(x) = c0 + c1 x + c2 x^2 with the given cell averages
        A = np.array([[1.0, (b * b - a * a) / 2.0, (b ** 3 - a ** 3) / 3.0] for a, b in cells])
        return Polynomial(np.linalg.solve(A, avgs))
    pl = quad(u[0:3], [(-1, 0), (0, 1), (1, 2)])
    pr = quad(u[1:4], [(0, 1), (1, 2), (2, 3)])
    def beta(pp):
        s1 = (pp.deriv() ** 2).integ()
        s2 = (pp.deriv(2) ** 2).integ()
        return (s1(1) - s1(0)) + (s2(1) - s2(0))
    al = 0.5 / (eps + beta(pl)) ** 2
    ar = 0.5 / (eps + beta(pr)) ** 2
    wl, wr = al / (al + ar), ar / (al + ar)
    wmax, wmin = max(wl, wr), min(wl, wr)
    if upwind_left:
        return wmax * pl(1.0) + wmin * pr(1.0)
    return wmin * pl(1.0) + wmax * pr(1.0)


def test_face_matches_definition(oracle):
    rng = np.random.default_rng(11)
    for _ in range(200):
        u = rng.standard_normal(4) * rng.choice([1e-2, 1.0, 10.0])
        for up in (True, False):
            a = oracle.face_limited(*u, up)
            b = definition_face(u, up)
            assert abs(a - b) <= 1e-11 * max(1.0, np.abs(u).max()), (u, up, a, b)


def test_upwind_assignment_on_a_step(oracle):
    right = oracle.face_limited(0.0, 0.0, 1.0, 1.0, True)
    left = oracle.face_limited(0.0, 0.0, 1.0, 1.0, False)
    assert right < 0.5 < left
    # both stay between the two candidates, 1/3 and 2/3
    assert 1 / 3 <= right <= 2 / 3 and 1 / 3 <= left <= 2 / 3


def test_smooth_limit_is_the_centred_face(oracle):
    diffs = []
    for h in (0.2, 0.1, 0.05):
        x = np.arange(-1, 3) * h + 0.3
        u = (np.cos(x) - np.cos(x + h)) / h            # cell averages of sin
        diffs.append(abs(oracle.face_limited(*u, True) - centered(*u)))
    rates = [math.log2(diffs[q] / diffs[q + 1]) for q in range(2)]
    assert min(rates) > 4.5, (diffs, rates)


def test_limited_advection_dissipates(oracle):
    p = I.landau(64, 24, eps=0.0)
    rng = np.random.default_rng(5)
    g = rng.random(p.nx)
    f = np.repeat(g[:, None], p.nv, axis=1)
    a = np.zeros(p.nx)
    k_l = oracle.rhs_limited(f, a, p.dx, p.dv, p.v_lo, p.vghost)
    k_c = oracle.rhs(f, a, p.dx, p.dv, p.v_lo, p.vghost)
    for j in range(1, p.nv - 1):
        e_c = g @ k_c[:, j]
        e_l = g @ k_l[:, j]
        scale = abs(p.v_lo + (j + 0.5) * p.dv) * (g @ g) / p.dx
        assert abs(e_c) < 1e-12 * scale
        assert e_l < -1e-4 * scale


def test_free_streaming_order(oracle):
    from test_oracle_pins import free_streaming_exact
    errs = []
    T = 0.5
    for n in (32, 64, 128):
        p = I.landau(n, n, eps=0.05)
        o = oracle.Oracle1D.from_problem(p)
        f = p.initial_state()
        nsteps = int(math.ceil(T / (0.5 * p.dx / 8.0)))
        for _ in range(nsteps):
            f = o.step_fixed_a_limited(f, np.zeros(n), T / nsteps)
        errs.append(np.abs(f - free_streaming_exact(p, T, 0.05, 0.5)).max())
    rates = [math.log2(errs[q] / errs[q + 1]) for q in range(2)]
    assert min(rates) > 3.5, (errs, rates)


def test_step_overshoot_and_mass(oracle):
    p = I.landau(64, 16, eps=0.0)
    o = oracle.Oracle1D.from_problem(p)
    x = (np.arange(p.nx) + 0.5) * p.dx
    g = ((x > 0.25 * p.x_len) & (x < 0.6 * p.x_len)).astype(float)
    f0 = g[:, None] * p.veq[None, 2:-2] / p.veq[2:-2].max()
    a = np.zeros(p.nx)
    dt = 0.4 * p.dx / 8.0
    fl, fc = f0, f0
    for _ in range(40):
        fl = o.step_fixed_a_limited(fl, a, dt)
        fc = o.step_fixed_a(fc, a, dt)
    over = lambda f: max(f.max() - f0.max(), -f.min())
    # a blend of two third-order candidates is not monotone, but the upwind
    # bias must cut the centred scheme's overshoot markedly
    assert over(fl) < 0.75 * over(fc), (over(fl), over(fc))
    assert abs(fl.sum() - f0.sum()) < 1e-12 * f0.sum()
