"""Pins of the oracle's subcycled two-level step (asynchronous time stepping,
named as future work in section 5; the reading: the coarse level takes dt
with the field of its own moment, the patches take R substeps of dt / R
with coarse data from the continuous extension of the coarse RK4 step, taken
as the RK4 stage values on its Taylor expansion at each substep start, then
refluxing and the average-down).

- the continuous extension: b(0) = 0, b(1) = the classical weights, and on
  y' = lambda y the interpolant at an interior theta is third order (local
  error O(h^4));
- the fine-stage weights against derivatives of a cubic fitted to samples
  of the extension, and on y' = lambda y against the RK4 stage values of
  the substep;
- no patches: the step is the single-level RK4 step on the coarse mesh
  (an independent code path);
- composite mass is conserved to round-off and covered coarse cells hold
  the mean of their fine cells;
- with no field (q/m = 0) the subcycled and synchronous steps integrate the
  same semi-discrete system, so their difference after a fixed time falls
  at fourth order in dt;
- the Landau damping rate and frequency of a subcycled two-level run.
"""
import cmath
import math

import numpy as np
import pytest

import vp_inputs as I
from test_oracle_amr import composite_mass, small_layout
from test_oracle_pins import landau_fit, landau_root


def test_dense_weights_endpoints(oracle):
    np.testing.assert_array_equal(oracle.rk4_dense_weights(0.0), np.zeros(4))
    np.testing.assert_allclose(oracle.rk4_dense_weights(1.0), [1 / 6, 1 / 3, 1 / 3, 1 / 6], rtol=0, atol=1e-16)
    for th in (0.25, 0.5, 0.8):
        assert abs(oracle.rk4_dense_weights(th).sum() - th) < 1e-15


def test_dense_output_third_order(oracle):
    """y' = lambda y, one classical RK4 step of h from y = 1: the continuous
    extension at theta = 0.3 against exp(lambda theta h)."""
    lam = complex(-0.7, 2.3)
    theta = 0.3

    def err(h):
        k1 = lam
        k2 = lam * (1 + 0.5 * h * k1)
        k3 = lam * (1 + 0.5 * h * k2)
        k4 = lam * (1 + h * k3)
        b = oracle.rk4_dense_weights(theta)
        y = 1 + h * (b[0] * k1 + b[1] * k2 + b[2] * k3 + b[3] * k4)
        return abs(y - cmath.exp(lam * theta * h))

    e1, e2 = err(0.1), err(0.05)
    assert 13.0 < e1 / e2 < 19.0, (e1, e2)


@pytest.mark.parametrize("theta0,eta", [(0.0, 0.5), (0.25, 0.25), (0.5, 0.5), (0.75, 0.25)])
def test_substage_weights_from_the_dense_polynomial(oracle, theta0, eta):
    """The fine-stage coarse data are the RK4 stage values on the Taylor
    expansion of the continuous extension P at theta0: the derivatives are
    taken here from a cubic fitted through samples of P (not from the
    oracle's closed forms)."""
    ts = np.linspace(0.0, 1.0, 7)
    W = np.array([oracle.rk4_dense_weights(t) for t in ts])
    for q in range(4):
        c = np.polynomial.Polynomial.fit(ts, W[:, q], 3).convert()
        P = [c.deriv(k)(theta0) for k in range(4)]
        want = [P[0], P[0] + eta / 2 * P[1], P[0] + eta / 2 * P[1] + eta ** 2 / 4 * P[2],
                P[0] + eta * P[1] + eta ** 2 / 2 * P[2] + eta ** 3 / 4 * P[3]]
        got = [oracle.rk4_substage_weights(theta0, eta, s)[q] for s in range(4)]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def test_substage_values_are_rk4_stages_on_exponential(oracle):
    """On y' = lambda y the four coarse data of a fine substep approach the
    RK4 stage values of that substep started from P(theta0) as the coarse
    step shrinks (each is off by the error of the cubic's derivatives)."""
    lam = complex(-0.4, 1.9)

    def err(dt, theta0=0.5, eta=0.25):
        k1 = lam
        k2 = lam * (1 + 0.5 * dt * k1)
        k3 = lam * (1 + 0.5 * dt * k2)
        k4 = lam * (1 + dt * k3)
        K = np.array([k1, k2, k3, k4])
        y0 = 1 + dt * (oracle.rk4_dense_weights(theta0) @ K)
        h = eta * dt
        Y = [y0]
        Y.append(y0 + 0.5 * h * lam * Y[0])
        Y.append(y0 + 0.5 * h * lam * Y[1])
        Y.append(y0 + h * lam * Y[2])
        return max(abs(1 + dt * (oracle.rk4_substage_weights(theta0, eta, s) @ K) - Y[s]) for s in range(4))

    e1, e2 = err(0.2), err(0.1)
    assert e1 / e2 > 14.0, (e1, e2)


def test_no_patches_is_single_level_step(oracle):
    ncx, ncv = 32, 48
    p = I.Problem1D(ncx, ncv, 0.0, 4 * math.pi, -8.0, 8.0, eps=0.2, k=0.5)
    o1 = oracle.Oracle1D.from_problem(p)
    veq_f = I.cell_average_1d(I.maxwellian, -8.0, 8.0, ncv * 2, first=-2, count=ncv * 2 + 4)
    o = oracle.OracleAMR(ncx, ncv, 4 * math.pi, -8.0, 8.0, -1.0, 2, [], p.veq, veq_f)
    f = p.initial_state()
    dt = 0.05
    g1 = o1.step(f, dt)
    g = o.subcycle_step(f.ravel(), dt)
    np.testing.assert_allclose(g, g1.ravel(), rtol=0, atol=1e-14 * np.abs(g1).max())
    assert np.abs(g1 - f).max() > 1e-6


def landau_hierarchy(oracle, boxes, qm=-1.0, eps=0.2, ncx=32, ncv=48, R=4):
    f, veq_c, veq_f = I._amr_state(I.maxwellian, 0.0, 4 * math.pi, -8.0, 8.0, eps, 0.5, boxes, (ncx, ncv), R)
    o = oracle.OracleAMR(ncx, ncv, 4 * math.pi, -8.0, 8.0, qm, R, boxes, veq_c, veq_f)
    return o, f


def test_subcycle_conserves_mass_and_averages_down(oracle):
    boxes = small_layout()
    o, f = landau_hierarchy(oracle, boxes)
    rng = np.random.default_rng(11)
    f = f * (1 + 0.01 * rng.random(f.size))
    dxc, dvc = 4 * math.pi / 32, 16.0 / 48
    m0 = composite_mass(o, f, boxes, dxc, dvc)
    g = f
    for _ in range(3):
        g = o.subcycle_step(g, 0.04)
    assert abs(composite_mass(o, g, boxes, dxc, dvc) - m0) < 1e-13 * m0
    assert np.abs(g - f).max() > 1e-6
    fc = g[:32 * 48].reshape(32, 48)
    for p, b in enumerate(boxes):
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        nx, nv = x1 - x0 + 1, v1 - v0 + 1
        fp = g[o.offset(p): o.offset(p) + nx * nv].reshape(nx // 4, 4, nv // 4, 4).mean(axis=(1, 3))
        np.testing.assert_allclose(fc[x0 // 4:x0 // 4 + nx // 4, v0 // 4:v0 // 4 + nv // 4], fp, rtol=1e-14)


def test_free_streaming_matches_synchronous_at_fourth_order(oracle):
    """q/m = 0: both steps integrate the same hierarchy ODE (ghosts from the
    coarse level, fine fluxes on coarse-fine faces, the average-down at each
    coarse step); only their time integration differs."""
    boxes = small_layout()
    o, f0 = landau_hierarchy(oracle, boxes, qm=0.0)

    def diff(n):
        dt = 0.2 / n
        fs, fa = f0, f0
        for _ in range(n):
            fs = o.step(fs, dt)
            fa = o.subcycle_step(fa, dt)
        return np.abs(fs - fa).max()

    d1, d2 = diff(8), diff(16)
    assert d1 > 1e-10, d1
    assert d1 / d2 > 12.0, (d1, d2)


@pytest.mark.slow
def test_subcycled_landau_damping_rate(oracle):
    """64 x 128 coarse cells with a ratio-2 patch over the resonant band
    v in [1, 3.625) on the positive side (every coarse column but the last):
    the field decays at the Landau rate."""
    w = landau_root()
    ncx, ncv, R = 64, 128, 2
    boxes = [{"level": 1, "lo": [0, 72 * R], "hi": [63 * R - 1, 93 * R - 1]}]
    f, veq_c, veq_f = I._amr_state(I.maxwellian, 0.0, 4 * math.pi, -8.0, 8.0, 0.01, 0.5, boxes, (ncx, ncv), R)
    o = oracle.OracleAMR(ncx, ncv, 4 * math.pi, -8.0, 8.0, -1.0, R, boxes, veq_c, veq_f)
    p = I.landau(ncx * R, ncv)        # dx of the field diagnostic: the fine configuration mesh

    class P:
        dx = p.dx

        @staticmethod
        def initial_state():
            return f

    dt = 0.5 / (8.0 / (4 * math.pi / ncx) + 0.01 / (16.0 / ncv))
    gamma, omega = landau_fit(o.subcycle_step, lambda g: o.constraints(g)[1], P, dt)
    assert abs(gamma - w.imag) < 0.003, gamma
    assert abs(omega - w.real) < 0.006, omega
