"""Pins of the oracle's discrete adjoint.

The adjoint is checked against the forward oracle (itself pinned by
test_oracle_pins.py) through identities that hold for any correct
transpose: the dot-product test <J u, w> = <u, J^T w> for each linear or
affine piece (right-hand side in f, right-hand side in a, the
moment-Poisson-field chain), and central finite differences of the full
nonlinear RK4 step.
"""
import numpy as np
import pytest

import vp_inputs as I


@pytest.fixture(scope="module")
def setup(oracle):
    p = I.landau(12, 14)
    o = oracle.Oracle1D.from_problem(p)
    rng = np.random.default_rng(11)
    f = p.initial_state() * (1 + 0.2 * rng.random((12, 14)))
    a = rng.normal(0, 0.3, 12)
    return p, o, f, a, rng


def test_rhs_adjoint_in_f(oracle, setup):
    p, o, f, a, rng = setup
    u = rng.normal(size=f.shape)
    w = rng.normal(size=f.shape)
    Ju = o.rhs(u, a) - o.rhs(np.zeros_like(u), a)       # L is affine in f
    fb, _ = oracle.rhs_adjoint(f, a, w, p.dx, p.dv, p.v_lo, p.vghost)
    lhs, rhs = (Ju * w).sum(), (u * fb).sum()
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0)


def test_rhs_adjoint_in_a(oracle, setup):
    p, o, f, a, rng = setup
    u = rng.normal(size=a.shape)
    w = rng.normal(size=f.shape)
    Ju = o.rhs(f, u) - o.rhs(f, np.zeros_like(u))       # L is affine in a
    _, ab = oracle.rhs_adjoint(f, a, w, p.dx, p.dv, p.v_lo, p.vghost)
    lhs, rhs = (Ju * w).sum(), (u * ab).sum()
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0)


def test_constraints_adjoint(oracle, setup):
    p, o, f, a, rng = setup
    u = rng.normal(size=f.shape)
    w = rng.normal(size=a.shape)
    Ku = o.constraints(u)[0] - o.constraints(np.zeros_like(u))[0]
    fb = o.constraints_adjoint(w, np.zeros_like(f))
    lhs, rhs = (Ku * w).sum(), (u * fb).sum()
    assert abs(lhs - rhs) < 1e-11 * max(abs(lhs), 1.0)


def test_step_adjoint_finite_difference(oracle, setup):
    p, o, f, a, rng = setup
    dt = 0.02
    lam = rng.normal(size=f.shape)
    mu = o.adjoint_step(f, lam, dt)
    for trial in range(3):
        u = rng.normal(size=f.shape)
        h = 1e-5
        fd = ((o.step(f + h * u, dt) - o.step(f - h * u, dt)) / (2 * h) * lam).sum()
        ad = (u * mu).sum()
        assert abs(fd - ad) < 1e-8 * max(abs(ad), 1.0), (fd, ad)


def test_step_adjoint_is_not_identity(oracle, setup):
    """The adjoint differs from lam by the stage terms (guards against a
    reverse pass that silently drops them)."""
    p, o, f, a, rng = setup
    lam = rng.normal(size=f.shape)
    mu = o.adjoint_step(f, lam, 0.02)
    assert np.abs(mu - lam).max() > 1e-3
