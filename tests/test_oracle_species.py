"""Pins of the several-species oracle (one field from the charge density of
every species, each species advanced on its own velocity mesh).

- one species of charge -1 over a unit background is the single-species
  oracle step (the background model of section 2);
- a pair plasma (charges -1, +1, q/m -1, +1) with equal distributions and no
  background has a field that vanishes exactly; each species then streams
  freely (the single-species oracle with a = 0);
- two beams of one species kept as two species evolve, summed, like their
  sum as one species (the equations are linear in f for a given field and
  the field depends on the total charge);
- a spatially uniform species of very heavy particles acts as the uniform
  neutralising background: the periodic Poisson solve ignores the mean of
  rho, and the heavy species barely moves.
"""
import math

import numpy as np
import pytest

import vp_inputs as I


def species_of(prob):
    return {"dv": prob.dv, "v_lo": prob.v_lo, "vghost": prob.vghost, "qm": prob.qm}


def test_one_species_is_the_background_model(oracle):
    p = I.landau(32, 48, eps=0.05)
    f = p.initial_state()
    o = oracle.Oracle1D.from_problem(p)
    dt = 0.02
    got = oracle.species_rk4_step([f], [species_of(p)], [-1.0], 1.0, p.dx, dt)[0]
    want = o.step(f, dt)
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()
    a, _ = oracle.species_field([f], [species_of(p)], [-1.0], 1.0, p.dx)
    assert np.abs(a[0] - o.constraints(f)[0]).max() <= 1e-14 * np.abs(a[0]).max()


def test_pair_plasma_has_no_field(oracle):
    pe = I.landau(24, 40, eps=0.1)
    pp = I.Problem1D(nx=24, nv=40, x_lo=pe.x_lo, x_len=pe.x_len, v_lo=pe.v_lo, v_hi=pe.v_hi, qm=+1.0, eps=0.1, k=0.5)
    f = pe.initial_state()
    sp = [species_of(pe), species_of(pp)]
    a, E = oracle.species_field([f, f], sp, [-1.0, 1.0], 0.0, pe.dx)
    assert np.all(E == 0.0) and np.all(a[0] == 0.0) and np.all(a[1] == 0.0)
    dt = 0.05
    out = oracle.species_rk4_step([f, f], sp, [-1.0, 1.0], 0.0, pe.dx, dt)
    want = oracle.Oracle1D.from_problem(pe).step_fixed_a(f, np.zeros(24), dt)
    for g in out:
        assert np.abs(g - want).max() <= 1e-15 * np.abs(want).max()


def test_two_beams_sum_like_one_species(oracle):
    nx, nv = 32, 64
    p = I.Problem1D(nx=nx, nv=nv, x_lo=0.0, x_len=10 * math.pi, v_lo=-8.0, v_hi=8.0, profile="two_stream",
                    eps=0.01, k=0.2)
    f = p.initial_state()
    v = p.v_lo + (np.arange(nv) + 0.5) * p.dv
    f1 = f * (v > 0)[None, :]
    f2 = f - f1
    dt = 0.05
    o1, o2 = oracle.species_rk4_step([f1, f2], [species_of(p)] * 2, [-1.0, -1.0], 1.0, p.dx, dt)
    want = oracle.Oracle1D.from_problem(p).step(f, dt)
    assert np.abs(o1 + o2 - want).max() <= 1e-13 * np.abs(want).max()
    # and not trivially: each beam alone is far from the sum
    assert np.abs(o1 - want).max() > 1e-3 * np.abs(want).max()


def test_uniform_heavy_species_is_a_background(oracle):
    nx = 32
    pe = I.landau(nx, 48, eps=0.05)
    vth = 0.01
    pi_ = I.Problem1D(nx=nx, nv=32, x_lo=pe.x_lo, x_len=pe.x_len, v_lo=-8 * vth, v_hi=8 * vth, qm=1e-10, eps=0.0,
                      k=0.5, veq=I.cell_average_1d(lambda u: I.maxwellian(u / vth) / vth, -8 * vth, 8 * vth, 32,
                                                   first=-2, count=36))
    fe, fi = pe.initial_state(), pi_.initial_state()
    dt = 0.02
    oe, oi = oracle.species_rk4_step([fe, fi], [species_of(pe), species_of(pi_)], [-1.0, 1.0], 0.0, pe.dx, dt)
    want = oracle.Oracle1D.from_problem(pe).step(fe, dt)
    assert np.abs(oe - want).max() <= 1e-12 * np.abs(want).max()
    assert np.abs(oi - fi).max() <= 1e-9 * np.abs(fi).max()


# ---- one two-level hierarchy per species

BOXES = [{"level": 1, "lo": [8, 16], "hi": [23, 39]}, {"level": 1, "lo": [40, 8], "hi": [51, 27]}]


def amr_setup(oracle, qm, eps=0.05, boxes=BOXES, coarse=(16, 12), R=4):
    f, vc, vf = I.amr_landau(boxes, coarse=coarse, ratio=R, eps=eps)
    o = oracle.OracleAMR(coarse[0], coarse[1], 4 * math.pi, -8.0, 8.0, qm, R, boxes, vc, vf)
    return o, f


def test_amr_one_species_is_the_background_model(oracle):
    o, f = amr_setup(oracle, -1.0)
    dt = 0.02
    got = oracle.amr_species_rk4_step([o], [f], [-1.0], 1.0, dt)[0]
    assert np.array_equal(got, o.step(f, dt))
    a = oracle.amr_species_field([o], [f], [-1.0], 1.0)[0]
    assert np.array_equal(a, o.constraints(f)[0])


def test_amr_pair_plasma_streams_freely(oracle):
    oe, f = amr_setup(oracle, -1.0)
    op, _ = amr_setup(oracle, +1.0)
    o0, _ = amr_setup(oracle, 0.0)
    a = oracle.amr_species_field([oe, op], [f, f], [-1.0, 1.0], 0.0)
    assert np.all(a[0] == 0.0) and np.all(a[1] == 0.0)
    dt = 0.05
    out = oracle.amr_species_rk4_step([oe, op], [f, f], [-1.0, 1.0], 0.0, dt)
    want = o0.step(f, dt)
    for g in out:
        assert np.abs(g - want).max() <= 1e-15 * np.abs(want).max()


def test_amr_two_beams_sum_like_one_species(oracle):
    o, f = amr_setup(oracle, -1.0, eps=0.1)
    rng = np.random.default_rng(3)
    w = rng.random(f.size)
    f1, f2 = f * w, f * (1.0 - w)
    dt = 0.03
    o1, o2 = oracle.amr_species_rk4_step([o, o], [f1, f2], [-1.0, -1.0], 1.0, dt)
    want = o.step(f, dt)
    assert np.abs(o1 + o2 - want).max() <= 1e-13 * np.abs(want).max()
    assert np.abs(o1 - want).max() > 1e-2 * np.abs(want).max()
