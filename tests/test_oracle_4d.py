"""Pins of the 2D+2V oracle (the direction-by-direction extension of the
fourth-order scheme of section 2).

- Poisson: a discrete Fourier mode is scaled by the closed-form symbol of
  the summed 1D operators; a y-independent density reproduces the 1D
  oracle's bordered-LU solve (a different algorithm); fourth-order
  convergence of the field against the exact solution.
- Right-hand side: exact (to rounding) cell averages of
  -v . grad_x f - a . grad_v f for f a product of quadratics in the four
  directions and a linear in x and y, at cells whose stencils stay inside
  the mesh: this fixes every face formula and every product-rule
  correction, including the cross terms (a_x varying along y, a_y along x).
- Dimensional reduction: f = F(x, vx) G(vy), independent of y, with
  dvy sum G = 1 steps exactly like the 1D+1V oracle on F.
- Free streaming along x and along y converges at fourth order to the
  exact solution; mass is conserved without a field.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import Polynomial

import vp_inputs as I


def cell_avg_poly(P, lo, h, n):
    Pi = P.integ()
    xl = lo + np.arange(n) * h
    return (Pi(xl + h) - Pi(xl)) / h


def make(oracle, nx, ny, nvx, nvy, x_len=4 * math.pi, y_len=4 * math.pi, v_lo=-6.0, v_hi=6.0):
    veq_x = I.cell_average_1d(I.maxwellian, v_lo, v_hi, nvx, first=-2, count=nvx + 4)
    veq_y = I.cell_average_1d(I.maxwellian, v_lo, v_hi, nvy, first=-2, count=nvy + 4)
    return oracle.Oracle4D(nx, ny, nvx, nvy, x_len, y_len, v_lo, v_hi, -1.0, veq_x, veq_y), veq_x, veq_y


# ------------------------------------------------------------------ Poisson


@pytest.mark.parametrize("nx,ny,m,l", [(8, 8, 1, 2), (12, 10, 3, 1), (16, 16, 0, 5), (9, 7, 4, 3)])
def test_poisson_fourier_mode_symbol(oracle, nx, ny, m, l):
    o, _, _ = make(oracle, nx, ny, 4, 4, x_len=3.0, y_len=5.0)
    dx, dy = 3.0 / nx, 5.0 / ny
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    tx, ty = 2 * math.pi * m / nx, 2 * math.pi * l / ny
    rho = np.cos(tx * i + ty * j + 0.3)
    rho -= rho.mean()
    sym = (30 - 32 * math.cos(tx) + 2 * math.cos(2 * tx)) / (12 * dx * dx) + \
          (30 - 32 * math.cos(ty) + 2 * math.cos(2 * ty)) / (12 * dy * dy)
    phi, res = o.poisson(rho)
    assert res < 1e-12
    np.testing.assert_allclose(phi, rho / sym, rtol=0, atol=1e-12 * np.abs(rho / sym).max())


def test_poisson_y_independent_matches_1d_lu(oracle):
    nx, ny = 24, 6
    o, _, _ = make(oracle, nx, ny, 4, 4)
    rng = np.random.default_rng(3)
    r1 = rng.standard_normal(nx)
    rho = np.repeat(r1[:, None], ny, axis=1)
    phi, _ = o.poisson(rho)
    phi1 = oracle.poisson_solve(r1, 4 * math.pi / nx)
    np.testing.assert_allclose(phi, np.repeat(phi1[:, None], ny, axis=1), rtol=0, atol=1e-12 * np.abs(phi1).max())
    E = o.field(phi)
    E1 = oracle.field(phi1, 4 * math.pi / nx)
    np.testing.assert_allclose(E[: nx * ny].reshape(nx, ny), np.repeat(E1[:, None], ny, axis=1), rtol=0,
                               atol=1e-11 * np.abs(E1).max())
    assert np.abs(E[nx * ny:]).max() < 1e-12 * np.abs(E1).max()


def test_poisson_field_fourth_order(oracle):
    """rho = cos(kx x) cos(ky y): phi = rho / (kx^2 + ky^2),
    Ex = kx sin(kx x) cos(ky y) / (kx^2 + ky^2) (cell averages)."""
    Lx, Ly = 4 * math.pi, 2 * math.pi
    kx, ky = 0.5, 2.0
    errs = []
    for n in (32, 64, 128):
        o, _, _ = make(oracle, n, n, 2, 2, x_len=Lx, y_len=Ly)
        dx, dy = Lx / n, Ly / n
        xl, yl = np.arange(n) * dx, np.arange(n) * dy
        cx = (np.sin(kx * (xl + dx)) - np.sin(kx * xl)) / (kx * dx)
        sx = -(np.cos(kx * (xl + dx)) - np.cos(kx * xl)) / (kx * dx)
        cy = (np.sin(ky * (yl + dy)) - np.sin(ky * yl)) / (ky * dy)
        sy = -(np.cos(ky * (yl + dy)) - np.cos(ky * yl)) / (ky * dy)
        rho = np.outer(cx, cy)
        phi, _ = o.poisson(rho)
        E = o.field(phi)
        k2 = kx * kx + ky * ky
        ex = kx * np.outer(sx, cy) / k2
        ey = ky * np.outer(cx, sy) / k2
        errs.append(max(np.abs(phi - rho / k2).max(), np.abs(E[: n * n].reshape(n, n) - ex).max(),
                        np.abs(E[n * n:].reshape(n, n) - ey).max()))
    rates = [math.log2(errs[q] / errs[q + 1]) for q in range(2)]
    assert min(rates) > 3.8, (errs, rates)


def test_moment_of_equilibrium(oracle):
    o, vx, vy = make(oracle, 3, 2, 16, 12)
    f = np.ones((3, 2))[:, :, None, None] * vx[None, None, 2:-2, None] * vy[None, None, None, 2:-2]
    n = o.moment(f)
    expect = (12.0 / 16 * vx[2:-2].sum()) * (12.0 / 12 * vy[2:-2].sum())
    np.testing.assert_allclose(n, expect, rtol=1e-14)
    assert abs(expect - math.erf(6 / math.sqrt(2)) ** 2) < 1e-13


# ------------------------------------------------------------------ right-hand side


def test_rhs_polynomial_exactness(oracle):
    n = 8
    Lx, Ly, vlo, vhi = 3.0, 2.5, -2.0, 2.0
    o, _, _ = make(oracle, n, n, n, n, x_len=Lx, y_len=Ly, v_lo=vlo, v_hi=vhi)
    dx, dy, dv = Lx / n, Ly / n, (vhi - vlo) / n
    X = Polynomial([0.3, -0.2, 0.15])
    Y = Polynomial([0.5, 0.1, -0.05])
    U = Polynomial([1.0, 0.2, -0.1])
    V = Polynomial([0.7, -0.3, 0.2])
    s = Polynomial([0.0, 1.0])
    Xb, Yb = cell_avg_poly(X, 0, dx, n), cell_avg_poly(Y, 0, dy, n)
    Ub, Vb = cell_avg_poly(U, vlo, dv, n), cell_avg_poly(V, vlo, dv, n)
    f = Xb[:, None, None, None] * Yb[None, :, None, None] * Ub[None, None, :, None] * Vb[None, None, None, :]
    xc, yc = (np.arange(n) + 0.5) * dx, (np.arange(n) + 0.5) * dy
    (ax0, axx, axy), (ay0, ayx, ayy) = (0.4, -0.3, 0.25), (-0.2, 0.15, 0.35)
    ax = ax0 + axx * xc[:, None] + axy * yc[None, :]
    ay = ay0 + ayx * xc[:, None] + ayy * yc[None, :]
    k = o.rhs(f, np.concatenate([ax.ravel(), ay.ravel()]))
    # exact cell averages of -vx df/dx - vy df/dy - ax df/dvx - ay df/dvy
    vU, vV = cell_avg_poly(s * U, vlo, dv, n), cell_avg_poly(s * V, vlo, dv, n)
    dX, dY = cell_avg_poly(X.deriv(), 0, dx, n), cell_avg_poly(Y.deriv(), 0, dy, n)
    dU, dV = cell_avg_poly(U.deriv(), vlo, dv, n), cell_avg_poly(V.deriv(), vlo, dv, n)
    xX, yY = cell_avg_poly(s * X, 0, dx, n), cell_avg_poly(s * Y, 0, dy, n)
    axXY = ax0 * np.outer(Xb, Yb) + axx * np.outer(xX, Yb) + axy * np.outer(Xb, yY)
    ayXY = ay0 * np.outer(Xb, Yb) + ayx * np.outer(xX, Yb) + ayy * np.outer(Xb, yY)
    exact = -(dX[:, None, None, None] * Yb[None, :, None, None] * vU[None, None, :, None] * Vb[None, None, None, :]) \
            - (Xb[:, None, None, None] * dY[None, :, None, None] * Ub[None, None, :, None] * vV[None, None, None, :]) \
            - axXY[:, :, None, None] * dU[None, None, :, None] * Vb[None, None, None, :] \
            - ayXY[:, :, None, None] * Ub[None, None, :, None] * dV[None, None, None, :]
    inner = (slice(2, -2),) * 4
    np.testing.assert_allclose(k[inner], exact[inner], rtol=0, atol=1e-13 * np.abs(exact).max())


def test_dimensional_reduction(oracle):
    """y-independent f = F(x, vx) G(vy), dvy sum G = 1: a full RK4 step with
    the field equals the 1D+1V oracle's step of F, times G."""
    nx, ny, nvx, nvy = 16, 4, 20, 10
    o, vx, vy = make(oracle, nx, ny, nvx, nvy)
    dvy = 12.0 / nvy
    sG = dvy * vy[2:-2].sum()
    G = vy[2:-2] / sG
    veq1 = vx * sG                                     # 1D equilibrium scaled so that the ghosts agree
    o1 = oracle.Oracle1D(nx, nvx, 4 * math.pi, -6.0, 6.0, -1.0, veq1[[0, 1, nvx + 2, nvx + 3]])
    cx = I.cos_cell_average(0.0, 4 * math.pi, nx, 0.5)
    F = (1.0 + 0.05 * cx)[:, None] * veq1[None, 2:-2]
    f = np.ascontiguousarray(np.broadcast_to(F[:, None, :, None] * G[None, None, None, :], (nx, ny, nvx, nvy)))
    a4, _, _ = o.constraints(f)
    a1, _, _, _ = o1.constraints(F)
    np.testing.assert_allclose(a4[: nx * ny].reshape(nx, ny), np.repeat(a1[:, None], ny, 1), rtol=0,
                               atol=1e-12 * np.abs(a1).max())
    assert np.abs(a4[nx * ny:]).max() < 1e-13 * np.abs(a1).max()
    dt = 0.05
    g, G1 = f, F
    for _ in range(2):
        g = o.step(g, dt)
        G1 = o1.step(G1, dt)
    want = G1[:, None, :, None] * G[None, None, None, :]
    np.testing.assert_allclose(g, np.broadcast_to(want, g.shape), rtol=0, atol=1e-13 * np.abs(want).max())


def free_stream_exact_1d(n, L, nv, v_lo, v_hi, t, eps, k):
    """Exact cell averages over (s, v) cells of (1 + eps cos(k (s - v t))) M(v)."""
    ds, dv = L / n, (v_hi - v_lo) / nv
    nodes, w = np.polynomial.legendre.leggauss(16)
    vl = v_lo + np.arange(nv) * dv
    v = vl[:, None] + 0.5 * dv * (nodes[None, :] + 1.0)
    Mv = I.maxwellian(v)
    sl = np.arange(n) * ds
    ss = (np.sin(k * (sl[:, None, None] + ds - v[None] * t)) - np.sin(k * (sl[:, None, None] - v[None] * t))) / (k * ds)
    base = 0.5 * (Mv * w[None, :]).sum(-1)
    return base[None, :] + eps * 0.5 * (Mv[None] * ss * w[None, None, :]).sum(-1)


@pytest.mark.parametrize("axis", ["x", "y"])
def test_free_streaming_fourth_order(oracle, axis):
    T, eps, k = 0.5, 0.05, 0.5
    errs = []
    for n in (32, 64, 128):
        shape = (n, 1, n, 1) if axis == "x" else (1, n, 1, n)
        o, vx, vy = make(oracle, *shape)
        other = vy[2:-2] if axis == "x" else vx[2:-2]        # the single cell of the other velocity
        e0 = free_stream_exact_1d(n, 4 * math.pi, n, -6.0, 6.0, 0.0, eps, k)
        eT = free_stream_exact_1d(n, 4 * math.pi, n, -6.0, 6.0, T, eps, k)
        f = (e0 * other[0]).reshape(shape)
        nsteps = int(math.ceil(T / (0.5 * (4 * math.pi / n) / 6.0)))
        a = np.zeros(2 * (shape[0] * shape[1]))
        for _ in range(nsteps):
            f = o.step_fixed_a(f, a, T / nsteps)
        errs.append(np.abs(f.reshape(n, n) - eT * other[0]).max())
    rates = [math.log2(errs[q] / errs[q + 1]) for q in range(2)]
    assert min(rates) > 3.7, (errs, rates)


def test_mass_conserved_without_field(oracle):
    o, _, _ = make(oracle, 5, 6, 7, 8)
    rng = np.random.default_rng(1234)
    f = rng.random((5, 6, 7, 8))
    g = o.step_fixed_a(f, np.zeros(60), 0.01)
    assert abs(g.sum() - f.sum()) < 1e-13 * f.sum()
    assert np.abs(g - f).max() > 1e-4
