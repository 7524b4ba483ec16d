"""Brute force in exact rational arithmetic on small meshes.

An independent evaluation of the semi-discrete operator of section 2 and
of one classic RK4 step (eq. rk4), written with ``fractions.Fraction`` from
the definitions, cell by cell, with the ghost cells addressed by their
indices (x periodic, velocity ghosts j = -2, -1, nv, nv+1 the equilibrium
values).  The fourth-order face average and the product-rule coefficients
are not typed in: the face weights come from the cubic whose averages over
the four cells around the face match the data, and the correction factor
h^2/12 from the second moment of a cell.  Every cell is compared with the
CPU oracle, including the velocity-boundary rows and the x-wrap columns
that the polynomial-exactness pins leave out.  The last tests plant
plausible mistakes in a copy of the oracle (swapped velocity ghost values,
a lost x wrap) and check that this comparison catches each of them.
"""
import ctypes
import os
import subprocess
from fractions import Fraction as Fr

import numpy as np
import pytest

import vp_inputs as I


# ------------------------------------------------------------------ exact helpers


def solve_exact(A, b):
    """Gauss-Jordan elimination over the rationals (A square, nonsingular)."""
    n = len(A)
    M = [list(map(Fr, row)) + [Fr(bi)] for row, bi in zip(A, b)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [x / piv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                fac = M[r][c]
                M[r] = [x - fac * y for x, y in zip(M[r], M[c])]
    return [M[r][n] for r in range(n)]


def cell_moment(k, m):
    """Average of x^m over the unit cell [k, k+1]."""
    return (Fr(k + 1) ** (m + 1) - Fr(k) ** (m + 1)) / (m + 1)


def face_weights():
    """Weights of the face value at x = 0 of the cubic whose averages over
    the cells [-2,-1], [-1,0], [0,1], [1,2] are the data (cells i-1, i, i+1,
    i+2 around the face i+1/2)."""
    cells = [-2, -1, 0, 1]
    A = [[cell_moment(k, m) for m in range(4)] for k in cells]
    w = []
    for q in range(4):
        e = [Fr(int(q == r)) for r in range(4)]
        w.append(solve_exact(A, e)[0])          # the constant coefficient = value at 0
    return w


W_FACE = face_weights()
# average of x^2 over a unit cell centred at 0: avg(p q) = avg(p) avg(q) + h^2/12 p' q'
# for linear p, q on a cell of width h
SECOND_MOMENT = (Fr(1, 2) ** 3 - Fr(-1, 2) ** 3) / 3


def test_derived_constants():
    """The derivation gives the centred fourth-order face average and 1/12."""
    assert W_FACE == [Fr(-1, 12), Fr(7, 12), Fr(7, 12), Fr(-1, 12)]
    assert SECOND_MOMENT == Fr(1, 12)


def face(u):
    return sum(w * x for w, x in zip(W_FACE, u))


# ------------------------------------------------------------------ 1D+1V


def brute_rhs(f, a, dx, dv, v_lo, veq):
    """k = L(f; a) of section 2 (eq. semi-discrete); f: nx lists of nv
    Fractions, a: nx Fractions, veq: dict j -> ghost value for j outside
    [0, nv)."""
    nx, nv = len(f), len(f[0])

    def F(i, j):
        return veq[j] if (j < 0 or j >= nv) else f[i % nx][j]

    def A(i):
        return a[i % nx]

    def fx(i, j):        # face average on x_{i+1/2}, velocity row j
        return face([F(i - 1, j), F(i, j), F(i + 1, j), F(i + 2, j)])

    def fv(i, j):        # face average on v_{j+1/2}, configuration column i
        return face([F(i, j - 1), F(i, j), F(i, j + 1), F(i, j + 2)])

    def vbar(j):         # average of v over velocity cell j
        return v_lo + (j + Fr(1, 2)) * dv

    def gx(i, j):        # <v f> on x_{i+1/2}: v varies along v with slope 1
        dfdv = (fx(i, j + 1) - fx(i, j - 1)) / (2 * dv)
        return vbar(j) * fx(i, j) + SECOND_MOMENT * dv * dv * 1 * dfdv

    def gv(i, j):        # <a f> on v_{j+1/2}: a varies along x
        dadx = (A(i + 1) - A(i - 1)) / (2 * dx)
        dfdx = (fv(i + 1, j) - fv(i - 1, j)) / (2 * dx)
        return A(i) * fv(i, j) + SECOND_MOMENT * dx * dx * dadx * dfdx

    return [[-(gx(i, j) - gx(i - 1, j)) / dx - (gv(i, j) - gv(i, j - 1)) / dv for j in range(nv)]
            for i in range(nx)]


def brute_field(f, dx, dv, qm):
    """a = (q/m) E of the state f: n = dv sum_j f, rho = 1 - n, the periodic
    fourth-order Poisson problem with the zero-mean projection and sum(phi)
    = 0 (one redundant equation replaced by the normalisation), then
    E = -D phi (readings of section 2: 12 dx^2 on the right-hand side,
    E = -grad phi)."""
    nx = len(f)
    rho = [1 - dv * sum(row) for row in f]
    mean = sum(rho) / nx
    stencil = {-2: Fr(1), -1: Fr(-16), 0: Fr(30), 1: Fr(-16), 2: Fr(1)}
    Amat = [[Fr(0)] * nx for _ in range(nx)]
    for i in range(nx):
        for o, c in stencil.items():
            Amat[i][(i + o) % nx] += c
    b = [12 * dx * dx * (r - mean) for r in rho]
    Amat[-1] = [Fr(1)] * nx
    b[-1] = Fr(0)
    phi = solve_exact(Amat, b)
    E = [-(8 * (phi[(i + 1) % nx] - phi[(i - 1) % nx]) - (phi[(i + 2) % nx] - phi[(i - 2) % nx])) / (12 * dx)
         for i in range(nx)]
    return [qm * e for e in E]


def add(f, g, c):
    return [[x + c * y for x, y in zip(rf, rg)] for rf, rg in zip(f, g)]


def brute_rk4(f, dt, slope):
    """Classic RK4 from its tableau (c = 0, 1/2, 1/2, 1; a21 = a32 = 1/2,
    a43 = 1; b = 1/6, 1/3, 1/3, 1/6); slope(state) -> k."""
    k1 = slope(f)
    k2 = slope(add(f, k1, dt / 2))
    k3 = slope(add(f, k2, dt / 2))
    k4 = slope(add(f, k3, dt))
    out = f
    for k, b in ((k1, Fr(1, 6)), (k2, Fr(1, 3)), (k3, Fr(1, 3)), (k4, Fr(1, 6))):
        out = add(out, k, dt * b)
    return out


def rational_case(nx=8, nv=8, seed=7):
    """Random dyadic data (exact in double and in Fraction)."""
    rng = np.random.default_rng(seed)
    f = rng.integers(0, 256, size=(nx, nv)) / 256.0
    a = rng.integers(-64, 65, size=nx) / 128.0
    vghost = np.array([5.0, 3.0, 7.0, 11.0]) / 64.0        # j = -2, -1, nv, nv+1: all distinct
    return f, a, vghost


MESH = dict(x_len=6.0, v_lo=-3.0, v_hi=3.0)    # dx = dv = 0.75 on 8 x 8


def to_fr(f):
    return [[Fr(float(x)) for x in row] for row in f]


def veq_dict(vghost, nv):
    return {-2: Fr(vghost[0]), -1: Fr(vghost[1]), nv: Fr(vghost[2]), nv + 1: Fr(vghost[3])}


def rel_err(approx, exact):
    ex = np.array([[float(x) for x in row] for row in exact])
    return np.abs(np.asarray(approx) - ex).max() / np.abs(ex).max()


def _rhs_case(nx, nv, seed):
    f, a, vg = rational_case(nx, nv, seed)
    dx, dv = MESH["x_len"] / nx, (MESH["v_hi"] - MESH["v_lo"]) / nv
    exact = brute_rhs(to_fr(f), [Fr(float(x)) for x in a], Fr(dx), Fr(dv), Fr(MESH["v_lo"]), veq_dict(vg, nv))
    return f, a, vg, dx, dv, exact


@pytest.mark.parametrize("shape", [(8, 8), (5, 7), (8, 4)])
def test_rhs_every_cell(oracle, shape):
    """vpo_rhs equals the exact rational right-hand side in every cell,
    boundary rows and wrap columns included (8 x 8 as in the brief, and
    ragged meshes where x wraps twice within the stencil)."""
    nx, nv = shape
    f, a, vg, dx, dv, exact = _rhs_case(nx, nv, 7 + nx + nv)
    k = oracle.rhs(f, a, dx, dv, MESH["v_lo"], vg)
    assert rel_err(k, exact) <= 1e-14


def test_boundary_rows_see_each_ghost(oracle):
    """Each of the four ghost values reaches the right rows: changing one
    ghost value changes k only in the rows its stencils touch."""
    nx, nv = 8, 8
    f, a, vg, dx, dv, _ = _rhs_case(nx, nv, 3)
    k0 = oracle.rhs(f, a, dx, dv, MESH["v_lo"], vg)
    touched = {0: {0}, 1: {0, 1}, 2: {nv - 2, nv - 1}, 3: {nv - 1}}
    for g, rows in touched.items():
        vg2 = vg.copy()
        vg2[g] += 0.5
        d = np.abs(oracle.rhs(f, a, dx, dv, MESH["v_lo"], vg2) - k0).max(axis=0)
        assert set(np.nonzero(d > 1e-12)[0]) == rows, (g, d)


def test_rk4_step_fixed_a(oracle):
    """One RK4 step with a prescribed acceleration (the linear map of
    eq. rk4 around L(.; a)) against the exact rational step."""
    nx, nv = 8, 8
    f, a, vg = rational_case(nx, nv, 11)
    p = I.Problem1D(nx, nv, 0.0, MESH["x_len"], MESH["v_lo"], MESH["v_hi"], qm=-1.0)
    p.veq = np.concatenate([vg[:2], np.zeros(nv), vg[2:]])
    o = oracle.Oracle1D.from_problem(p)
    dt = 1.0 / 16.0
    dx, dv = Fr(p.dx), Fr(p.dv)
    af = [Fr(float(x)) for x in a]
    exact = brute_rk4(to_fr(f), Fr(dt), lambda s: brute_rhs(s, af, dx, dv, Fr(p.v_lo), veq_dict(vg, nv)))
    assert rel_err(o.step_fixed_a(f, a, dt), exact) <= 1e-14


def test_field_exact(oracle):
    """Moment, zero-mean projection, Poisson solve and field against the
    exact rational solve of the same equations."""
    nx, nv = 8, 8
    f, _, vg = rational_case(nx, nv, 5)
    p = I.Problem1D(nx, nv, 0.0, MESH["x_len"], MESH["v_lo"], MESH["v_hi"], qm=-1.0)
    p.veq = np.concatenate([vg[:2], np.zeros(nv), vg[2:]])
    o = oracle.Oracle1D.from_problem(p)
    a, _, _, _ = o.constraints(f)
    exact = brute_field(to_fr(f), Fr(p.dx), Fr(p.dv), Fr(-1))
    ex = np.array([float(x) for x in exact])
    assert np.abs(a - ex).max() <= 1e-14 * np.abs(ex).max()


def test_rk4_step_with_field(oracle):
    """One full Vlasov-Poisson RK4 step (the field re-solved at every stage
    state) against the exact rational step, every cell."""
    nx, nv = 8, 8
    f, _, vg = rational_case(nx, nv, 13)
    # a state with a sizeable field: density far from uniform
    f = f * (1.0 + np.arange(nx)[:, None] / 8.0) / 4.0
    p = I.Problem1D(nx, nv, 0.0, MESH["x_len"], MESH["v_lo"], MESH["v_hi"], qm=-1.0)
    p.veq = np.concatenate([vg[:2], np.zeros(nv), vg[2:]])
    o = oracle.Oracle1D.from_problem(p)
    dt = 1.0 / 32.0
    dx, dv = Fr(p.dx), Fr(p.dv)
    ghosts = veq_dict(vg, nv)

    def slope(s):
        return brute_rhs(s, brute_field(s, dx, dv, Fr(-1)), dx, dv, Fr(p.v_lo), ghosts)

    exact = brute_rk4(to_fr(f), Fr(dt), slope)
    assert rel_err(o.step(f, dt), exact) <= 1e-13


# ------------------------------------------------------------------ 2D+2V


def brute_rhs4(f, a, h, v_lo, veq_x, veq_y):
    """2D+2V right-hand side, direction by direction (the 1D+1V formulas of
    section 2 applied along each direction; the product-rule correction
    along every direction in which the advection speed varies).  f is a
    dict (i, j, k, l) -> value on the nx x ny x nvx x nvy mesh; velocity
    ghosts hold veq_x[k] veq_y[l]; a = (ax, ay), each a dict (i, j) -> value."""
    nx, ny, nvx, nvy = f["shape"]
    dx, dy, dvx, dvy = h

    def F(i, j, k, l):
        if k < 0 or k >= nvx or l < 0 or l >= nvy:
            return veq_x[k] * veq_y[l]
        return f[(i % nx, j % ny, k, l)]

    def Ac(c, i, j):
        return a[c][(i % nx, j % ny)]

    def favg(d, i, j, k, l):
        """face average on the upper face of cell (i, j, k, l) along d"""
        e = [0, 0, 0, 0]
        e[d] = 1
        return face([F(i + m * e[0], j + m * e[1], k + m * e[2], l + m * e[3]) for m in (-1, 0, 1, 2)])

    def shift(c, d, s):
        c = list(c)
        c[d] += s
        return c

    def flux(d, c):
        i, j, k, l = c
        if d == 0 or d == 1:       # speed v_d: varies along velocity direction d + 2 only
            dvd = dvx if d == 0 else dvy
            vd = v_lo + ((k if d == 0 else l) + Fr(1, 2)) * dvd
            slope = (favg(d, *shift(c, d + 2, 1)) - favg(d, *shift(c, d + 2, -1))) / (2 * dvd)
            return vd * favg(d, *c) + SECOND_MOMENT * dvd * dvd * slope
        comp = d - 2               # speed a_comp(x, y): varies along x and y
        val = Ac(comp, i, j) * favg(d, *c)
        for dd, hh in ((0, dx), (1, dy)):
            da = (Ac(comp, *shift(c, dd, 1)[:2]) - Ac(comp, *shift(c, dd, -1)[:2])) / (2 * hh)
            df = (favg(d, *shift(c, dd, 1)) - favg(d, *shift(c, dd, -1))) / (2 * hh)
            val += SECOND_MOMENT * hh * hh * da * df
        return val

    out = {}
    for i in range(nx):
        for j in range(ny):
            for k in range(nvx):
                for l in range(nvy):
                    c = [i, j, k, l]
                    out[(i, j, k, l)] = -sum((flux(d, c) - flux(d, shift(c, d, -1))) / h[d] for d in range(4))
    return out


def test_rhs4_every_cell(oracle):
    """The 2D+2V oracle's right-hand side equals the exact rational one in
    every cell, including cells whose stencils reach velocity ghosts in one
    or both velocity directions (products of the two equilibrium factors)."""
    nx, ny, nvx, nvy = 4, 3, 5, 6
    rng = np.random.default_rng(21)
    f = rng.integers(0, 256, size=(nx, ny, nvx, nvy)) / 256.0
    a = rng.integers(-64, 65, size=2 * nx * ny) / 128.0
    veq_x = rng.integers(1, 64, size=nvx + 4) / 64.0
    veq_y = rng.integers(1, 64, size=nvy + 4) / 64.0
    x_len, y_len, v_lo, v_hi = 3.0, 4.5, -3.0, 3.0      # dx = 0.75, dy = 1.5, dvx = 1.2, dvy = 1
    o = oracle.Oracle4D(nx, ny, nvx, nvy, x_len, y_len, v_lo, v_hi, -1.0, veq_x, veq_y)
    k = o.rhs(f, a)
    fd = {"shape": (nx, ny, nvx, nvy)}
    for idx in np.ndindex(nx, ny, nvx, nvy):
        fd[idx] = Fr(float(f[idx]))
    ad = [{(i, j): Fr(float(a[c * nx * ny + i * ny + j])) for i in range(nx) for j in range(ny)} for c in (0, 1)]
    vx = {kk - 2: Fr(float(veq_x[kk])) for kk in range(nvx + 4)}
    vy = {ll - 2: Fr(float(veq_y[ll])) for ll in range(nvy + 4)}
    h = (Fr(x_len / nx), Fr(y_len / ny), Fr((v_hi - v_lo) / nvx), Fr((v_hi - v_lo) / nvy))
    ex = brute_rhs4(fd, ad, h, Fr(v_lo), vx, vy)
    exact = np.array([float(ex[idx]) for idx in np.ndindex(nx, ny, nvx, nvy)]).reshape(k.shape)
    assert np.abs(k - exact).max() <= 1e-14 * np.abs(exact).max()


# ------------------------------------------------------------------ AMR ghost cells


def subcell_weights(R):
    """Averages over the R sub-cells of coarse cell 0 = [0, 1] of the quartic
    whose averages over the cells [-2,-1] .. [2,3] are the data (the
    conservative fifth-order sub-cell interpolation of section 3), derived
    from that definition: rows s, columns j = -2..2."""
    A = [[cell_moment(k, m) for m in range(5)] for k in range(-2, 3)]
    out = []
    for s in range(R):
        lo, hi = Fr(s, R), Fr(s + 1, R)
        row = []
        for q in range(5):
            c = solve_exact(A, [Fr(int(q == r)) for r in range(5)])
            row.append(sum(cm * (hi ** (m + 1) - lo ** (m + 1)) / (m + 1) for m, cm in enumerate(c)) * R)
        out.append(row)
    return out


@pytest.mark.parametrize("R", [2, 4])
def test_amr_ghost_frame(oracle, R):
    """Every ghost cell of a level-1 patch (two layers, corners included)
    equals the definition: outside the velocity box the fine equilibrium
    value of that fine cell index, else the sub-cell interpolation of the
    coarse level along x, then along v, with the coarse level periodic in x
    and its own equilibrium values in its velocity ghosts.  The patches
    touch the lower and the upper velocity boundary and the x seam."""
    ncx, ncv = 8, 8
    rng = np.random.default_rng(30 + R)
    boxes = [{"level": 1, "lo": [0, 0], "hi": [2 * R - 1, 3 * R - 1]},
             {"level": 1, "lo": [4 * R, 5 * R], "hi": [ncx * R - 1, ncv * R - 1]}]
    nfv = ncv * R
    veq_c = rng.integers(1, 64, size=ncv + 4) / 64.0
    veq_f = rng.integers(1, 64, size=nfv + 4) / 64.0
    o = oracle.OracleAMR(ncx, ncv, 4.0, -2.0, 2.0, -1.0, R, boxes, veq_c, veq_f)
    f = rng.integers(0, 256, size=o.size) / 256.0
    fc = f[:ncx * ncv].reshape(ncx, ncv)
    W = subcell_weights(R)

    def coarse(i, j):
        if j < 0 or j >= ncv:
            return Fr(float(veq_c[j + 2]))
        return Fr(float(fc[i % ncx, j]))

    for p, b in enumerate(boxes):
        g = o.ghosted_patch(f, p)
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        nxp, nvp = x1 - x0 + 1, v1 - v0 + 1
        for r in range(-2, nxp + 2):
            for q in range(-2, nvp + 2):
                if 0 <= r < nxp and 0 <= q < nvp:
                    continue
                X, V = x0 + r, v0 + q
                if V < 0 or V >= nfv:
                    want = Fr(float(veq_f[V + 2]))
                else:
                    ci, s = X // R, X % R
                    cj, t = V // R, V % R
                    want = sum(W[t][bb + 2] * sum(W[s][aa + 2] * coarse(ci + aa, cj + bb) for aa in range(-2, 3))
                               for bb in range(-2, 3))
                got = g[r + 2, q + 2]
                assert abs(got - float(want)) <= 1e-14 * max(1.0, abs(float(want))), (p, r, q, got, float(want))


# ------------------------------------------------------------------ planted mistakes


ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

MUTATIONS = {
    "swap ghosts j=-2 and j=-1": ("dst[0] = vghost[0];", "dst[0] = vghost[1];",
                                  "dst[1] = vghost[1];", "dst[1] = vghost[0];"),
    "swap ghosts j=nv and j=nv+1": ("dst[nv + GH] = vghost[2];", "dst[nv + GH] = vghost[3];",
                                    "dst[nv + GH + 1] = vghost[3];", "dst[nv + GH + 1] = vghost[2];"),
    "no x wrap in the ghost rows": ("f + (size_t)wrap(i, nx) * nv", "f + (size_t)(i < 0 ? 0 : (i >= nx ? nx - 1 : i)) * nv",
                                    None, None),
    "acceleration difference not periodic": ("double da = a[wrap(i + 1, nx)] - a[wrap(i - 1, nx)];\n        for (int j = 0; j < nv; ++j) {\n            double vb",
                                             "double da = a[i + 1 < nx ? i + 1 : i] - a[i > 0 ? i - 1 : i];\n        for (int j = 0; j < nv; ++j) {\n            double vb",
                                             None, None),
}


def build_mutant(tmp_path, old1, new1, old2, new2):
    src = open(os.path.join(ORACLE_DIR, "vp_oracle.c")).read()
    for old, new in ((old1, new1), (old2, new2)):
        if old is None:
            continue
        assert src.count(old) == 1, old
        src = src.replace(old, new)
    path = tmp_path / "vp_oracle_mutant.c"
    path.write_text(src)
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-I", ORACLE_DIR,
                    "-o", str(lib), str(path), "-lm"], check=True)
    L = ctypes.CDLL(str(lib))
    D = ctypes.POINTER(ctypes.c_double)
    L.vpo_rhs.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, D, D, D, D]
    L.vpo_rhs.restype = None
    return L


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    """A copy of the oracle with one plausible indexing mistake fails the
    exact comparison of test_rhs_every_cell (so that comparison pins the
    ghost rows and the wrap)."""
    L = build_mutant(tmp_path, *MUTATIONS[name])
    nx, nv = 8, 8
    f, a, vg, dx, dv, exact = _rhs_case(nx, nv, 7 + nx + nv)
    f, a, vg = (np.ascontiguousarray(x, dtype=np.float64) for x in (f, a, vg))
    k = np.empty_like(f)
    D = ctypes.POINTER(ctypes.c_double)
    L.vpo_rhs(nx, nv, dx, dv, MESH["v_lo"], vg.ctypes.data_as(D), f.ctypes.data_as(D), a.ctypes.data_as(D),
              k.ctypes.data_as(D))
    assert rel_err(k, exact) > 1e-6
