"""Pins of the multi-level oracle (oracle/vp_oracle_hier.c: L <= 4 levels,
a refinement ratio per level and direction, touching patches).

- Two levels with one ratio: the same constraint, right-hand side and step
  as the two-level oracle (itself pinned), on separated and touching
  layouts and for ratios 2 and 4.
- Full coverage: three and four levels that each cover the whole domain,
  with the section-4 ratios [2,4], [4,2], [2,2], advance the finest level
  exactly like the uniform finest mesh; every coarser level becomes the
  mean of the next finer one.
- Ghost cells: with exact cell averages of a polynomial of degree four in
  x and in v on every level, every ghost cell of every patch (copied from a
  touching patch, or interpolated from the parent level across two parent
  patches, anisotropic ratios) is the exact cell average.
- Reduction: patches whose data are the interpolation of their parent
  level leave the charge density unchanged (the finest level of three, and
  an anisotropic second level), so the masks and each level's velocity
  cell size are right.
- Composite mass is conserved by a three-level anisotropic step with
  touching patches; splitting a level-2 patch into two touching patches
  leaves the step unchanged.
Each fails for a planted mistake of its kind (swapped ratios, a wrong
velocity cell size or mask, a missing flux correction, an interpolated
instead of copied ghost).
"""
import math

import numpy as np
import pytest
from numpy.polynomial import Polynomial

import vp_inputs as I

X_LEN, V_LO, V_HI = 4 * math.pi, -8.0, 8.0


def box(level, x0, v0, x1, v1):
    return {"level": level, "lo": [x0, v0], "hi": [x1, v1]}


def landau_hier(oracle, ncx, ncv, ratios, boxes, noise=0.02, seed=0, eps=0.05):
    f, veqs = I.hier_state(I.maxwellian, 0.0, X_LEN, V_LO, V_HI, eps, 0.5, (ncx, ncv), ratios, boxes)
    f = f * (1 + noise * np.random.default_rng(seed).random(f.size))
    o = oracle.OracleHier(len(ratios) + 1, ncx, ncv, X_LEN, V_LO, V_HI, -1.0, ratios, boxes, veqs)
    return o, f, veqs


TWO_LEVEL = {
    "separated_r4": (32, 48, 4, [box(1, 16, 40, 39, 63), box(1, 60, 68, 83, 87), box(1, 0, 96, 15, 111)]),
    "touching_r4": (32, 48, 4, [box(1, 16, 40, 39, 63), box(1, 40, 40, 55, 63), box(1, 24, 64, 31, 79),
                                box(1, 0, 96, 15, 111), box(1, 112, 100, 127, 115)]),
    "edges_r2": (24, 45, 2, [box(1, 6, 20, 17, 33), box(1, 0, 50, 9, 61), box(1, 20, 0, 27, 7),
                             box(1, 36, 80, 41, 89), box(1, 0, 20, 5, 33)]),
}


@pytest.mark.parametrize("name", list(TWO_LEVEL))
def test_two_levels_match_the_two_level_oracle(oracle, name):
    ncx, ncv, R, boxes = TWO_LEVEL[name]
    o, f, veqs = landau_hier(oracle, ncx, ncv, [(R, R)], boxes)
    b2 = [{"level": 1, "lo": b["lo"], "hi": b["hi"]} for b in boxes]
    o2 = oracle.OracleAMR(ncx, ncv, X_LEN, V_LO, V_HI, -1.0, R, b2, veqs[0], veqs[1])
    assert o.size == o2.size
    scale = np.abs(f).max()
    np.testing.assert_allclose(o.reduce_mask(f), o2.reduce_mask(f), rtol=1e-14, atol=1e-15)
    a, E = o.constraints(f)
    a2, E2 = o2.constraints(f)
    np.testing.assert_allclose(a, a2, rtol=0, atol=1e-13 * np.abs(a2).max())
    k, k2 = o.rhs(f, a2), o2.rhs(f, a2)
    assert np.abs(k - k2).max() <= 1e-13 * np.abs(k2).max()
    dt = 0.004
    g, g2 = o.step(f, dt), o2.step(f, dt)
    assert np.abs(g - g2).max() <= 1e-14 * scale


def tile_level(nx, nv, xcuts, vcuts, level):
    xs, vs = [0] + xcuts + [nx], [0] + vcuts + [nv]
    return [box(level, xs[i], vs[j], xs[i + 1] - 1, vs[j + 1] - 1)
            for i in range(len(xs) - 1) for j in range(len(vs) - 1)]


def unpack_level(o, f, boxes, level):
    F = np.full((o.nx[level], o.nv[level]), np.nan)
    for p, b in enumerate(boxes):
        if b["level"] != level:
            continue
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        nx, nv = x1 - x0 + 1, v1 - v0 + 1
        F[x0:x1 + 1, v0:v1 + 1] = f[o.offset(p): o.offset(p) + nx * nv].reshape(nx, nv)
    return F


@pytest.mark.parametrize("ratios", [[(2, 4), (4, 2)], [(2, 4), (4, 2), (2, 2)]])
def test_full_coverage_equals_uniform_finest_mesh(oracle, ratios):
    ncx, ncv = 4, 4
    nx, nv = [ncx], [ncv]
    for rx, rv in ratios:
        nx.append(nx[-1] * rx)
        nv.append(nv[-1] * rv)
    boxes = []
    for lv in range(1, len(ratios) + 1):
        rx, rv = ratios[lv - 1]
        boxes += tile_level(nx[lv], nv[lv], [rx * (nx[lv - 1] // 2 - 1)], [rv * (nv[lv - 1] // 3)], lv)
    L = len(ratios) + 1
    # data: the finest level is a noisy field; coarser levels its means
    rng = np.random.default_rng(7)
    veqs = [I.cell_average_1d(I.maxwellian, V_LO, V_HI, n, first=-2, count=n + 4) for n in nv]
    xf = 1 + 0.05 * I.cos_cell_average(0.0, X_LEN, nx[-1], 0.5)
    F = [None] * L
    F[-1] = xf[:, None] * veqs[-1][None, 2:-2] * (1 + 0.02 * rng.random((nx[-1], nv[-1])))
    for lv in range(L - 2, -1, -1):
        rx, rv = ratios[lv]
        F[lv] = F[lv + 1].reshape(nx[lv], rx, nv[lv], rv).mean(axis=(1, 3))
    parts = [F[0].ravel()]
    for b in boxes:
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        parts.append(F[b["level"]][x0:x1 + 1, v0:v1 + 1].ravel())
    f = np.concatenate(parts)
    o = oracle.OracleHier(L, ncx, ncv, X_LEN, V_LO, V_HI, -1.0, ratios, boxes, veqs)
    dt = 0.5 / (V_HI / (X_LEN / nx[-1]) + 0.1 / (16.0 / nv[-1]))
    g = o.step(f, dt)
    vg = veqs[-1]
    uni = oracle.Oracle1D(nx[-1], nv[-1], X_LEN, V_LO, V_HI, -1.0, np.array([vg[0], vg[1], vg[-2], vg[-1]]))
    Fu = uni.step(F[-1], dt)
    G = [None] * L
    G[0] = g[: ncx * ncv].reshape(ncx, ncv)
    for lv in range(1, L):
        G[lv] = unpack_level(o, g, boxes, lv)
    assert np.abs(G[-1] - Fu).max() <= 1e-13 * np.abs(Fu).max()
    for lv in range(L - 1):
        rx, rv = ratios[lv]
        np.testing.assert_allclose(G[lv], G[lv + 1].reshape(nx[lv], rx, nv[lv], rv).mean(axis=(1, 3)),
                                   rtol=1e-13, atol=0)


# a polynomial of degree four in x and in v, and its exact cell averages
PX = Polynomial([1.0, 0.3, -0.05, 0.004, -0.0002])
PV = Polynomial([2.0, -0.4, 0.07, 0.006, -0.0004])


def poly_avgs(n_x, n_v, dx, dv, v_lo):
    ix, iv = PX.integ(), PV.integ()
    xe = np.arange(n_x + 1) * dx
    ve = v_lo + np.arange(n_v + 1) * dv
    ax = (ix(xe[1:]) - ix(xe[:-1])) / dx
    av = (iv(ve[1:]) - iv(ve[:-1])) / dv
    return ax[:, None] * av[None, :]


def test_ghost_cells_exact_for_quartics(oracle):
    """Level 0: 16 x 16 on [0, 16) x [-8, 8); ratios [2,4] then [4,2]; two
    touching level-1 patches and a level-2 patch whose interpolated ghosts
    read both; everything three or more cells from the periodic seam and
    the velocity boundary, so only the polynomial is seen."""
    ratios = [(2, 4), (4, 2)]
    ncx = ncv = 16
    x_len = 16.0
    boxes = [box(1, 8, 16, 19, 39), box(1, 20, 16, 23, 39), box(2, 48, 40, 79, 71)]
    nx, nv = [16, 32, 128], [16, 64, 128]
    full = [poly_avgs(nx[lv], nv[lv], x_len / nx[lv], 16.0 / nv[lv], V_LO) for lv in range(3)]
    parts = [full[0].ravel()]
    for b in boxes:
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        parts.append(full[b["level"]][x0:x1 + 1, v0:v1 + 1].ravel())
    f = np.concatenate(parts)
    veqs = [np.zeros(n + 4) for n in nv]          # never read: all ghosts are inside the velocity box
    o = oracle.OracleHier(3, ncx, ncv, x_len, V_LO, V_HI, -1.0, ratios, boxes, veqs)
    for p, b in enumerate(boxes):
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        g = o.ghosted(f, p)
        want = full[b["level"]][x0 - 2:x1 + 3, v0 - 2:v1 + 3]
        assert np.abs(g - want).max() <= 1e-12 * np.abs(want).max(), p


def interp_patch(oracle, parent, rx, rv, x0, v0, x1, v1):
    """The x-then-v sub-cell interpolation of a parent array (no periodic
    wrap needed: the caller stays inside) onto fine cells [x0..x1]x[v0..v1]."""
    Bx, Bv = oracle.interp_weights(rx), oracle.interp_weights(rv)
    out = np.empty((x1 - x0 + 1, v1 - v0 + 1))
    for X in range(x0, x1 + 1):
        ci, s = divmod(X, rx)
        gx = sum(Bx[s, a + 2] * parent[ci + a, :] for a in range(-2, 3))
        for V in range(v0, v1 + 1):
            cj, t = divmod(V, rv)
            out[X - x0, V - v0] = sum(Bv[t, b + 2] * gx[cj + b] for b in range(-2, 3))
    return out


def test_reduction_invariant_under_interpolated_refinement(oracle):
    ratios = [(2, 4), (4, 2)]
    ncx, ncv = 16, 16
    lvl1 = [box(1, 4, 16, 23, 47), box(1, 24, 16, 27, 47)]
    rng = np.random.default_rng(3)
    f0 = rng.random((ncx, ncv))
    F1 = rng.random((32, 64))                      # level-1 data where patches are (arbitrary)
    veqs = [I.cell_average_1d(I.maxwellian, V_LO, V_HI, n, first=-2, count=n + 4) for n in (16, 64, 128)]
    base = [f0.ravel()] + [F1[b["lo"][0]:b["hi"][0] + 1, b["lo"][1]:b["hi"][1] + 1].ravel() for b in lvl1]
    oA = oracle.OracleHier(3, ncx, ncv, X_LEN, V_LO, V_HI, -1.0, ratios, lvl1, veqs)
    nA = oA.reduce_mask(np.concatenate(base))
    # level 2 over part of level 1, holding the interpolation of level 1
    l2 = box(2, 40, 40, 87, 79)
    P1 = np.zeros((32, 64))
    for b in lvl1:
        P1[b["lo"][0]:b["hi"][0] + 1, b["lo"][1]:b["hi"][1] + 1] = F1[b["lo"][0]:b["hi"][0] + 1,
                                                                       b["lo"][1]:b["hi"][1] + 1]
    d2 = interp_patch(oracle, P1, 4, 2, 40, 40, 87, 79)
    oB = oracle.OracleHier(3, ncx, ncv, X_LEN, V_LO, V_HI, -1.0, ratios, lvl1 + [l2], veqs)
    nB = oB.reduce_mask(np.concatenate(base + [d2.ravel()]))
    np.testing.assert_allclose(nB, nA, rtol=1e-13, atol=1e-14)
    # an anisotropic second level over the interpolation of level 0
    fz = np.tile(f0, (3, 1))[ncx - 2:2 * ncx + 2]   # level 0 with two periodic rows on each side
    o1 = oracle.OracleHier(2, ncx, ncv, X_LEN, V_LO, V_HI, -1.0, [(2, 4)], [], veqs[:2])
    d1 = interp_patch(oracle, np.pad(fz, ((0, 0), (2, 2)), mode="edge"), 2, 4, 4 + 4, 16 + 8, 23 + 4, 47 + 8)
    o2 = oracle.OracleHier(2, ncx, ncv, X_LEN, V_LO, V_HI, -1.0, [(2, 4)], [box(1, 4, 16, 23, 47)], veqs[:2])
    np.testing.assert_allclose(o2.reduce_mask(np.concatenate([f0.ravel(), d1.ravel()])),
                               o1.reduce_mask(f0.ravel()), rtol=1e-13, atol=1e-14)


def composite_mass(o, f, boxes, ratios):
    L = o.L
    dx = [X_LEN / n for n in o.nx]
    dv = [16.0 / n for n in o.nv]
    cov = [np.zeros((o.nx[lv], o.nv[lv]), bool) for lv in range(L)]
    for b in boxes:
        lv = b["level"]
        rx, rv = ratios[lv - 1]
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        cov[lv - 1][x0 // rx:(x1 + 1) // rx, v0 // rv:(v1 + 1) // rv] = True
    m = (f[: o.ncx * o.ncv].reshape(o.ncx, o.ncv)[~cov[0]]).sum() * dx[0] * dv[0]
    for p, b in enumerate(boxes):
        lv = b["level"]
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        d = f[o.offset(p): o.offset(p) + (x1 - x0 + 1) * (v1 - v0 + 1)].reshape(x1 - x0 + 1, v1 - v0 + 1)
        m += d[~cov[lv][x0:x1 + 1, v0:v1 + 1]].sum() * dx[lv] * dv[lv]
    return m


HIER3 = [box(1, 8, 24, 31, 71), box(1, 32, 24, 43, 71), box(1, 0, 32, 7, 55), box(1, 56, 40, 63, 55),
         box(2, 56, 64, 119, 119), box(2, 120, 64, 143, 119), box(2, 240, 88, 255, 95)]


def test_three_level_step_conserves_composite_mass(oracle):
    ratios = [(2, 4), (4, 2)]
    o, f, _ = landau_hier(oracle, 32, 24, ratios, HIER3, seed=5)
    m0 = composite_mass(o, f, HIER3, ratios)
    g = f
    for _ in range(3):
        g = o.step(g, 0.01)
    assert abs(composite_mass(o, g, HIER3, ratios) - m0) <= 1e-13 * m0
    assert np.abs(g - f).max() > 1e-6


def test_level_two_split_is_invariant(oracle):
    ratios = [(2, 4), (4, 2)]
    whole = HIER3
    split = HIER3[:4] + [box(2, 56, 64, 87, 119), box(2, 88, 64, 143, 91), box(2, 88, 92, 143, 119),
                         HIER3[6]]
    o1, f1, _ = landau_hier(oracle, 32, 24, ratios, whole, seed=9)
    o2, f2, _ = landau_hier(oracle, 32, 24, ratios, split, seed=9, noise=0.0)
    # the same data on both layouts: level-2 values moved from the whole patches to the split ones
    F2 = unpack_level(o1, f1, whole, 2)
    parts = [f1[: o1.offset(4)]]
    for b in split[4:]:
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        parts.append(F2[x0:x1 + 1, v0:v1 + 1].ravel())
    f2 = np.concatenate(parts)
    dt = 0.01
    g1, g2 = o1.step(f1, dt), o2.step(f2, dt)
    scale = np.abs(g1).max()
    assert np.abs(g1[: o1.offset(4)] - g2[: o2.offset(4)]).max() <= 1e-14 * scale
    G1, G2 = unpack_level(o1, g1, whole, 2), unpack_level(o2, g2, split, 2)
    cov = ~np.isnan(G1)
    assert np.abs(G1[cov] - G2[cov]).max() <= 1e-14 * scale


def test_bad_hierarchies_are_rejected(oracle):
    veqs = [np.zeros(n + 4) for n in (24, 96, 192)]
    ratios = [(2, 4), (4, 2)]
    with pytest.raises(ValueError, match="code 2"):        # not aligned to the ratio
        oracle.OracleHier(3, 32, 24, X_LEN, V_LO, V_HI, -1.0, ratios, [box(1, 9, 24, 31, 71)], veqs)
    with pytest.raises(ValueError, match="code 3"):        # overlapping on a level
        oracle.OracleHier(3, 32, 24, X_LEN, V_LO, V_HI, -1.0, ratios,
                          [box(1, 8, 24, 31, 71), box(1, 30, 24, 43, 71)], veqs)
    with pytest.raises(ValueError, match="code 4"):        # level 2 too close to the edge of level 1
        oracle.OracleHier(3, 32, 24, X_LEN, V_LO, V_HI, -1.0, ratios,
                          [box(1, 8, 24, 31, 71), box(2, 32, 48, 63, 79)], veqs)


# ---- regridding pieces of a multi-level hierarchy -------------------------

def test_tag_values_equal_the_single_level_criterion(oracle):
    """Level 0, and a level 1 that the patches tile completely, give the
    single-level criterion of the same array bit for bit."""
    ratios = [(2, 4)]
    ncx, ncv = 8, 6
    boxes = tile_level(16, 24, [6], [8], 1)
    o, f, veqs = landau_hier(oracle, ncx, ncv, ratios, boxes, noise=0.05, seed=4)
    for lv in range(2):
        arr = o.level_array(f, lv)
        vg = veqs[lv]
        want = oracle.tag_values(arr, X_LEN / o.nx[lv], 16.0 / o.nv[lv], np.array([vg[0], vg[1], vg[-2], vg[-1]]))
        got = o.tag_values(f, lv)
        assert np.array_equal(got, want), lv


def test_tag_values_only_where_the_level_has_patches(oracle):
    o, f, _ = landau_hier(oracle, 32, 24, [(2, 4), (4, 2)], HIER3, seed=2)
    t1 = o.tag_values(f, 1)
    held = ~np.isnan(o.level_array(f, 1))
    assert np.array_equal(~np.isnan(t1), held)
    assert (t1[held] > 0).all()


@pytest.mark.parametrize("R", [2, 4])
def test_prolong_box_equals_the_two_level_prolongation(oracle, R):
    ncx, ncv = 16, 12
    boxes = [box(1, 4 * R, 2 * R, 9 * R - 1, 8 * R - 1)]
    o, f, veqs = landau_hier(oracle, ncx, ncv, [(R, R)], boxes, noise=0.1, seed=8)
    fc = f[: ncx * ncv].reshape(ncx, ncv)
    vg = veqs[0]
    b = boxes[0]
    want = oracle.prolong_box(fc, np.array([vg[0], vg[1], vg[-2], vg[-1]]), R,
                              (b["lo"][0], b["lo"][1], b["hi"][0], b["hi"][1]))
    got = o.prolong_box(f, 1, boxes[0]["lo"], boxes[0]["hi"])
    assert np.array_equal(got, want)


def test_prolong_box_anisotropic_conserves_and_reads_parent_patches(oracle):
    """Level 2 ([4,2] from level 1) prolonged from two touching level-1
    patches: every parent cell's mean is kept exactly (conservation), and a
    smooth parent is reproduced to the scheme's order."""
    o, f, _ = landau_hier(oracle, 32, 24, [(2, 4), (4, 2)], HIER3, seed=12)
    lo, hi = [56, 64], [143, 119]                       # across level-1 patches 0 and 1
    fine = o.prolong_box(f, 2, lo, hi)
    parent = o.level_array(f, 1)[lo[0] // 4:(hi[0] + 1) // 4, lo[1] // 2:(hi[1] + 1) // 2]
    means = fine.reshape(parent.shape[0], 4, parent.shape[1], 2).mean(axis=(1, 3))
    np.testing.assert_allclose(means, parent, rtol=1e-14, atol=0)
    with pytest.raises(ValueError):
        o.prolong_box(f, 2, [0, 0], [31, 31])            # level 1 does not hold those parents


def test_regrid_transfer_keeps_old_cells_and_conserves(oracle):
    ratios = [(2, 4), (4, 2)]
    o, f, veqs = landau_hier(oracle, 32, 24, ratios, HIER3, seed=3)
    new_boxes = [box(1, 8, 24, 43, 71), box(1, 0, 32, 7, 55), box(1, 56, 32, 63, 63),
                 box(2, 60, 60, 131, 119), box(2, 240, 88, 255, 95)]
    n = oracle.OracleHier(3, 32, 24, X_LEN, V_LO, V_HI, -1.0, ratios, new_boxes, veqs)
    g = oracle.hier_regrid_transfer(o, f, n)
    np.testing.assert_array_equal(g[: 32 * 24], f[: 32 * 24])
    for lv in (1, 2):
        old, new = o.level_array(f, lv), n.level_array(g, lv)
        kept = ~np.isnan(old) & ~np.isnan(new)
        assert np.array_equal(new[kept], old[kept])
    # new level-1 cells that no old patch held keep the parent's mean
    new1, old1 = n.level_array(g, 1), o.level_array(f, 1)
    fresh = ~np.isnan(new1) & np.isnan(old1)
    assert fresh.any()
    m = new1.reshape(32, 2, 24, 4).mean(axis=(1, 3))
    c = f[: 32 * 24].reshape(32, 24)
    whole = fresh.reshape(32, 2, 24, 4).all(axis=(1, 3))
    np.testing.assert_allclose(m[whole], c[whole], rtol=1e-14)


def test_stability_limit_closed_form(oracle):
    ratios = [(2, 4), (4, 2)]
    o, f, _ = landau_hier(oracle, 32, 24, ratios, HIER3, seed=3)
    a = np.zeros(o.field_elems)
    lim = oracle.hier_stability_limit(o, a, V_LO, V_HI)
    # a = 0: the fastest patch is level 2, |v| up to |v_lo + 88 dv_2| or so; the rate is max |v| / dx over patches
    rates = [8.0 / (X_LEN / 32)]
    for b in HIER3:
        lv = b["level"]
        dv = 16.0 / o.nv[lv]
        vmax = max(abs(V_LO + b["lo"][1] * dv), abs(V_LO + (b["hi"][1] + 1) * dv))
        rates.append(vmax / (X_LEN / o.nx[lv]))
    assert abs(lim - oracle.linear_stability_courant() / max(rates)) <= 1e-15 * lim
