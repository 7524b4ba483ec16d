"""Seeded synthetic inputs for the Vlasov-Poisson workloads.

This module only builds input arrays: exact cell averages of analytic
initial conditions, the equilibrium values used in the velocity ghost
cells, random states for parity tests, and the seeded AMR patch layout.
It contains none of the discretisation's arithmetic (no face averages,
fluxes, moments, Poisson solve or time stepping), so both the CPU oracle
and the GPU path can consume what it produces.

Cell averages are exact: the x-factor of each initial condition is a
cosine whose cell average has a closed form, and the velocity factor is
integrated per cell with a 16-point Gauss-Legendre rule (relative error
far below 1e-15 for the smooth Maxwellian-type profiles used here).
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field

import numpy as np

_GL_NODES, _GL_WEIGHTS = np.polynomial.legendre.leggauss(16)
SQRT_2PI = math.sqrt(2.0 * math.pi)


def maxwellian(v):
    return np.exp(-0.5 * np.asarray(v) ** 2) / SQRT_2PI


def two_stream_profile(v):
    v = np.asarray(v)
    return v * v * np.exp(-0.5 * v * v) / SQRT_2PI


def bump_on_tail_profile(v):
    v = np.asarray(v)
    return (0.9 * np.exp(-0.5 * v * v) + 0.2 * np.exp(-4.0 * (v - 4.5) ** 2)) / SQRT_2PI


PROFILES = {
    "maxwellian": maxwellian,
    "two_stream": two_stream_profile,
    "bump_on_tail": bump_on_tail_profile,
}


def cell_average_1d(fn, lo: float, hi: float, n: int, first: int = 0, count: int | None = None):
    """Exact (quadrature) cell averages of fn over cells first..first+count-1
    of the uniform mesh of n cells on [lo, hi]; indices may lie outside
    [0, n) to produce ghost-cell values."""
    if count is None:
        count = n
    h = (hi - lo) / n
    j = np.arange(first, first + count, dtype=np.float64)
    left = lo + j * h
    mid = left + 0.5 * h
    pts = mid[:, None] + 0.5 * h * _GL_NODES[None, :]
    vals = fn(pts)
    return 0.5 * (vals * _GL_WEIGHTS[None, :]).sum(axis=1)


def cos_cell_average(x_lo: float, x_len: float, nx: int, k: float):
    """Cell averages of cos(k x) on the uniform periodic mesh of nx cells."""
    dx = x_len / nx
    xl = x_lo + np.arange(nx, dtype=np.float64) * dx
    xr = xl + dx
    return (np.sin(k * xr) - np.sin(k * xl)) / (k * dx)


@dataclass
class Problem1D:
    """1D+1V single-level problem on [x_lo, x_lo + x_len) x [v_lo, v_hi]."""
    nx: int
    nv: int
    x_lo: float
    x_len: float
    v_lo: float
    v_hi: float
    qm: float = -1.0
    profile: str = "maxwellian"
    eps: float = 0.01
    k: float = 0.5
    veq: np.ndarray = field(default=None, repr=False)   # nv + 4 values, j = -2 .. nv+1

    def __post_init__(self):
        if self.veq is None:
            self.veq = cell_average_1d(PROFILES[self.profile], self.v_lo, self.v_hi,
                                       self.nv, first=-2, count=self.nv + 4)

    @property
    def dx(self):
        return self.x_len / self.nx

    @property
    def dv(self):
        return (self.v_hi - self.v_lo) / self.nv

    @property
    def vghost(self):
        """Equilibrium cell averages of the four velocity ghost cells
        j = -2, -1, nv, nv+1."""
        return np.array([self.veq[0], self.veq[1], self.veq[-2], self.veq[-1]])

    def initial_state(self):
        """Exact cell averages of (1 + eps cos(k x)) g(v)."""
        xfac = 1.0 + self.eps * cos_cell_average(self.x_lo, self.x_len, self.nx, self.k)
        return np.ascontiguousarray(xfac[:, None] * self.veq[None, 2:self.nv + 2])


def landau_64():
    """Landau damping, 64x64, x in [0, 4 pi), v in [-8, 8], k = 0.5, eps = 0.01."""
    return Problem1D(64, 64, 0.0, 4.0 * math.pi, -8.0, 8.0, profile="maxwellian", eps=0.01, k=0.5)


def landau(nx, nv, eps=0.01):
    return Problem1D(nx, nv, 0.0, 4.0 * math.pi, -8.0, 8.0, profile="maxwellian", eps=eps, k=0.5)


def two_stream(nx=4096, nv=4096):
    """Two-stream instability, x in [0, 10 pi), v in [-8, 8], k = 0.2, eps = 1e-3."""
    return Problem1D(nx, nv, 0.0, 10.0 * math.pi, -8.0, 8.0, profile="two_stream", eps=1e-3, k=0.2)


def adjoint_setup(nx: int = 512, nv: int = 512, seed: int = 0):
    """Adjoint workload: Landau mesh, f0_ij = (1 + c_i + p_i) g_j with c the
    exact cell averages of 0.01 cos(0.5 x) and the perturbation profile
    p ~ N(0, sigma = 1e-3) (seeded)."""
    prob = landau(nx, nv, eps=0.0)
    c = 0.01 * cos_cell_average(prob.x_lo, prob.x_len, nx, 0.5)
    p = np.random.default_rng(seed).normal(0.0, 1e-3, nx)
    return prob, c, p


def adjoint_directions(nx: int, count: int = 8, seed: int = 1):
    """Unit-norm random directions for finite-difference checks."""
    d = np.random.default_rng(seed).normal(size=(count, nx))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def random_state(nx: int, nv: int, seed: int = 1234):
    """Random parity input: f ~ U[0, 1), a ~ N(0, 0.1)."""
    rng = np.random.default_rng(seed)
    f = rng.random((nx, nv))
    a = rng.normal(0.0, 0.1, nx)
    return f, a


def stable_dt(prob: Problem1D, a_max: float, cfl: float = 0.5):
    """Time step with nu = dt (max|v|/dx + max|a|/dv) equal to cfl, where
    max|v| is taken over the velocity cell faces."""
    vmax = max(abs(prob.v_lo), abs(prob.v_hi))
    return cfl / (vmax / prob.dx + a_max / prob.dv)


# ---------------------------------------------------------------- 2D+2V


@dataclass
class Problem2D:
    """2D+2V single-level problem, f stored as [x][y][vx][vy]."""
    nx: int
    ny: int
    nvx: int
    nvy: int
    x_len: float = 4.0 * math.pi
    y_len: float = 4.0 * math.pi
    v_lo: float = -6.0
    v_hi: float = 6.0
    qm: float = -1.0
    eps: float = 0.01
    k: float = 0.5

    @property
    def veq_x(self):
        return cell_average_1d(maxwellian, self.v_lo, self.v_hi, self.nvx, first=-2, count=self.nvx + 4)

    @property
    def veq_y(self):
        return cell_average_1d(maxwellian, self.v_lo, self.v_hi, self.nvy, first=-2, count=self.nvy + 4)

    def initial_state(self):
        """Exact cell averages of (1 + eps (cos kx + cos ky)) M(vx) M(vy)."""
        cx = cos_cell_average(0.0, self.x_len, self.nx, self.k)
        cy = cos_cell_average(0.0, self.y_len, self.ny, self.k)
        xy = 1.0 + self.eps * (cx[:, None] + cy[None, :])
        gx = self.veq_x[2:self.nvx + 2]
        gy = self.veq_y[2:self.nvy + 2]
        return np.ascontiguousarray(xy[:, :, None, None] * gx[None, None, :, None] * gy[None, None, None, :])


def amr4d_state(ncells, R, boxes, eps=0.05, k=0.5, x_len=4.0 * math.pi, y_len=4.0 * math.pi, v_lo=-6.0,
                v_hi=6.0):
    """Two-level 2D+2V state: exact cell averages of (1 + eps (cos kx +
    cos ky)) M(vx) M(vy) on level 0 (ncells = (nx, ny, nvx, nvy)) and on
    every level-1 patch (ratio R in every direction; boxes with 4-entry
    lo/hi), concatenated [level 0][patches in order]; returns (state, gxc,
    gyc, gxf, gyf), the 1D equilibria with two ghosts per side."""
    c = Problem2D(*ncells, x_len=x_len, y_len=y_len, v_lo=v_lo, v_hi=v_hi, eps=eps, k=k)
    fpb = Problem2D(*[n * R for n in ncells], x_len=x_len, y_len=y_len, v_lo=v_lo, v_hi=v_hi, eps=eps, k=k)
    parts = [c.initial_state().ravel()]
    ff = None
    for b in boxes:
        if ff is None:
            ff = fpb.initial_state()
        sl = tuple(slice(b["lo"][d], b["hi"][d] + 1) for d in range(4))
        parts.append(np.ascontiguousarray(ff[sl]).ravel())
    return np.concatenate(parts), c.veq_x, c.veq_y, fpb.veq_x, fpb.veq_y


def amr4d_boxes(seed: int = 0, ncells=(32, 32, 32, 32), ratio: int = 2, npatch: int = 6, sides=(4, 8, 12),
                v_band=(0.25, 0.75), touch: bool = True):
    """Seeded level-1 patches of a two-level 2D+2V hierarchy (4-entry lo/hi in
    level-1 indices): sides drawn from `sides` coarse cells per direction,
    corners on coarse cells (so aligned to the ratio), x and y anywhere (no
    wrap inside a patch), velocity corners inside the central fraction
    v_band of each velocity range; disjoint, touching allowed.  With touch,
    the second patch is placed against the first along x when it fits."""
    rng = np.random.default_rng(seed)
    boxes = []
    tries = 0
    while len(boxes) < npatch and tries < 10000:
        tries += 1
        lo, hi = [], []
        for d in range(4):
            w = int(rng.choice(sides))
            if d < 2:
                if w > ncells[d]:
                    w = ncells[d]
                c0 = int(rng.integers(0, ncells[d] - w + 1))
            else:
                a = int(math.ceil(v_band[0] * ncells[d]))
                bnd = int(math.floor(v_band[1] * ncells[d]))
                w = min(w, bnd - a)
                c0 = int(rng.integers(a, bnd - w + 1))
            if touch and len(boxes) == 1 and d == 0:
                prev = boxes[0]
                c1 = (prev["hi"][0] + 1) // ratio
                if c1 + w <= ncells[0]:
                    c0 = c1
            lo.append(c0 * ratio)
            hi.append((c0 + w) * ratio - 1)
        clash = any(all(max(lo[d], b["lo"][d]) <= min(hi[d], b["hi"][d]) for d in range(4)) for b in boxes)
        if not clash:
            boxes.append({"level": 1, "lo": lo, "hi": hi})
    return boxes


# ---------------------------------------------------------------- AMR layout


def amr_boxes(seed: int = 0, coarse=(512, 512), ratio: int = 4, npatch: int = 40,
              side_lo: int = 16, side_hi: int = 128, v_lo: float = -8.0, v_hi: float = 8.0,
              v_band: float = 3.0, gap: int = 0):
    """Seeded layout of level-1 patches (inclusive lo/hi in the level-1 index
    space): sides drawn uniformly from {side_lo, side_lo+4, ..., side_hi},
    corners aligned to the refinement ratio, confined to the velocity band
    |v| < v_band, not wrapping in x.  Patches grown by `gap` fine cells must
    not intersect; draws that violate this are rejected.  gap = 0: disjoint,
    touching allowed (seed 0: 40 patches, two touching pairs)."""
    rng = np.random.default_rng(seed)
    nxf, nvf = coarse[0] * ratio, coarse[1] * ratio
    dvf = (v_hi - v_lo) / nvf
    band_lo = int(math.ceil((-v_band - v_lo) / dvf))
    band_hi = int(math.floor((v_band - v_lo) / dvf))       # exclusive
    sides = np.arange(side_lo, side_hi + 1, 4)
    boxes = []
    tries = 0
    while len(boxes) < npatch:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place patches")
        wx = int(rng.choice(sides))
        wv = int(rng.choice(sides))
        if wv > band_hi - band_lo:
            continue
        x0 = int(rng.integers(0, (nxf - wx) // ratio + 1)) * ratio
        v0 = int(rng.integers(-(-band_lo // ratio), (band_hi - wv) // ratio + 1)) * ratio
        lo = (x0, v0)
        hi = (x0 + wx - 1, v0 + wv - 1)
        if v0 < band_lo or hi[1] >= band_hi:
            continue
        ok = all(hi[0] + gap < b[0][0] or b[1][0] + gap < lo[0] or hi[1] + gap < b[0][1] or b[1][1] + gap < lo[1]
                 for b in boxes)
        if ok:
            boxes.append((lo, hi))
    return [{"level": 1, "lo": list(b[0]), "hi": list(b[1])} for b in boxes]


def _amr_state(profile, x_lo, x_len, v_lo, v_hi, eps, k, boxes, coarse, ratio):
    """Exact cell averages of (1 + eps cos(k x)) profile(v) on the coarse
    level (all cells) and on every patch, concatenated in the state layout
    [coarse][patch 0][patch 1]...; returns (state, veq_c, veq_f)."""
    ncx, ncv = coarse
    veq_c = cell_average_1d(profile, v_lo, v_hi, ncv, first=-2, count=ncv + 4)
    nvf = ncv * ratio
    veq_f = cell_average_1d(profile, v_lo, v_hi, nvf, first=-2, count=nvf + 4)
    xc = 1.0 + eps * cos_cell_average(x_lo, x_len, ncx, k)
    xf = 1.0 + eps * cos_cell_average(x_lo, x_len, ncx * ratio, k)
    parts = [(xc[:, None] * veq_c[None, 2:ncv + 2]).ravel()]
    for b in boxes:
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        parts.append((xf[x0:x1 + 1, None] * veq_f[None, 2 + v0:2 + v1 + 1]).ravel())
    return np.concatenate(parts), veq_c, veq_f


def amr_landau(boxes, coarse=(512, 512), ratio: int = 4, eps: float = 0.01, k: float = 0.5):
    """Two-level Landau problem on [0, 4 pi) x [-8, 8]: (1 + eps cos(k x)) M(v);
    returns (state, veq_c, veq_f)."""
    return _amr_state(maxwellian, 0.0, 4.0 * math.pi, -8.0, 8.0, eps, k, boxes, coarse, ratio)


def hier_state(profile, x_lo, x_len, v_lo, v_hi, eps, k, coarse, ratios, boxes):
    """Exact cell averages of (1 + eps cos(k x)) profile(v) on level 0 and on
    every patch of a multi-level hierarchy (ratios[l-1] = (r_x, r_v) of
    level l-1 -> l; boxes with "level" and inclusive lo/hi in that level's
    indices), concatenated as [level 0][boxes in order]; returns
    (state, [equilibrium with ghosts of each level])."""
    nx, nv = [coarse[0]], [coarse[1]]
    for rx, rv in ratios:
        nx.append(nx[-1] * rx)
        nv.append(nv[-1] * rv)
    veqs = [cell_average_1d(profile, v_lo, v_hi, n, first=-2, count=n + 4) for n in nv]
    xs = [1.0 + eps * cos_cell_average(x_lo, x_len, n, k) for n in nx]
    parts = [(xs[0][:, None] * veqs[0][None, 2:nv[0] + 2]).ravel()]
    for b in boxes:
        lv = b["level"]
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        parts.append((xs[lv][x0:x1 + 1, None] * veqs[lv][None, 2 + v0:2 + v1 + 1]).ravel())
    return np.concatenate(parts), veqs


# bump-on-tail problem of the numerical results (section 4)
BUMP_X_LO = -10.0 * math.pi / 3.0
BUMP_X_LEN = 20.0 * math.pi / 3.0
BUMP_V_LO, BUMP_V_HI = -8.0, 10.0


def amr_bump_on_tail(boxes, coarse=(16, 32), ratio: int = 4, eps: float = 0.04, k: float = 0.3):
    """Two-level bump-on-tail problem: (1 + 0.04 cos(0.3 x)) f_b(v) on
    [-10 pi/3, 10 pi/3) x [-8, 10]; returns (state, veq_c, veq_f)."""
    return _amr_state(bump_on_tail_profile, BUMP_X_LO, BUMP_X_LEN, BUMP_V_LO, BUMP_V_HI, eps, k, boxes, coarse,
                      ratio)


def bump_on_tail_initial_boxes(coarse=(16, 32), ratio: int = 4):
    """The initial refinement of the bump-on-tail run, level-0 cells
    [0, 15] x [8, 24] of a 16 x 32 mesh (the whole periodic x range),
    scaled to `coarse`."""
    ncx, ncv = coarse
    sv = ncv // 32
    return [{"level": 1, "lo": [0, 8 * sv * ratio], "hi": [ncx * ratio - 1, (24 * sv + sv) * ratio - 1]}]


def save_boxes(path, boxes):
    with open(path, "w") as fh:
        json.dump(boxes, fh, indent=1)


def load_boxes(path):
    with open(path) as fh:
        return json.load(fh)
