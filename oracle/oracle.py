"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

ctypes/numpy wrapper around the plain FP64 C oracle (vp_oracle.c,
vp_oracle_adjoint.c, ...).  Only the tests, the smoke check and the CPU
baseline leg of the benchmark import this module; the GPU library never
does.  All arrays are float64, row-major [x][v].
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["vp_oracle.c", "vp_oracle_adjoint.c", "vp_oracle_amr.c", "vp_oracle_4d.c", "vp_oracle_limited.c",
           "vp_oracle_regrid.c", "vp_oracle_hier.c",
           "vp_oracle_amr4d.c"]
LIB = os.path.join(HERE, "libvp_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP over rows)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(s) for s in srcs + [os.path.join(HERE, "vp_oracle.h")])
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = ctypes.CDLL(LIB)
        _declare(_lib)
    return _lib


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.c_int
_F = ctypes.c_double
_V = ctypes.c_void_p


def _declare(L):
    sig = {
        "vpo_num_threads": (_I, []),
        "vpo_set_num_threads": (None, [_I]),
        "vpo_moment": (None, [_I, _I, _F, _D, _D]),
        "vpo_poisson_new": (_V, [_I]),
        "vpo_poisson_free": (None, [_V]),
        "vpo_poisson_solve": (None, [_V, _F, _D, _D]),
        "vpo_field": (None, [_I, _F, _D, _D]),
        "vpo_rhs": (None, [_I, _I, _F, _F, _F, _D, _D, _D, _D]),
        "vpo_vboundary_flux": (None, [_I, _I, _F, _F, _D, _D, _D, _D, _D]),
        "vpo_ctx_new": (_V, [_I, _I, _F, _F, _F, _F, _D]),
        "vpo_ctx_free": (None, [_V]),
        "vpo_constraints": (None, [_V, _D, _D, _D, _D, _D]),
        "vpo_rk4_step_stages": (None, [_V, _D, _D, _F, _D, _D]),
        "vpo_rk4_step": (None, [_V, _D, _D, _F]),
        "vpo_rk4_step_fixed_a": (None, [_V, _D, _D, _D, _F]),
        "vpo_rhs_adjoint": (None, [_I, _I, _F, _F, _F, _D, _D, _D, _D, _D, _D]),
        "vpo_constraints_adjoint": (None, [_V, _D, _D]),
        "vpo_rk4_adjoint_step": (None, [_V, _D, _D, _D, _F]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _declare_extra(L)


def _declare_extra(L):
    """Entry points of the AMR and 2D+2V oracle files, when present."""
    extra = {
        "vpo_interp_weights": (None, [_I, _D]),
        "vpo_amr_new": (_V, [_I, _I, _F, _F, _F, _F, _I, _I, ctypes.POINTER(ctypes.c_int),
                             _D, _D]),
        "vpo_amr_free": (None, [_V]),
        "vpo_amr_state_size": (ctypes.c_long, [_V]),
        "vpo_amr_patch_offset": (ctypes.c_long, [_V, _I]),
        "vpo_amr_reduce_mask": (None, [_V, _D, _D]),
        "vpo_amr_constraints": (None, [_V, _D, _D, _D]),
        "vpo_amr_fill_ghosts": (None, [_V, _D, _I, _D]),
        "vpo_amr_rk4_step": (None, [_V, _D, _D, _F]),
        "vpo_amr_subcycle_step": (None, [_V, _D, _D, _F]),
        "vpo4_tag": (None, [_V, _D, _F, ctypes.c_void_p, _D]),
        "vpo4_tag_value": (_F, [_V, _D, _I, _I, _I, _I]),
        "vpo_rk4_dense_weights": (None, [_F, _D]),
        "vpo_rk4_substage_weights": (None, [_F, _F, _I, _D]),
        "vpo_amr_rhs": (None, [_V, _D, _D, _D]),
        "vpo_amr_set_limited": (None, [_V, _I]),
        "vpo_a4_new": (_V, [ctypes.POINTER(ctypes.c_int), _F, _F, _F, _F, _F, _I, _I, ctypes.POINTER(ctypes.c_int),
                            _D, _D, _D, _D]),
        "vpo_a4_free": (None, [_V]),
        "vpo_a4_state_size": (ctypes.c_long, [_V]),
        "vpo_a4_patch_offset": (ctypes.c_long, [_V, _I]),
        "vpo_a4_fill_ghosts": (None, [_V, _D, _I, _D]),
        "vpo_a4_reduce_mask": (None, [_V, _D, _D]),
        "vpo_a4_constraints": (None, [_V, _D, _D, _D]),
        "vpo_a4_rhs": (None, [_V, _D, _D, _D]),
        "vpo_a4_rk4_step": (None, [_V, _D, _D, _F]),
        "vpo_hier_new": (_V, [_I, _I, _I, _F, _F, _F, _F, ctypes.POINTER(ctypes.c_int), _I,
                              ctypes.POINTER(ctypes.c_int), _D, ctypes.POINTER(ctypes.c_int)]),
        "vpo_hier_free": (None, [_V]),
        "vpo_hier_state_size": (ctypes.c_long, [_V]),
        "vpo_hier_patch_offset": (ctypes.c_long, [_V, _I]),
        "vpo_hier_fill_ghosts": (None, [_V, _D, _I, _D]),
        "vpo_hier_reduce_mask": (None, [_V, _D, _D]),
        "vpo_hier_constraints": (None, [_V, _D, _D, _D]),
        "vpo_hier_rhs": (None, [_V, _D, _D, _D]),
        "vpo_hier_rk4_step": (None, [_V, _D, _D, _F]),
        "vpo_hier_tag_values": (None, [_V, _D, _I, _D]),
        "vpo_hier_prolong_box": (_I, [_V, _D, _I, _I, _I, _I, _I, _D]),
        "vpo_amr_species_constraints": (None, [_I, ctypes.POINTER(_V), ctypes.POINTER(_D), _D, _F,
                                               ctypes.POINTER(_D)]),
        "vpo_amr_species_rk4_step": (None, [_I, ctypes.POINTER(_V), ctypes.POINTER(_D), ctypes.POINTER(_D), _D,
                                            _F, _F]),
        "vpo_face_limited": (_F, [_F, _F, _F, _F, _I]),
        "vpo_rhs_limited": (None, [_I, _I, _F, _F, _F, _D, _D, _D, _D]),
        "vpo_rk4_step_limited": (None, [_V, _D, _D, _F]),
        "vpo_rk4_step_fixed_a_limited": (None, [_V, _D, _D, _D, _F]),
        "vpo_tag_value": (_F, [_I, _I, _F, _F, _D, _D, _I, _I]),
        "vpo_tag": (None, [_I, _I, _F, _F, _D, _D, _F, ctypes.POINTER(ctypes.c_ubyte)]),
        "vpo_prolong1d": (None, [_D, _I, _D]),
        "vpo_prolong_box": (None, [_I, _I, _D, _D, _I, _I, _I, _I, _I, _D]),
        "vpo4_ctx_new": (_V, [_I, _I, _I, _I, _F, _F, _F, _F, _F, _D, _D]),
        "vpo4_ctx_free": (None, [_V]),
        "vpo4_moment": (None, [_V, _D, _D]),
        "vpo4_poisson": (_F, [_V, _D, _D]),
        "vpo4_field": (None, [_V, _D, _D]),
        "vpo4_constraints": (None, [_V, _D, _D, _D, _D]),
        "vpo4_rhs": (None, [_V, _D, _D, _D]),
        "vpo4_rk4_step": (None, [_V, _D, _D, _F]),
        "vpo4_rk4_step_fixed_a": (None, [_V, _D, _D, _D, _F]),
    }
    for name, (res, args) in extra.items():
        fn = getattr(L, name, None)
        if fn is not None:
            fn.restype = res
            fn.argtypes = args


def _p(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads():
    return lib().vpo_num_threads()


def set_num_threads(n):
    """Threads of the oracle's OpenMP loops from now on (timing only)."""
    lib().vpo_set_num_threads(int(n))


def moment(f, dv):
    f = _f64(f)
    n = np.empty(f.shape[0])
    lib().vpo_moment(f.shape[0], f.shape[1], dv, _p(f), _p(n))
    return n


class Poisson:
    def __init__(self, nx):
        self.nx = nx
        self.h = lib().vpo_poisson_new(nx)

    def solve(self, rho, dx):
        rho = _f64(rho)
        phi = np.empty(self.nx)
        lib().vpo_poisson_solve(self.h, dx, _p(rho), _p(phi))
        return phi

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.vpo_poisson_free(self.h)
            self.h = None


def poisson_solve(rho, dx):
    return Poisson(len(rho)).solve(rho, dx)


def field(phi, dx):
    phi = _f64(phi)
    E = np.empty_like(phi)
    lib().vpo_field(len(phi), dx, _p(phi), _p(E))
    return E


def rhs(f, a, dx, dv, v_lo, vghost):
    f, a, vg = _f64(f), _f64(a), _f64(vghost)
    k = np.empty_like(f)
    lib().vpo_rhs(f.shape[0], f.shape[1], dx, dv, v_lo, _p(vg), _p(f), _p(a), _p(k))
    return k


def vboundary_flux(f, a, dx, dv, vghost):
    f, a, vg = _f64(f), _f64(a), _f64(vghost)
    lo = np.empty(f.shape[0])
    hi = np.empty(f.shape[0])
    lib().vpo_vboundary_flux(f.shape[0], f.shape[1], dx, dv, _p(vg), _p(f), _p(a), _p(lo), _p(hi))
    return lo, hi


def face_limited(um1, u0, u1, u2, upwind_left):
    """limited face average between u0 and u1 (section 2, eq. limitedFace)"""
    return lib().vpo_face_limited(float(um1), float(u0), float(u1), float(u2), int(bool(upwind_left)))


def rhs_limited(f, a, dx, dv, v_lo, vghost):
    f, a, vg = _f64(f), _f64(a), _f64(vghost)
    k = np.empty_like(f)
    lib().vpo_rhs_limited(f.shape[0], f.shape[1], dx, dv, v_lo, _p(vg), _p(f), _p(a), _p(k))
    return k


def rhs_adjoint(f, a, kbar, dx, dv, v_lo, vghost):
    f, a, kb, vg = _f64(f), _f64(a), _f64(kbar), _f64(vghost)
    fb = np.empty_like(f)
    ab = np.empty(f.shape[0])
    lib().vpo_rhs_adjoint(f.shape[0], f.shape[1], dx, dv, v_lo, _p(vg), _p(f), _p(a), _p(kb),
                          _p(fb), _p(ab))
    return fb, ab


def tag_values(f, dx, dv, vghost):
    """delta1 f + delta2 f of every cell of a level (section 3, refinement criterion)."""
    f = _f64(f)
    nx, nv = f.shape
    vg = _f64(vghost)
    out = np.empty((nx, nv))
    L = lib()
    for i in range(nx):
        for j in range(nv):
            out[i, j] = L.vpo_tag_value(nx, nv, dx, dv, _p(vg), _p(f), i, j)
    return out


def tag(f, dx, dv, vghost, tol):
    """1 where delta1 f + delta2 f > tol, else 0 (uint8 [nx][nv])."""
    f = _f64(f)
    nx, nv = f.shape
    vg = _f64(vghost)
    t = np.zeros((nx, nv), dtype=np.uint8)
    lib().vpo_tag(nx, nv, dx, dv, _p(vg), _p(f), tol, t.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
    return t


def prolong1d(u, R):
    """R fine cell averages of the middle of five coarse cell averages (section 3, conservative
    limited interpolation)."""
    u = _f64(u)
    out = np.empty(R)
    lib().vpo_prolong1d(_p(u), R, _p(out))
    return out


def prolong_box(fc, vghost_c, R, box):
    """Fine cell averages on the level-1 box (fx0, fv0, fx1, fv1), x then v."""
    fc = _f64(fc)
    vg = _f64(vghost_c)
    fx0, fv0, fx1, fv1 = box
    out = np.empty((fx1 - fx0 + 1, fv1 - fv0 + 1))
    lib().vpo_prolong_box(fc.shape[0], fc.shape[1], _p(fc), _p(vg), R, fx0, fv0, fx1, fv1, _p(out))
    return out


def regrid_transfer(f_old, old_boxes, new_boxes, ncx, ncv, R, vghost_c):
    """State of a new two-level hierarchy after a regrid (section 3): level 0
    unchanged; a new fine cell keeps the old fine value where an old patch
    covered it, else takes the conservative limited interpolation of level 0
    (x then v).  Boxes: dicts with inclusive level-1 lo/hi; states flat
    [level 0][patch 0][patch 1]..."""
    f_old = _f64(f_old)
    nc = ncx * ncv
    f0 = f_old[:nc].reshape(ncx, ncv)
    old, off = [], nc
    for b in old_boxes:
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        n = (x1 - x0 + 1) * (v1 - v0 + 1)
        old.append(((x0, v0, x1, v1), f_old[off:off + n].reshape(x1 - x0 + 1, v1 - v0 + 1)))
        off += n
    parts = [f_old[:nc].copy()]
    for b in new_boxes:
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        fine = prolong_box(f0, vghost_c, R, (x0, v0, x1, v1))
        for (a0, b0, a1, b1), blk in old:
            ix0, ix1, iv0, iv1 = max(x0, a0), min(x1, a1), max(v0, b0), min(v1, b1)
            if ix0 <= ix1 and iv0 <= iv1:
                fine[ix0 - x0:ix1 - x0 + 1, iv0 - v0:iv1 - v0 + 1] = blk[ix0 - a0:ix1 - a0 + 1, iv0 - b0:iv1 - b0 + 1]
        parts.append(fine.ravel())
    return np.concatenate(parts)


def linear_stability_courant():
    """Largest Courant number nu = dt (|v| / dx + |a| / dv) for which classic
    RK4 (eq. rk4) on the centred fourth-order flux divergence of section 2 is
    linearly stable.  The divergence of the face averages maps the Fourier
    mode exp(i theta j) to i s(theta) / h, s(theta) = (8 sin theta -
    sin 2 theta) / 6, whose maximum is at cos theta = 1 - sqrt(6)/2; summed
    over the two phase directions the largest eigenvalue modulus is
    nu max s.  RK4's amplification |P(i y)|^2 = 1 - y^6/72 + y^8/576 stays
    <= 1 exactly for y <= 2 sqrt 2, so nu <= 2 sqrt 2 / max s (about 2.0612)."""
    c = 1.0 - math.sqrt(6.0) / 2.0
    s_max = math.sqrt(1.0 - c * c) * (4.0 - c) / 3.0
    return 2.0 * math.sqrt(2.0) / s_max


def amr_stability_limit(a, ncx, ncv, R, x_len, v_lo, v_hi, boxes):
    """Largest dt for which the step is linearly stable on every level of a
    two-level hierarchy (section 4's time step control takes a fraction of
    it): dt (max|v| / dx + max|a| / dv) <= linear_stability_courant(), on
    level 0 over its whole mesh; on level 1 per patch, with the largest |v| on
    the patch's velocity faces and the largest |a| over the fine
    configuration columns it covers.  a = [a_coarse (ncx)][a_fine (ncx R)]."""
    a = _f64(a)
    dxc, dvc = x_len / ncx, (v_hi - v_lo) / ncv
    dxf, dvf = dxc / R, dvc / R
    rate = max(abs(v_lo), abs(v_hi)) / dxc + np.abs(a[:ncx]).max() / dvc
    af = a[ncx:]
    for b in boxes:
        (x0, v0), (x1, v1) = b["lo"], b["hi"]
        vmax = max(abs(v_lo + v0 * dvf), abs(v_lo + (v1 + 1) * dvf))
        rate = max(rate, vmax / dxf + np.abs(af[x0:x1 + 1]).max() / dvf)
    return linear_stability_courant() / rate


class Oracle1D:
    """Single-level 1D+1V oracle bound to one mesh (Poisson factors kept)."""

    def __init__(self, nx, nv, x_len, v_lo, v_hi, qm, vghost):
        self.nx, self.nv = nx, nv
        self.dx = x_len / nx
        self.dv = (v_hi - v_lo) / nv
        self.v_lo = v_lo
        self.qm = qm
        self.vghost = _f64(vghost)
        self.h = lib().vpo_ctx_new(nx, nv, x_len, v_lo, v_hi, qm, _p(self.vghost))

    @classmethod
    def from_problem(cls, prob):
        return cls(prob.nx, prob.nv, prob.x_len, prob.v_lo, prob.v_hi, prob.qm, prob.vghost)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.vpo_ctx_free(self.h)
            self.h = None

    def constraints(self, f):
        """Return (a, n, phi, E) for the state f."""
        f = _f64(f)
        a, n, phi, E = (np.empty(self.nx) for _ in range(4))
        lib().vpo_constraints(self.h, _p(f), _p(a), _p(n), _p(phi), _p(E))
        return a, n, phi, E

    def rhs(self, f, a):
        return rhs(f, a, self.dx, self.dv, self.v_lo, self.vghost)

    def step(self, f, dt):
        f = _f64(f)
        out = np.empty_like(f)
        lib().vpo_rk4_step(self.h, _p(f), _p(out), dt)
        return out

    def step_stages(self, f, dt):
        f = _f64(f)
        out = np.empty_like(f)
        sf = np.empty((4,) + f.shape)
        sa = np.empty((4, self.nx))
        lib().vpo_rk4_step_stages(self.h, _p(f), _p(out), dt, _p(sf), _p(sa))
        return out, sf, sa

    def step_fixed_a(self, f, a, dt):
        f, a = _f64(f), _f64(a)
        out = np.empty_like(f)
        lib().vpo_rk4_step_fixed_a(self.h, _p(f), _p(out), _p(a), dt)
        return out

    def rhs_limited(self, f, a):
        return rhs_limited(f, a, self.dx, self.dv, self.v_lo, self.vghost)

    def step_limited(self, f, dt):
        f = _f64(f)
        out = np.empty_like(f)
        lib().vpo_rk4_step_limited(self.h, _p(f), _p(out), dt)
        return out

    def step_fixed_a_limited(self, f, a, dt):
        f, a = _f64(f), _f64(a)
        out = np.empty_like(f)
        lib().vpo_rk4_step_fixed_a_limited(self.h, _p(f), _p(out), _p(a), dt)
        return out

    def constraints_adjoint(self, abar, fbar):
        abar = _f64(abar)
        fbar = np.array(fbar, dtype=np.float64, copy=True)
        lib().vpo_constraints_adjoint(self.h, _p(abar), _p(fbar))
        return fbar

    def adjoint_step(self, f_n, lam_np1, dt):
        f_n, lam = _f64(f_n), _f64(lam_np1)
        out = np.empty_like(f_n)
        lib().vpo_rk4_adjoint_step(self.h, _p(f_n), _p(lam), _p(out), dt)
        return out


def species_field(fs, species, charges, background, dx, poisson=None):
    """Accelerations of several species on one configuration mesh: the charge
    density rho = background + sum_s charge_s n_s (n_s the velocity moment of
    species s), the periodic Poisson solve and field stencil of section 2,
    a_s = (q/m)_s E.  species: dicts with dv and qm.  Returns ([a_s], E)."""
    nx = fs[0].shape[0]
    rho = np.full(nx, float(background))
    for f, sp, q in zip(fs, species, charges):
        rho = rho + q * moment(f, sp["dv"])
    P = poisson if poisson is not None else Poisson(nx)
    E = field(P.solve(rho, dx), dx)
    return [sp["qm"] * E for sp in species], E


def species_rk4_step(fs, species, charges, background, dx, dt):
    """One classic RK4 step (eq. rk4) of several species that share the field:
    at every stage the field of all predictor states, then each species'
    semi-discrete right-hand side with its own velocity mesh, equilibrium
    ghosts and acceleration.  species: dicts with dv, v_lo, vghost, qm."""
    alpha = [0.0, 0.5, 0.5, 1.0]
    b = [1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0]
    fn = [_f64(f) for f in fs]
    P = Poisson(fn[0].shape[0])
    ks = []
    for s in range(4):
        stage = [f if s == 0 else f + alpha[s] * dt * k for f, k in zip(fn, ks[-1] if ks else fn)]
        a, _ = species_field(stage, species, charges, background, dx, P)
        ks.append([rhs(f, ai, dx, sp["dv"], sp["v_lo"], sp["vghost"]) for f, ai, sp in zip(stage, a, species)])
    return [f + dt * (b[0] * ks[0][q] + b[1] * ks[1][q] + b[2] * ks[2][q] + b[3] * ks[3][q])
            for q, f in enumerate(fn)]


def interp_weights(R):
    """b_j(s) table (R x 5) of the conservative fifth-order sub-cell interpolation."""
    out = np.empty((R, 5))
    lib().vpo_interp_weights(R, _p(out))
    return out


class OracleAMR:
    """Two-level 1D+1V oracle: coarse (ncx x ncv) plus level-1 patches
    (boxes: dicts with inclusive lo/hi in the level-1 index space)."""

    def __init__(self, ncx, ncv, x_len, v_lo, v_hi, qm, R, boxes, veq_c, veq_f):
        self.ncx, self.ncv, self.R = ncx, ncv, R
        self.boxes = boxes
        arr = np.array([[b["lo"][0], b["lo"][1], b["hi"][0], b["hi"][1]] for b in boxes], dtype=np.int32).ravel()
        if arr.size == 0:
            arr = np.zeros(4, dtype=np.int32)
        self._boxes = np.ascontiguousarray(arr)
        self.veq_c, self.veq_f = _f64(veq_c), _f64(veq_f)
        self.h = lib().vpo_amr_new(ncx, ncv, x_len, v_lo, v_hi, qm, R, len(boxes),
                                   self._boxes.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                   _p(self.veq_c), _p(self.veq_f))
        self.size = lib().vpo_amr_state_size(self.h)
        self.nfx = ncx * R

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.vpo_amr_free(self.h)
            self.h = None

    def offset(self, p):
        return lib().vpo_amr_patch_offset(self.h, p)

    def set_limited(self, on=True):
        """Limited face averages (section 2, eq. limitedFace) on both levels."""
        lib().vpo_amr_set_limited(self.h, int(bool(on)))
        return self

    def reduce_mask(self, f):
        f = _f64(f)
        n = np.empty(self.nfx)
        lib().vpo_amr_reduce_mask(self.h, _p(f), _p(n))
        return n

    def constraints(self, f):
        """(a = [a_coarse (ncx), a_fine (ncx R)], E on the fine mesh)"""
        f = _f64(f)
        a = np.empty(self.ncx + self.nfx)
        E = np.empty(self.nfx)
        lib().vpo_amr_constraints(self.h, _p(f), _p(a), _p(E))
        return a, E

    def ghosted_patch(self, f, p):
        f = _f64(f)
        b = self.boxes[p]
        nx, nv = b["hi"][0] - b["lo"][0] + 1, b["hi"][1] - b["lo"][1] + 1
        out = np.empty((nx + 4, nv + 4))
        lib().vpo_amr_fill_ghosts(self.h, _p(f), p, _p(out))
        return out

    def rhs(self, f, a):
        """k = L(f; a) on every patch, a = [a_coarse, a_fine]"""
        f, a = _f64(f), _f64(a)
        k = np.empty_like(f)
        lib().vpo_amr_rhs(self.h, _p(f), _p(a), _p(k))
        return k

    def step(self, f, dt):
        f = _f64(f)
        out = np.empty_like(f)
        lib().vpo_amr_rk4_step(self.h, _p(f), _p(out), dt)
        return out

    def subcycle_step(self, f, dt):
        """One subcycled step: the coarse level takes dt with the field of its
        own moment on the coarse configuration mesh, the patches R substeps of
        dt / R with coarse data from the continuous extension of the coarse
        RK4 step, then refluxing and the average-down (section 5 names
        asynchronous stepping as future work; the reading is in vp_oracle_amr.c)."""
        f = _f64(f)
        out = np.empty_like(f)
        lib().vpo_amr_subcycle_step(self.h, _p(f), _p(out), dt)
        return out


class OracleHier:
    """L-level 1D+1V oracle (vp_oracle_hier.c): level 0 (ncx x ncv) and
    patches on levels 1 .. L-1 (boxes: dicts with "level" and inclusive
    lo/hi in that level's index space); ratios[l-1] = (r_x, r_v) of level
    l-1 -> l; veqs[l]: level-l equilibrium with two ghosts per side."""

    def __init__(self, L, ncx, ncv, x_len, v_lo, v_hi, qm, ratios, boxes, veqs):
        self.L, self.ncx, self.ncv = L, ncx, ncv
        self.x_len_ = x_len
        self.ratios = [tuple(r) for r in ratios]
        self.boxes = boxes
        self.nx, self.nv = [ncx], [ncv]
        for rx, rv in self.ratios:
            self.nx.append(self.nx[-1] * rx)
            self.nv.append(self.nv[-1] * rv)
        rat = np.ascontiguousarray(np.array(self.ratios, dtype=np.int32).ravel() if ratios else np.zeros(2, np.int32))
        arr = np.array([[b["level"], b["lo"][0], b["lo"][1], b["hi"][0], b["hi"][1]] for b in boxes],
                       dtype=np.int32).ravel()
        self._rat, self._boxes = rat, np.ascontiguousarray(arr if arr.size else np.zeros(5, np.int32))
        self._veq = _f64(np.concatenate([np.asarray(v, dtype=np.float64) for v in veqs]))
        err = ctypes.c_int(0)
        self.h = lib().vpo_hier_new(L, ncx, ncv, x_len, v_lo, v_hi, qm,
                                    self._rat.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(boxes),
                                    self._boxes.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(self._veq),
                                    ctypes.byref(err))
        if not self.h:
            raise ValueError(f"bad hierarchy (code {err.value})")
        self.size = lib().vpo_hier_state_size(self.h)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.vpo_hier_free(self.h)
            self.h = None

    @property
    def nfx(self):
        return self.nx[-1]

    @property
    def field_elems(self):
        return sum(self.nx)

    def offset(self, p):
        """element offset of boxes[p] (p = -1: level 0)"""
        return lib().vpo_hier_patch_offset(self.h, p)

    def ghosted(self, f, p):
        """patch p (-1: level 0) with two ghost layers"""
        f = _f64(f)
        if p < 0:
            nx, nv = self.ncx, self.ncv
        else:
            b = self.boxes[p]
            nx, nv = b["hi"][0] - b["lo"][0] + 1, b["hi"][1] - b["lo"][1] + 1
        out = np.empty((nx + 4, nv + 4))
        lib().vpo_hier_fill_ghosts(self.h, _p(f), p + 1, _p(out))
        return out

    def reduce_mask(self, f):
        f = _f64(f)
        n = np.empty(self.nfx)
        lib().vpo_hier_reduce_mask(self.h, _p(f), _p(n))
        return n

    def constraints(self, f):
        """(a on every level, concatenated from level 0; E on the finest mesh)"""
        f = _f64(f)
        a = np.empty(self.field_elems)
        E = np.empty(self.nfx)
        lib().vpo_hier_constraints(self.h, _p(f), _p(a), _p(E))
        return a, E

    def rhs(self, f, a):
        f, a = _f64(f), _f64(a)
        k = np.empty_like(f)
        lib().vpo_hier_rhs(self.h, _p(f), _p(a), _p(k))
        return k

    def step(self, f, dt):
        f = _f64(f)
        out = np.empty_like(f)
        lib().vpo_hier_rk4_step(self.h, _p(f), _p(out), dt)
        return out

    def tag_values(self, f, level):
        """delta1 f + delta2 f on the cells level `level` holds (NaN elsewhere)"""
        f = _f64(f)
        out = np.empty(self.nx[level] * self.nv[level])
        lib().vpo_hier_tag_values(self.h, _p(f), level, _p(out))
        return out.reshape(self.nx[level], self.nv[level])

    def prolong_box(self, f, level, lo, hi):
        """WENO5 prolongation of level-1 data into the level-`level` box [lo, hi]"""
        f = _f64(f)
        out = np.empty((hi[0] - lo[0] + 1, hi[1] - lo[1] + 1))
        ok = lib().vpo_hier_prolong_box(self.h, _p(f), level, lo[0], lo[1], hi[0], hi[1], _p(out))
        if not ok:
            raise ValueError("a parent cell of the box is not held by the parent level")
        return out

    def patch_data(self, f, p):
        b = self.boxes[p]
        nx, nv = b["hi"][0] - b["lo"][0] + 1, b["hi"][1] - b["lo"][1] + 1
        o = self.offset(p)
        return np.asarray(f)[o:o + nx * nv].reshape(nx, nv)

    def level_array(self, f, level):
        """level `level` as a dense array, NaN where it has no patch"""
        if level == 0:
            return np.asarray(f)[: self.ncx * self.ncv].reshape(self.ncx, self.ncv).copy()
        out = np.full((self.nx[level], self.nv[level]), np.nan)
        for p, b in enumerate(self.boxes):
            if b["level"] == level:
                out[b["lo"][0]:b["hi"][0] + 1, b["lo"][1]:b["hi"][1] + 1] = self.patch_data(f, p)
        return out


class OracleAMR4D:
    """Two-level 2D+2V oracle (vp_oracle_amr4d.c): level 0 of ncells =
    (nx, ny, nvx, nvy) cells and level-1 patches (boxes with 4-entry lo/hi
    in level-1 indices), one ratio R in every direction; g*: the 1D
    equilibria with two ghosts per side along vx and vy of both levels."""

    def __init__(self, ncells, x_len, y_len, v_lo, v_hi, qm, R, boxes, gxc, gyc, gxf, gyf):
        self.n = tuple(ncells)
        self.R = R
        self.nf = tuple(c * R for c in ncells)
        self.boxes = boxes
        arr = np.array([list(b["lo"]) + list(b["hi"]) for b in boxes], dtype=np.int32).ravel()
        self._boxes = np.ascontiguousarray(arr if arr.size else np.zeros(8, np.int32))
        self._n = np.ascontiguousarray(np.array(ncells, dtype=np.int32))
        self._g = [_f64(g) for g in (gxc, gyc, gxf, gyf)]
        self.h = lib().vpo_a4_new(self._n.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), x_len, y_len, v_lo, v_hi,
                                  qm, R, len(boxes), self._boxes.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                  *[_p(g) for g in self._g])
        self.size = lib().vpo_a4_state_size(self.h)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.vpo_a4_free(self.h)
            self.h = None

    def offset(self, p):
        return lib().vpo_a4_patch_offset(self.h, p)

    def shape(self, p):
        if p < 0:
            return self.n
        b = self.boxes[p]
        return tuple(b["hi"][d] - b["lo"][d] + 1 for d in range(4))

    def patch(self, f, p):
        s = self.shape(p)
        o = self.offset(p)
        return np.asarray(f)[o:o + int(np.prod(s))].reshape(s)

    def ghosted(self, f, p):
        f = _f64(f)
        s = tuple(c + 4 for c in self.shape(p))
        out = np.empty(s)
        lib().vpo_a4_fill_ghosts(self.h, _p(f), p, _p(out))
        return out

    def reduce_mask(self, f):
        f = _f64(f)
        out = np.empty(self.nf[0] * self.nf[1])
        lib().vpo_a4_reduce_mask(self.h, _p(f), _p(out))
        return out

    def constraints(self, f):
        f = _f64(f)
        a = np.empty(2 * (self.n[0] * self.n[1] + self.nf[0] * self.nf[1]))
        E = np.empty(2 * self.nf[0] * self.nf[1])
        lib().vpo_a4_constraints(self.h, _p(f), _p(a), _p(E))
        return a, E

    def rhs(self, f, a):
        f, a = _f64(f), _f64(a)
        k = np.empty_like(f)
        lib().vpo_a4_rhs(self.h, _p(f), _p(a), _p(k))
        return k

    def step(self, f, dt):
        f = _f64(f)
        out = np.empty_like(f)
        lib().vpo_a4_rk4_step(self.h, _p(f), _p(out), dt)
        return out


def hier_regrid_transfer(old, f_old, new):
    """State of hierarchy `new` from hierarchy `old` after a regrid (section 3):
    level 0 copied; on each finer level, from the coarsest, every new cell an
    old patch of the same level held keeps the old value, the others are the
    conservative limited WENO5 prolongation of the new parent level."""
    f_new = np.zeros(new.size)
    f_new[: new.ncx * new.ncv] = np.asarray(f_old)[: old.ncx * old.ncv]
    for lv in range(1, new.L):
        old_lv = old.level_array(f_old, lv) if lv < old.L else None
        for p, b in enumerate(new.boxes):
            if b["level"] != lv:
                continue
            vals = new.prolong_box(f_new, lv, b["lo"], b["hi"])
            if old_lv is not None:
                o = old_lv[b["lo"][0]:b["hi"][0] + 1, b["lo"][1]:b["hi"][1] + 1]
                vals = np.where(np.isnan(o), vals, o)
            off = new.offset(p)
            f_new[off:off + vals.size] = vals.ravel()
    return f_new


def hier_stability_limit(o, a, v_lo, v_hi):
    """Largest linearly stable RK4 step of a multi-level hierarchy: dt times
    max over every level's patches of (max |v| on the patch's velocity faces
    / dx_l + max |a_l| over its configuration columns / dv_l) at the RK4 +
    centred fourth-order limit."""
    rate = 0.0
    off = 0
    a = np.asarray(a)
    al = []
    for lv in range(o.L):
        al.append(a[off:off + o.nx[lv]])
        off += o.nx[lv]
    patches = [(0, 0, 0, o.ncx - 1, o.ncv - 1)] + [(b["level"], b["lo"][0], b["lo"][1], b["hi"][0], b["hi"][1])
                                                    for b in o.boxes]
    for lv, x0, v0, x1, v1 in patches:
        dxl = o.x_len_ / o.nx[lv]
        dvl = (v_hi - v_lo) / o.nv[lv]
        vmax = max(abs(v_lo + v0 * dvl), abs(v_lo + (v1 + 1) * dvl))
        amax = np.abs(al[lv][x0:x1 + 1]).max()
        rate = max(rate, vmax / dxl + amax / dvl)
    return linear_stability_courant() / rate


def rk4_dense_weights(theta):
    """b_1..b_4(theta) of the third-order continuous extension of classical RK4."""
    b = np.empty(4)
    lib().vpo_rk4_dense_weights(theta, _p(b))
    return b


def rk4_substage_weights(theta0, eta, s):
    """Weights w_q (coarse data f_c^n + dt sum_q w_q K_q) of fine stage s of
    the substep [theta0, theta0 + eta]: the RK4 stage values on the Taylor
    expansion of the continuous extension at theta0."""
    w = np.empty(4)
    lib().vpo_rk4_substage_weights(theta0, eta, s, _p(w))
    return w


def _ptr_list(arrays):
    return (_D * len(arrays))(*[_p(x) for x in arrays])


def amr_species_field(hier, fs, charges, background):
    """[a_s] ([coarse][fine] per species) of several species, each on its own
    two-level hierarchy (OracleAMR objects with the same finest configuration
    mesh): rho = background + sum_s charge_s n_s (Mask Reduction)."""
    fs = [_f64(f) for f in fs]
    a = [np.empty(h.ncx + h.nfx) for h in hier]
    hs = (_V * len(hier))(*[h.h for h in hier])
    ch = np.ascontiguousarray(charges, dtype=np.float64)
    lib().vpo_amr_species_constraints(len(hier), hs, _ptr_list(fs), _p(ch), float(background), _ptr_list(a))
    return a


def amr_species_rk4_step(hier, fs, charges, background, dt):
    """One RK4 step of several species' two-level hierarchies sharing the field."""
    fs = [_f64(f) for f in fs]
    out = [np.empty_like(f) for f in fs]
    hs = (_V * len(hier))(*[h.h for h in hier])
    ch = np.ascontiguousarray(charges, dtype=np.float64)
    lib().vpo_amr_species_rk4_step(len(hier), hs, _ptr_list(fs), _ptr_list(out), _p(ch), float(background), dt)
    return out


class Oracle4D:
    """Single-level 2D+2V oracle, f as [x][y][vx][vy]; a and E hold the x
    component (nx ny values, [x][y]) followed by the y component."""

    def __init__(self, nx, ny, nvx, nvy, x_len, y_len, v_lo, v_hi, qm, veq_x, veq_y):
        self.nx, self.ny, self.nvx, self.nvy = nx, ny, nvx, nvy
        self.veq_x, self.veq_y = _f64(veq_x), _f64(veq_y)
        self.h = lib().vpo4_ctx_new(nx, ny, nvx, nvy, x_len, y_len, v_lo, v_hi, qm, _p(self.veq_x),
                                    _p(self.veq_y))

    @classmethod
    def from_problem(cls, p):
        return cls(p.nx, p.ny, p.nvx, p.nvy, p.x_len, p.y_len, p.v_lo, p.v_hi, p.qm, p.veq_x, p.veq_y)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.vpo4_ctx_free(self.h)
            self.h = None

    def tag(self, f, tol):
        """(tags uint8, delta1 f + delta2 f) of every cell, the criterion of
        section 3 summed over x, y, vx, vy."""
        f = _f64(f)
        tags = np.empty(f.size, dtype=np.uint8)
        vals = np.empty(f.size)
        lib().vpo4_tag(self.h, _p(f), tol, tags.ctypes.data_as(ctypes.c_void_p), _p(vals))
        shape = (self.nx, self.ny, self.nvx, self.nvy)
        return tags.reshape(shape), vals.reshape(shape)

    def tag_value(self, f, i, j, k, l):
        f = _f64(f)
        return lib().vpo4_tag_value(self.h, _p(f), i, j, k, l)

    def moment(self, f):
        f = _f64(f)
        n = np.empty(self.nx * self.ny)
        lib().vpo4_moment(self.h, _p(f), _p(n))
        return n.reshape(self.nx, self.ny)

    def poisson(self, rho):
        """(phi, relative residual)"""
        rho = _f64(rho).ravel()
        phi = np.empty_like(rho)
        res = lib().vpo4_poisson(self.h, _p(rho), _p(phi))
        return phi.reshape(self.nx, self.ny), res

    def field(self, phi):
        phi = _f64(phi).ravel()
        E = np.empty(2 * phi.size)
        lib().vpo4_field(self.h, _p(phi), _p(E))
        return E

    def constraints(self, f):
        """(a, phi, E): a = (q/m) E, each [Ex; Ey] flattened"""
        f = _f64(f)
        n = self.nx * self.ny
        a, phi, E = np.empty(2 * n), np.empty(n), np.empty(2 * n)
        lib().vpo4_constraints(self.h, _p(f), _p(a), _p(phi), _p(E))
        return a, phi, E

    def rhs(self, f, a):
        f, a = _f64(f), _f64(a)
        k = np.empty_like(f)
        lib().vpo4_rhs(self.h, _p(f), _p(a), _p(k))
        return k

    def step(self, f, dt):
        f = _f64(f)
        out = np.empty_like(f)
        lib().vpo4_rk4_step(self.h, _p(f), _p(out), dt)
        return out

    def step_fixed_a(self, f, a, dt):
        f, a = _f64(f), _f64(a)
        out = np.empty_like(f)
        lib().vpo4_rk4_step_fixed_a(self.h, _p(f), _p(out), _p(a), dt)
        return out
