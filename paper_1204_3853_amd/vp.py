"""Python binding of the MI355X Vlasov-Poisson library (include/vp.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libvp.so.  Device memory and streams come from PyTorch; arrays
are passed to the C ABI as raw pointers of contiguous tensors, and work is
enqueued on torch's current stream.  There is no CPU fallback: if the
library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvp.so")

VP_F64, VP_F32 = 0, 1
VP_MAX_LEVELS = 4
_STATUS = {0: "VP_OK", 1: "VP_EINVAL", 2: "VP_ESHAPE", 3: "VP_EDTYPE", 4: "VP_ENOTSUP", 5: "VP_EHIP",
           6: "VP_ENOMEM"}


class VPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class vp_problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("n_levels", ctypes.c_int32),
        ("cells", ctypes.c_int32 * 4),
        ("ratio", (ctypes.c_int32 * 4) * (VP_MAX_LEVELS - 1)),
        ("x_lo", ctypes.c_double * 2),
        ("x_len", ctypes.c_double * 2),
        ("v_lo", ctypes.c_double * 2),
        ("v_hi", ctypes.c_double * 2),
        ("qm", ctypes.c_double),
        ("veq", (ctypes.POINTER(ctypes.c_double) * 2) * VP_MAX_LEVELS),
    ]


class vp_box(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("lo", ctypes.c_int32 * 4), ("hi", ctypes.c_int32 * 4)]


class vp_amr_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("regrid_interval", ctypes.c_int32), ("efficiency", ctypes.c_double),
                ("min_width", ctypes.c_int32), ("buffer", ctypes.c_int32), ("cfl", ctypes.c_double),
                ("dt_growth", ctypes.c_double), ("dt_initial", ctypes.c_double),
                ("max_size", (ctypes.c_int32 * 2) * VP_MAX_LEVELS)]


class vp_amr_info(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double), ("steps", ctypes.c_int64),
                ("regrids", ctypes.c_int32), ("npatch", ctypes.c_int32), ("state_elems", ctypes.c_int64),
                ("regrid_seconds", ctypes.c_double)]


_lib = None

_P = ctypes.c_void_p
_D = ctypes.c_double
_S = ctypes.c_size_t

SIGNATURES = {
    "vp_plan_create": (ctypes.c_int, [ctypes.POINTER(vp_problem), ctypes.POINTER(vp_box), ctypes.c_int32,
                                      ctypes.POINTER(_P)]),
    "vp_plan_destroy": (ctypes.c_int, [_P]),
    "vp_last_error": (ctypes.c_char_p, []),
    "vp_state_elems": (_S, [_P]),
    "vp_patch_offset": (ctypes.c_int64, [_P, ctypes.c_int32]),
    "vp_config_elems": (_S, [_P]),
    "vp_field_elems": (_S, [_P]),
    "vp_workspace_bytes": (_S, [_P]),
    "vp_stage_elems": (_S, [_P]),
    "vp_rhs": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "vp_reduce_moment": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "vp_poisson_periodic": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "vp_inject_field": (ctypes.c_int, [_P, _P, _P, _P]),
    "vp_rk4_step": (ctypes.c_int, [_P, _P, _P, _D, _P, _P]),
    "vp_rk4_step_noalloc": (ctypes.c_int, [_P, _P, _P, _D, _P]),
    "vp_amr_subcycle_step": (ctypes.c_int, [_P, _P, _P, _D, _P, _P]),
    "vp_rk4_step_record": (ctypes.c_int, [_P, _P, _P, _D, _P, _P, _P]),
    "vp_adjoint_step": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _D, _P, _P]),
    "vp_field_adjoint": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "vp_tile_shape_count": (ctypes.c_int32, [_P]),
    "vp_tile_shape_get": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "vp_tile_shape_set": (ctypes.c_int, [_P, ctypes.c_int32]),
    "vp_launch_mode_set": (ctypes.c_int, [_P, ctypes.c_int32]),
    "vp_reduction_set": (ctypes.c_int, [_P, ctypes.c_int32]),
    "vp_face_scheme_set": (ctypes.c_int, [_P, ctypes.c_int32]),
    "vp_autotune": (ctypes.c_int, [_P, _P, _P, _D, ctypes.c_int32, _P, _P, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_float)]),
    "vp_timing_enable": (ctypes.c_int, [_P, ctypes.c_int32]),
    "vp_timing_read": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.c_int32]),
    "vp_tag_cells": (ctypes.c_int, [_P, _P, _D, _P, _P, _P]),
    "vp_cluster_tags": (ctypes.c_int, [ctypes.POINTER(ctypes.c_uint8), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       _D, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(vp_box), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32)]),
    "vp_regrid_transfer": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "vp_tag_level": (ctypes.c_int, [_P, _P, ctypes.c_int32, _D, _P, _P, _P, _P]),
    "vp_cluster_level": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint8), ctypes.c_int32,
                                        ctypes.c_int32, _D, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.POINTER(vp_box), ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32)]),
    "vp_amr_run_create": (ctypes.c_int, [ctypes.POINTER(vp_problem), ctypes.POINTER(vp_box), ctypes.c_int32, _P,
                                         ctypes.POINTER(vp_amr_params), ctypes.POINTER(_P), _P]),
    "vp_amr_run_advance": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "vp_amr_run_info": (ctypes.c_int, [_P, ctypes.POINTER(vp_amr_info)]),
    "vp_amr_run_plan": (_P, [_P]),
    "vp_amr_run_boxes": (ctypes.c_int, [_P, ctypes.POINTER(vp_box), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "vp_amr_run_read_state": (ctypes.c_int, [_P, _P, _S, _P]),
    "vp_amr_run_destroy": (ctypes.c_int, [_P]),
    "vp_amr_run_create_species": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.POINTER(vp_problem)),
                                                 ctypes.POINTER(ctypes.POINTER(vp_box)),
                                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_P),
                                                 ctypes.POINTER(ctypes.c_double), _D, ctypes.POINTER(vp_amr_params),
                                                 ctypes.POINTER(_P), _P]),
    "vp_amr_run_species_count": (ctypes.c_int32, [_P]),
    "vp_amr_run_plan_of": (_P, [_P, ctypes.c_int32]),
    "vp_amr_run_boxes_of": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(vp_box), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32)]),
    "vp_amr_run_read_state_of": (ctypes.c_int, [_P, ctypes.c_int32, _P, _S, _P]),
    "vp_species_group_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                               _D, ctypes.POINTER(_P)]),
    "vp_species_group_destroy": (ctypes.c_int, [_P]),
    "vp_species_workspace_bytes": (_S, [_P]),
    "vp_species_field": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P), _P, _P]),
    "vp_species_rk4_step": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _D, ctypes.POINTER(_P), _P,
                                           _P]),
}

TIMING_CLASSES = ["stage", "field", "moment", "sync", "adjoint", "other"]
LAUNCH_PERSISTENT, LAUNCH_PER_PATCH = 0, 1
REDUCE_SUBPATCH, REDUCE_MASK, REDUCE_FUSED = 0, 1, 2
FACE_CENTERED, FACE_LIMITED = 0, 1


def lib():
    """Load libvp.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise VPError(code, lib().vp_last_error().decode(errors="replace"))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _make_problem(spec, dtype):
    """vp_problem from a spec dict; returns (problem, buffers to keep alive)."""
    pb = vp_problem()
    keep = []
    pb.ndim = spec["ndim"]
    pb.dtype = VP_F64 if dtype == torch.float64 else VP_F32
    pb.n_levels = spec.get("n_levels", 1)
    for d, c in enumerate(spec["cells"]):
        pb.cells[d] = c
    ratios = spec.get("ratios")
    if ratios is None:                       # one ratio vector: level 0 -> level 1
        ratios = [spec.get("ratio", [1, 1, 1, 1])]
    for lvl, rv in enumerate(ratios):
        for d, r in enumerate(rv):
            pb.ratio[lvl][d] = r
    for d in range(spec["ndim"]):
        pb.x_lo[d] = spec["x_lo"][d]
        pb.x_len[d] = spec["x_len"][d]
        pb.v_lo[d] = spec["v_lo"][d]
        pb.v_hi[d] = spec["v_hi"][d]
    pb.qm = spec["qm"]
    for lvl, dirs in enumerate(spec["veq"]):
        for d, arr in enumerate(dirs):
            buf = (ctypes.c_double * len(arr))(*[float(x) for x in arr])
            keep.append(buf)
            pb.veq[lvl][d] = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
    return pb, keep


def _make_boxes(boxes):
    """(vp_box array or None, count) from dicts with level, lo, hi."""
    if not boxes:
        return None, 0
    bx = (vp_box * len(boxes))()
    for q, b in enumerate(boxes):
        bx[q].level = b.get("level", 1)
        for d, v in enumerate(b["lo"]):
            bx[q].lo[d] = v
        for d, v in enumerate(b["hi"]):
            bx[q].hi[d] = v
    return bx, len(boxes)


def _boxes_out(arr, n):
    return [{"level": arr[q].level, "lo": [arr[q].lo[0], arr[q].lo[1]], "hi": [arr[q].hi[0], arr[q].hi[1]]}
            for q in range(n)]


class Plan:
    """An immutable plan (vp_plan) plus the device workspace used by its calls.

    problem: a vp_inputs.Problem1D-like object (nx, nv, x_lo, x_len, v_lo,
    v_hi, qm, veq) or a dict with the fields of vp_problem.
    """

    def __init__(self, problem, dtype=torch.float64, boxes=None, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("the Vlasov-Poisson library needs a HIP GPU (torch.cuda is unavailable)")
        self.device = torch.device(device)
        self.dtype = dtype
        spec = problem if isinstance(problem, dict) else _problem_dict(problem)
        pb, self._keep = _make_problem(spec, dtype)
        self.spec = spec
        bx, nbox = _make_boxes(boxes)
        h = ctypes.c_void_p()
        _check(lib().vp_plan_create(ctypes.byref(pb), bx, nbox, ctypes.byref(h)))
        self.h = h
        L = lib()
        self.state_elems = L.vp_state_elems(h)
        self.config_elems = L.vp_config_elems(h)
        self.field_elems = L.vp_field_elems(h)
        self.workspace_bytes = L.vp_workspace_bytes(h)
        self.stage_elems = L.vp_stage_elems(h)
        self.work = torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=self.device)

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.vp_plan_destroy(self.h)
            self.h = None

    def timing_enable(self, enable=True):
        _check(lib().vp_timing_enable(self.h, int(enable)))

    def timing_read(self):
        """{class: (total ms, launches)} since the last read; clears the record."""
        n = len(TIMING_CLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _check(lib().vp_timing_read(self.h, ms, cnt, n))
        return {c: (ms[i], cnt[i]) for i, c in enumerate(TIMING_CLASSES)}

    def tile_shapes(self):
        """[(threads, cells per thread, rows per tile)] compiled for this plan."""
        out = []
        for q in range(lib().vp_tile_shape_count(self.h)):
            a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            _check(lib().vp_tile_shape_get(self.h, q, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
            out.append((a.value, b.value, c.value))
        return out

    def set_tile_shape(self, index):
        _check(lib().vp_tile_shape_set(self.h, index))

    def level_shape(self, level):
        """(nx, nv) of a level's index space"""
        nx, nv = self.spec["cells"][0], self.spec["cells"][1]
        ratios = self.spec.get("ratios") or [self.spec.get("ratio", [1, 1])]
        for l in range(level):
            nx *= ratios[l][0]
            nv *= ratios[l][1]
        return nx, nv

    def patch_offset(self, p):
        return lib().vp_patch_offset(self.h, p)

    def set_launch_mode(self, mode):
        """LAUNCH_PERSISTENT (one launch per stage over the tile table) or
        LAUNCH_PER_PATCH (one launch per patch)."""
        _check(lib().vp_launch_mode_set(self.h, int(mode)))

    def set_face_scheme(self, scheme):
        """FACE_CENTERED (ideal weights) or FACE_LIMITED (section 2, eq. limitedFace)."""
        _check(lib().vp_face_scheme_set(self.h, int(scheme)))

    def set_reduction(self, algorithm):
        """REDUCE_SUBPATCH (Alg. spreduce), REDUCE_MASK (Alg. mreduce) or REDUCE_FUSED
        (the Mask reduction from the stage kernels' row sums, the default), two-level plans."""
        _check(lib().vp_reduction_set(self.h, int(algorithm)))

    def autotune(self, f, a, dt, reps=3):
        """Times every tile shape on `reps` RK4 steps of copies of (f, a),
        selects the fastest; returns (index, shape, ms per step)."""
        self._state(f, "f")
        self._cfg(a, "a", self.field_elems)
        fw, aw = f.clone(), a.clone()
        best, ms = ctypes.c_int32(), ctypes.c_float()
        _check(lib().vp_autotune(self.h, _ptr(fw), _ptr(aw), ctypes.c_double(dt), int(reps), _ptr(self.work),
                                 _stream(), ctypes.byref(best), ctypes.byref(ms)))
        return best.value, self.tile_shapes()[best.value], ms.value

    # ---------------------------------------------------------------- checks
    def _state(self, t, name):
        if not (t.is_cuda and t.dtype == self.dtype and t.is_contiguous() and t.numel() == self.state_elems):
            raise ValueError(f"{name}: expected a contiguous {self.dtype} CUDA tensor of {self.state_elems} "
                             f"elements, got {t.dtype} {tuple(t.shape)} on {t.device}")
        return t

    def _cfg(self, t, name, n):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == n):
            raise ValueError(f"{name}: expected a contiguous float64 CUDA tensor of {n} elements")
        return t


def two_level_spec(ncx, ncv, x_len, v_lo, v_hi, qm, ratio, veq_c, veq_f, x_lo=0.0):
    """Problem spec of a two-level 1D+1V hierarchy (level 0: ncx x ncv)."""
    return {"ndim": 1, "n_levels": 2, "cells": [ncx, ncv], "ratio": [ratio, ratio], "x_lo": [x_lo],
            "x_len": [x_len], "v_lo": [v_lo], "v_hi": [v_hi], "qm": qm, "veq": [[veq_c], [veq_f]]}


def hierarchy_spec(ncx, ncv, x_len, v_lo, v_hi, qm, ratios, veqs, x_lo=0.0):
    """Problem of a 1D+1V hierarchy of len(ratios) + 1 levels: ratios[l] =
    (r_x, r_v) of level l -> l+1; veqs[l]: level-l equilibrium with two ghost
    cells per side."""
    return {"ndim": 1, "n_levels": len(ratios) + 1, "cells": [ncx, ncv], "ratios": [list(r) for r in ratios],
            "x_lo": [x_lo], "x_len": [x_len], "v_lo": [v_lo], "v_hi": [v_hi], "qm": qm,
            "veq": [[list(v)] for v in veqs]}


def amr4d_spec(ncells, x_len, y_len, v_lo, v_hi, qm, ratio, veqs):
    """Problem of a two-level 2D+2V hierarchy: level 0 of ncells = (nx, ny,
    nvx, nvy) cells, one ratio in every direction, the same velocity
    interval along vx and vy; veqs = (gx, gy) of level 0 and of level 1, each
    with two ghost cells per side."""
    gxc, gyc, gxf, gyf = veqs
    return {"ndim": 2, "n_levels": 2, "cells": list(ncells), "ratio": [ratio] * 4, "x_lo": [0.0, 0.0],
            "x_len": [x_len, y_len], "v_lo": [v_lo, v_lo], "v_hi": [v_hi, v_hi], "qm": qm,
            "veq": [[list(gxc), list(gyc)], [list(gxf), list(gyf)]]}


def _problem_dict(p):
    """Problem spec from a vp_inputs.Problem1D / Problem2D."""
    if hasattr(p, "nvx"):
        return {"ndim": 2, "cells": [p.nx, p.ny, p.nvx, p.nvy], "x_lo": [0.0, 0.0],
                "x_len": [p.x_len, p.y_len], "v_lo": [p.v_lo, p.v_lo], "v_hi": [p.v_hi, p.v_hi],
                "qm": p.qm, "veq": [[p.veq_x, p.veq_y]]}
    return {"ndim": 1, "cells": [p.nx, p.nv], "x_lo": [p.x_lo], "x_len": [p.x_len], "v_lo": [p.v_lo],
            "v_hi": [p.v_hi], "qm": p.qm, "veq": [[p.veq]]}


# -------------------------------------------------------------------- entry points


def rhs(plan, f, a, k=None):
    plan._state(f, "f")
    plan._cfg(a, "a", plan.field_elems)
    if k is None:
        k = torch.empty_like(f)
    plan._state(k, "k")
    _check(lib().vp_rhs(plan.h, _ptr(f), _ptr(a), _ptr(k), _stream()))
    return k


def reduce_moment(plan, f, n=None):
    plan._state(f, "f")
    if n is None:
        n = torch.empty(plan.config_elems, dtype=torch.float64, device=f.device)
    plan._cfg(n, "n", plan.config_elems)
    _check(lib().vp_reduce_moment(plan.h, _ptr(f), _ptr(n), _ptr(plan.work), _stream()))
    return n


def poisson_periodic(plan, n, phi=None, E=None):
    ndir = plan.spec["ndim"]
    plan._cfg(n, "n", plan.config_elems)
    if phi is None:
        phi = torch.empty(plan.config_elems, dtype=torch.float64, device=n.device)
    if E is None:
        E = torch.empty(plan.config_elems * ndir, dtype=torch.float64, device=n.device)
    plan._cfg(phi, "phi", plan.config_elems)
    plan._cfg(E, "E", plan.config_elems * ndir)
    _check(lib().vp_poisson_periodic(plan.h, _ptr(n), _ptr(phi), _ptr(E), _ptr(plan.work), _stream()))
    return phi, E


def inject_field(plan, E, a=None):
    if a is None:
        a = torch.empty(plan.field_elems, dtype=torch.float64, device=E.device)
    plan._cfg(a, "a", plan.field_elems)
    _check(lib().vp_inject_field(plan.h, _ptr(E), _ptr(a), _stream()))
    return a


def field_of(plan, f):
    """a = (q/m) E(f): moment, Poisson and injection in sequence."""
    n = reduce_moment(plan, f)
    _, E = poisson_periodic(plan, n)
    return inject_field(plan, E)


def rk4_step(plan, f, a, dt):
    plan._state(f, "f")
    plan._cfg(a, "a", plan.field_elems)
    _check(lib().vp_rk4_step(plan.h, _ptr(f), _ptr(a), ctypes.c_double(dt), _ptr(plan.work), _stream()))
    return f, a


def rk4_step_noalloc(plan, f, a, dt):
    """vp_rk4_step with the library's static scratch array as workspace."""
    plan._state(f, "f")
    plan._cfg(a, "a", plan.field_elems)
    _check(lib().vp_rk4_step_noalloc(plan.h, _ptr(f), _ptr(a), ctypes.c_double(dt), _stream()))
    return f, a


def amr_subcycle_step(plan, f, a, dt):
    """One subcycled step of a two-level plan in place (the coarse level
    takes dt, the patches R substeps of dt / R); a out: the field of the new
    state."""
    plan._state(f, "f")
    plan._cfg(a, "a", plan.field_elems)
    _check(lib().vp_amr_subcycle_step(plan.h, _ptr(f), _ptr(a), ctypes.c_double(dt), _ptr(plan.work), _stream()))
    return f, a


def rk4_step_record(plan, f, a, dt, stages=None):
    plan._state(f, "f")
    plan._cfg(a, "a", plan.field_elems)
    if stages is None:
        stages = torch.empty(plan.stage_elems, dtype=plan.dtype, device=f.device)
    _check(lib().vp_rk4_step_record(plan.h, _ptr(f), _ptr(a), ctypes.c_double(dt), _ptr(stages),
                                    _ptr(plan.work), _stream()))
    return f, a, stages


def adjoint_step(plan, f_n, a_n, lam_np1, dt, stages=None, lam_n=None):
    plan._state(f_n, "f_n")
    plan._cfg(a_n, "a_n", plan.field_elems)
    plan._state(lam_np1, "lam_np1")
    if lam_n is None:
        lam_n = torch.empty_like(lam_np1)
    _check(lib().vp_adjoint_step(plan.h, _ptr(f_n), _ptr(a_n), _ptr(stages), _ptr(lam_np1), _ptr(lam_n),
                                 ctypes.c_double(dt), _ptr(plan.work), _stream()))
    return lam_n


def field_adjoint(plan, abar, fbar=None):
    """fbar = K^T abar: adjoint of f -> a (moment, Poisson, field, injection)."""
    plan._cfg(abar, "abar", plan.field_elems)
    if fbar is None:
        fbar = torch.empty(plan.state_elems, dtype=torch.float64, device=abar.device)
    _check(lib().vp_field_adjoint(plan.h, _ptr(abar), _ptr(fbar), _ptr(plan.work), _stream()))
    return fbar


# -------------------------------------------------------------------- regridding


def tag_cells(plan, f, tol, values=False):
    """Refinement tags of level 0 (uint8 [ncx][ncv] on the device; for a
    2D+2V plan uint8 [nx][ny][nvx][nvy]); with values=True also
    delta1 f + delta2 f per cell."""
    plan._state(f, "f")
    if plan.spec["ndim"] == 2:
        shape = tuple(plan.spec["cells"])               # every cell of the 2D+2V mesh
    else:
        shape = (plan.spec["cells"][0], plan.spec["cells"][1])
    tags = torch.empty(shape, dtype=torch.uint8, device=f.device)
    vals = torch.empty(shape, dtype=torch.float64, device=f.device) if values else None
    _check(lib().vp_tag_cells(plan.h, _ptr(f), ctypes.c_double(tol), _ptr(tags), _ptr(vals), _stream()))
    return (tags, vals) if values else tags


def cluster_tags(tags, ratio, efficiency=0.7, min_width=2, buffer=1, max_boxes=4096):
    """Level-1 boxes (dicts with level, lo, hi) covering the tagged level-0
    cells of a host uint8 [ncx][ncv] array (a numpy array or a CPU tensor)."""
    import numpy as np
    t = tags.cpu().numpy() if hasattr(tags, "cpu") else tags
    t = np.ascontiguousarray(t, dtype=np.uint8)
    ncx, ncv = t.shape
    out = (vp_box * max_boxes)()
    n = ctypes.c_int32()
    _check(lib().vp_cluster_tags(t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ncx, ncv, ratio,
                                 ctypes.c_double(efficiency), min_width, buffer, out, max_boxes, ctypes.byref(n)))
    return _boxes_out(out, n.value)


def regrid_transfer(old_plan, f_old, new_plan, f_new=None):
    """The state of new_plan from the state of old_plan after a regrid."""
    old_plan._state(f_old, "f_old")
    if f_new is None:
        f_new = torch.empty(new_plan.state_elems, dtype=new_plan.dtype, device=f_old.device)
    new_plan._state(f_new, "f_new")
    _check(lib().vp_regrid_transfer(old_plan.h, _ptr(f_old), new_plan.h, _ptr(f_new), _stream()))
    return f_new


def tag_level(plan, f, level, tol, values=False):
    """Criterion on level `level` of a multi-level plan: (tags, values or None)
    as [nx_l, nv_l] device tensors (values NaN where the level has no patch)."""
    plan._state(f, "f")
    nx, nv = plan.level_shape(level)
    tags = torch.empty((nx, nv), dtype=torch.uint8, device=f.device)
    vals = torch.empty((nx, nv), dtype=torch.float64, device=f.device) if values else None
    _check(lib().vp_tag_level(plan.h, _ptr(f), int(level), ctypes.c_double(tol), _ptr(tags), _ptr(vals),
                              _ptr(plan.work), _stream()))
    return tags, vals


def cluster_level(plan, level, tags, ratio, efficiency=0.7, min_width=2, buffer=1, max_size=(0, 0), max_boxes=4096):
    """Level-(level+1) boxes nested in the plan's level `level` from host tags."""
    t = np.ascontiguousarray(tags.cpu().numpy() if hasattr(tags, "cpu") else tags, dtype=np.uint8)
    arr = (vp_box * max_boxes)()
    n = ctypes.c_int32()
    _check(lib().vp_cluster_level(plan.h, int(level), t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                  int(ratio[0]), int(ratio[1]), ctypes.c_double(efficiency), int(min_width),
                                  int(buffer), int(max_size[0]), int(max_size[1]), arr, max_boxes, ctypes.byref(n)))
    return _boxes_out(arr, n.value)


def regrid(plan, f, tol, efficiency=0.7, min_width=2, buffer=1):
    """Regrid a two-level plan: tag level 0, cluster on the host, create the
    plan of the new hierarchy and transfer the state.  Returns
    (new_plan, f_new, boxes)."""
    tags = tag_cells(plan, f, tol)
    boxes = cluster_tags(tags.cpu(), plan.spec["ratio"][0], efficiency, min_width, buffer)
    new_plan = Plan(plan.spec, dtype=plan.dtype, boxes=boxes, device=plan.device)
    return new_plan, regrid_transfer(plan, f, new_plan), boxes


# -------------------------------------------------------------------- adaptive run


class AmrRun:
    """Adaptive run (vp_amr_run): RK4 steps with a time step limited by the
    stability condition, regridding every regrid_interval steps.  spec: a
    spec dict of two or more levels (two_level_spec, hierarchy_spec); boxes:
    the initial boxes; f0: the initial state in that plan's layout;
    max_size: largest patch per level (multi-level runs)."""

    def __init__(self, spec, boxes, f0, tol, regrid_interval, efficiency=0.7, min_width=2, buffer=1, cfl=0.5,
                 dt_growth=1.1, dt_initial=0.01, charges=None, background=None, max_size=None):
        """One species: spec (a two-level spec dict), boxes, f0.  Several
        species: lists spec[s], boxes[s], f0[s] and their charges; the field
        of rho = background + sum_s charge_s n_s."""
        if not torch.cuda.is_available():
            raise RuntimeError("the Vlasov-Poisson library needs a HIP GPU (torch.cuda is unavailable)")
        prm = vp_amr_params(float(tol), int(regrid_interval), float(efficiency), int(min_width), int(buffer),
                            float(cfl), float(dt_growth), float(dt_initial))
        for lvl, (mx, mv) in enumerate(max_size or []):       # largest patch per level, in its own cells
            prm.max_size[lvl][0], prm.max_size[lvl][1] = int(mx), int(mv)
        several = charges is not None
        specs, blist, flist = (spec, boxes, f0) if several else ([spec], [boxes], [f0])
        for f in flist:
            if f.dtype != torch.float64 or not f.is_cuda or not f.is_contiguous():
                raise ValueError("f0: contiguous float64 tensor on the GPU expected")
        h = ctypes.c_void_p()
        if several:
            n = len(specs)
            made = [_make_problem(sp, torch.float64) for sp in specs]
            self._keep = made
            pbs = (ctypes.POINTER(vp_problem) * n)(*[ctypes.pointer(m[0]) for m in made])
            bxs = [_make_boxes(b) for b in blist]
            self._keep_boxes = bxs
            bptr = (ctypes.POINTER(vp_box) * n)(*[ctypes.cast(b[0], ctypes.POINTER(vp_box)) if b[0] is not None
                                                  else ctypes.POINTER(vp_box)() for b in bxs])
            nb = (ctypes.c_int32 * n)(*[b[1] for b in bxs])
            fp = (_P * n)(*[f.data_ptr() for f in flist])
            ch = (ctypes.c_double * n)(*[float(c) for c in charges])
            _check(lib().vp_amr_run_create_species(n, pbs, bptr, nb, fp, ch, ctypes.c_double(background or 0.0),
                                                   ctypes.byref(prm), ctypes.byref(h), _stream()))
        else:
            pb, keep = _make_problem(spec, torch.float64)
            bx, nbox = _make_boxes(boxes)
            _check(lib().vp_amr_run_create(ctypes.byref(pb), bx, nbox, _ptr(f0), ctypes.byref(prm),
                                           ctypes.byref(h), _stream()))
        self.h = h
        self.spec = spec
        self.device = flist[0].device

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.vp_amr_run_destroy(self.h)
            self.h = None

    def advance(self, steps):
        _check(lib().vp_amr_run_advance(self.h, int(steps), _stream()))

    def info(self):
        i = vp_amr_info()
        _check(lib().vp_amr_run_info(self.h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in vp_amr_info._fields_}

    @property
    def species_count(self):
        return lib().vp_amr_run_species_count(self.h)

    def boxes(self, species=0):
        n = ctypes.c_int32()
        cap = max(self.info()["npatch"], 1)
        arr = (vp_box * cap)()
        _check(lib().vp_amr_run_boxes_of(self.h, species, arr, cap, ctypes.byref(n)))
        return _boxes_out(arr, n.value)

    def state(self, species=0):
        """A copy of the current state of a species (layout of its current hierarchy)."""
        n = lib().vp_state_elems(lib().vp_amr_run_plan_of(self.h, species))
        out = torch.empty(n, dtype=torch.float64, device=self.device)
        _check(lib().vp_amr_run_read_state_of(self.h, species, _ptr(out), n, _stream()))
        return out


# -------------------------------------------------------------------- several species


class SpeciesGroup:
    """Species on one configuration mesh (vp_species_group): plans of 1D+1V
    problems, single-level or two-level (each with its own velocity mesh,
    boxes and qm) sharing the finest configuration mesh, their charges, and
    a uniform neutralising background; rho = background + sum_s charge_s n_s."""

    def __init__(self, plans, charges, background=0.0):
        n = len(plans)
        hs = (_P * n)(*[p.h.value for p in plans])
        ch = (ctypes.c_double * n)(*[float(c) for c in charges])
        h = ctypes.c_void_p()
        _check(lib().vp_species_group_create(hs, ch, n, ctypes.c_double(background), ctypes.byref(h)))
        self.h = h
        self.plans = list(plans)
        self.charges = [float(c) for c in charges]
        self.background = float(background)
        self.gwork = torch.empty(max(lib().vp_species_workspace_bytes(h), 1), dtype=torch.uint8,
                                 device=plans[0].device)

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.vp_species_group_destroy(self.h)
            self.h = None

    def _lists(self, fs, as_):
        if len(fs) != len(self.plans) or len(as_) != len(self.plans):
            raise ValueError("one state and one acceleration per species expected")
        for p, f, a in zip(self.plans, fs, as_):
            p._state(f, "f")
            p._cfg(a, "a", p.field_elems)
        n = len(self.plans)
        return (_P * n)(*[f.data_ptr() for f in fs]), (_P * n)(*[a.data_ptr() for a in as_])

    def field(self, fs, as_=None):
        """[a_s = (q/m)_s E] of the states fs."""
        if as_ is None:
            as_ = [torch.empty(p.field_elems, dtype=torch.float64, device=p.device) for p in self.plans]
        fp, ap = self._lists(fs, as_)
        wp = (_P * len(self.plans))(*[p.work.data_ptr() for p in self.plans])
        _check(lib().vp_species_field(self.h, fp, ap, wp, _ptr(self.gwork), _stream()))
        return as_

    def rk4_step(self, fs, as_, dt):
        """One RK4 step of every species in place; as_ in/out."""
        fp, ap = self._lists(fs, as_)
        wp = (_P * len(self.plans))(*[p.work.data_ptr() for p in self.plans])
        _check(lib().vp_species_rk4_step(self.h, fp, ap, ctypes.c_double(dt), wp, _ptr(self.gwork), _stream()))
        return fs, as_
