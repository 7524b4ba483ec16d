// Host runtime and C ABI of the MI355X Vlasov-Poisson library: plan
// creation and validation, workspace layout, and the enqueue sequences of
// the entry points declared in include/vp.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "vp_internal.hpp"

namespace vp {

namespace {
thread_local std::string g_last_error;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Periodic Green's function of (S + S^-1 - 14) on n cells:
//   g_k = c (r^k + r^(n-k)) / (1 - r^n),  r = 1 / (7 + sqrt 48),  c = -1 / (1/r - r),
// the sum over periodic images of the free-space solution c r^|k|.
std::vector<double> tridiag_green(int n, int taps)
{
    const double r = 1.0 / (7.0 + std::sqrt(48.0));
    const double c = -1.0 / (1.0 / r - r);
    const double rn = std::pow(r, n);
    const int cnt = (n <= 2 * taps + 1) ? n : taps + 1;
    std::vector<double> g(cnt);
    for (int k = 0; k < cnt; ++k) g[k] = c * (std::pow(r, k) + std::pow(r, n - k)) / (1.0 - rn);
    return g;
}

// shapes compiled into the stage-kernel dispatch, per dtype
const int kTxChoices[] = {8, 16, 32, 64, 128};
std::vector<StageShape> shape_table(int dtype)
{
    std::vector<StageShape> v;
    const int nw[][2] = {{64, 2}, {128, 2}, {256, 2}};
    const int nwf[][2] = {{64, 4}, {128, 4}};
    if (dtype == VP_F64) {
        for (auto& a : nw)
            for (int tx : kTxChoices) v.push_back(StageShape{a[0], a[1], tx});
    } else {
        for (auto& a : nwf)
            for (int tx : kTxChoices) v.push_back(StageShape{a[0], a[1], tx});
    }
    return v;
}

StageShape pick_shape(const vp_plan* p, std::initializer_list<const void*> ptrs)
{
    bool al = true;
    for (const void* q : ptrs)
        if (q && !aligned16(q)) al = false;
    if (p->dtype == VP_F64) {
        if (al && p->nv % 2 == 0) return p->shape;
        return StageShape{128, 1, p->shape.tx};
    }
    if (al && p->nv % 4 == 0) return p->shape;
    return StageShape{128, 1, p->shape.tx};
}

int strips_for(const vp_plan* p, const StageShape& sh)
{
    const int tv = sh.nt * sh.w;
    return (p->nv + tv - 1) / tv;
}

char* wsp(void* work, size_t off) { return static_cast<char*>(work) + off; }

Stage1DArgs base_args(const vp_plan* p, const StageShape& sh)
{
    Stage1DArgs a{};
    a.nx = p->nx;
    a.nv = p->nv;
    a.tx = sh.tx;
    a.nstrip = strips_for(p, sh);
    a.dxi = 1.0 / p->dx;
    a.dvi = 1.0 / p->dv;
    a.dv24 = p->dv / 24.0;
    a.v_lo = p->v_lo;
    a.dv = p->dv;
    for (int q = 0; q < 4; ++q) a.vg[q] = p->vg[q];
    a.lim = p->face_scheme == VP_FACE_LIMITED;
    return a;
}

vp_status check_plan(const vp_plan* p)
{
    if (!p) return fail(VP_EINVAL, "plan is NULL");
    return VP_OK;
}

}  // namespace

std::vector<double> poisson_green_table(int n) { return tridiag_green(n, kGreenTaps); }

Rk4Setup1D rk4_setup_1d(const vp_plan* p, void* f, void* work, double dt, void* st_f)
{
    Rk4Setup1D R{};
    const size_t sb = p->state_elems * p->esize;
    void* acc = wsp(work, p->ws_acc);
    void* s2 = st_f ? st_f : wsp(work, p->ws_fsa);
    void* s3 = st_f ? static_cast<char*>(st_f) + sb : wsp(work, p->ws_fsb);
    void* s4 = st_f ? static_cast<char*>(st_f) + 2 * sb : wsp(work, p->ws_fsa);
    R.part = reinterpret_cast<double*>(wsp(work, p->ws_part));
    R.sh = pick_shape(p, {f, acc, s2, s3, s4});
    R.A = base_args(p, R.sh);
    R.A.part = R.part;
    R.A.fn = f;
    R.A.acc = acc;
    // the lean schedule: stage 2 adds dt/3 k2 to the accumulator, stage 4
    // dt/6 k4 (the other slopes come from the predictors)
    const double cacc[4] = {0.0, dt / 3.0, 0.0, dt / 6.0};
    const double cnext[4] = {0.5 * dt, 0.5 * dt, dt, 0.0};
    const int kinds[4] = {kLean1, kLean2, kLean3, kLean4};
    const void* in[4] = {f, s2, s3, s4};
    void* out[4] = {s2, s3, s4, f};
    for (int s = 0; s < 4; ++s) {
        R.in[s] = in[s];
        R.out[s] = out[s];
        R.c_acc[s] = cacc[s];
        R.c_next[s] = cnext[s];
        R.kind[s] = kinds[s];
    }
    return R;
}

Stage1DArgs rk4_stage_args_1d(const Rk4Setup1D& R, int s, const double* a)
{
    Stage1DArgs A = R.A;
    A.fs = R.in[s];
    A.fout = R.out[s];
    A.a = a;
    A.c_acc = R.c_acc[s];
    A.c_next = R.c_next[s];
    return A;
}

namespace {

// one RK4 step; stage states go to st[0..2] (or the workspace ping-pong
// buffers) and stage accelerations to sa[0..3] (or in place in `a`)
vp_status rk4_1d(const vp_plan* p, void* f, double* a, double dt, void* work, void* st_f,
                 double* st_a, hipStream_t stream)
{
    const Rk4Setup1D R = rk4_setup_1d(p, f, work, dt, st_f);
    const StageShape sh = R.sh;
    double* part = R.part;
    double* ncfg = reinterpret_cast<double*>(wsp(work, p->ws_cfg));
    double* sa[5] = {a, a, a, a, a};
    if (st_a) {
        VP_HIP(hipMemcpyAsync(st_a, a, sizeof(double) * p->nx, hipMemcpyDeviceToDevice, stream));
        for (int s = 0; s < 4; ++s) sa[s] = st_a + (size_t)s * p->nx;
    }
    for (int s = 0; s < 4; ++s) {
        const Stage1DArgs A = rk4_stage_args_1d(R, s, sa[s]);
        const int kind = R.kind[s];
        VP_HIP(timed(p, kTStage, stream, [&] { return launch_stage1d(p->dtype, sh, kind, A, stream); }));
        double* a_next = (s < 3) ? sa[s + 1] : a;
        VP_HIP(timed(p, kTField, stream, [&] {
            if (p->nx >= kFieldSplitMin)
                return launch_field_split(part, A.nstrip, p->nx, p->dv, p->dx, p->pb.qm, p->d_green, ncfg, a_next,
                                          stream);
            return launch_poisson1d(part, A.nstrip, nullptr, p->dv, p->nx, p->dx, p->pb.qm, p->d_green, p->gk,
                                    ncfg, nullptr, nullptr, a_next, stream);
        }));
    }
    return VP_OK;
}

// The allocation-free RK4 step keeps its workspace in this file-scope
// device array (each device holds its own copy until the process ends).
// On the host the array's name is only a stand-in for the symbol, never a
// device address: host code takes the address once per device with
// hipGetSymbolAddress (scratch_address) and passes that pointer on.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// device address of `scratch` on the current device (looked up on the first
// call on that device, with that device current)
vp_status scratch_address(void** out)
{
    int dev = -1;
    VP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) return fail(VP_ENOTSUP, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        VP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(VP_EHIP, "hipGetSymbolAddress returned a null address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return VP_OK;
}

// plan of two or more levels: geometry, box calculus and tables (two-level
// engine in vp_amr.hip, multi-level engine in vp_hier.hip), then the Poisson
// tables of the finest configuration mesh
vp_status create_multi_level(const vp_problem* pb, const vp_box* boxes, int nbox, vp_plan** out, bool force_hier,
                             bool tag_only = false)
{
    vp_plan* p = new (std::nothrow) vp_plan();
    if (!p) return fail(VP_ENOMEM, "out of host memory");
    p->pb = *pb;
    p->ndim = pb->ndim;
    p->dtype = pb->dtype;
    p->nlev = 2;
    p->esize = pb->dtype == VP_F64 ? 8 : 4;
    for (int l = 0; l < VP_MAX_LEVELS; ++l)
        for (int d = 0; d < 2; ++d) p->pb.veq[l][d] = nullptr;
    p->nlev = pb->n_levels;
    // two levels with one ratio (2 or 4) in x and v take the two-level engine
    // (ghost interpolation fused into the stage tiles, subcycling, species,
    // adaptive runs); deeper or anisotropic hierarchies the multi-level one
    const bool two = !force_hier && pb->n_levels == 2 && pb->ratio[0][0] == pb->ratio[0][1] &&
                     (pb->ratio[0][0] == 2 || pb->ratio[0][0] == 4);
    vp_status st = two ? amr_create(p, pb, boxes, nbox) : hier_create(p, pb, boxes, nbox, tag_only);
    if (st == VP_OK) {
        // kept so that a plan of another hierarchy can be made from this one
        int nv = pb->cells[1];
        for (int l = 0; l < pb->n_levels; ++l) {
            if (l > 0) nv *= pb->ratio[l - 1][1];
            p->veq[l][0].assign(pb->veq[l][0], pb->veq[l][0] + nv + 4);
        }
    }
    if (st != VP_OK) {
        amr_destroy(p);
        hier_destroy(p);
        delete p;
        return st;
    }
    // the configuration-space calls act on the finest configuration mesh
    if (p->amr) {
        const AmrPlan& M = *p->amr;
        p->nx = M.nfx;
        p->nv = M.nfv;
        p->dx = M.dxf;
        p->dv = M.dvf;
        p->v_lo = M.v_lo;
    } else {
        const HierPlan& H = *p->hier;
        p->nx = H.lv[H.L - 1].nx;
        p->nv = H.lv[H.L - 1].nv;
        p->dx = H.dxf;
        p->dv = H.lv[H.L - 1].dv;
        p->v_lo = pb->v_lo[0];
        if (H.tag_only) {
            *out = p;
            return VP_OK;
        }
    }
    std::vector<double> g = tridiag_green(p->nx, kGreenTaps);
    p->gk = kGreenTaps;
    hipError_t e = hipMalloc(&p->d_green, g.size() * sizeof(double));
    if (e == hipSuccess)
        e = hipMemcpy(p->d_green, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = poisson1d_prepare();
    if (e != hipSuccess) {
        st = hip_fail(e, "vp_plan_create: Poisson tables");
        if (p->d_green) (void)hipFree(p->d_green);
        amr_destroy(p);
        hier_destroy(p);
        delete p;
        return st;
    }
    *out = p;
    return VP_OK;
}

// two-level 2D+2V plan (vp_amr4d.hip): the configuration-space calls act
// on the fine configuration mesh
vp_status create_amr4d(const vp_problem* pb, const vp_box* boxes, int nbox, vp_plan** out)
{
    if (pb->n_levels != 2) return fail(VP_ENOTSUP, "2D+2V hierarchies have two levels");
    vp_plan* p = new (std::nothrow) vp_plan();
    if (!p) return fail(VP_ENOMEM, "out of host memory");
    p->pb = *pb;
    p->ndim = 2;
    p->dtype = pb->dtype;
    p->nlev = 2;
    p->esize = 8;
    for (int l = 0; l < VP_MAX_LEVELS; ++l)
        for (int d = 0; d < 2; ++d) p->pb.veq[l][d] = nullptr;
    vp_status st = a4_create(p, pb, boxes, nbox);
    if (st != VP_OK) {
        a4_destroy(p);
        delete p;
        return st;
    }
    p->nx = p->a4->nf[0] * p->a4->nf[1];
    p->shape = StageShape{256, 1, 1};
    *out = p;
    return VP_OK;
}

// single-level 2D+2V plan (vp_4d.hip)
vp_status create_4d(const vp_problem* pb, vp_plan** out)
{
    vp_plan* p = new (std::nothrow) vp_plan();
    if (!p) return fail(VP_ENOMEM, "out of host memory");
    p->pb = *pb;
    p->ndim = 2;
    p->dtype = pb->dtype;
    p->nlev = 1;
    p->esize = 8;
    for (int l = 0; l < VP_MAX_LEVELS; ++l)
        for (int d = 0; d < 2; ++d) p->pb.veq[l][d] = nullptr;
    vp_status st = p4_create(p, pb);
    if (st != VP_OK) {
        p4_destroy(p);
        delete p;
        return st;
    }
    p->nx = pb->cells[0] * pb->cells[1];        // configuration cells
    p->shape = StageShape{1024, 4, 4};
    *out = p;
    return VP_OK;
}

// 2D+2V shapes: threads, then a tile of w x tx configuration cells (one wave per cell)
std::vector<StageShape> shape_table_4d()
{
    return {StageShape{1024, 4, 4}, StageShape{512, 2, 4}, StageShape{512, 4, 2}, StageShape{256, 2, 2}};
}

// two-level tile shapes: threads x cells per thread x rows per tile
std::vector<StageShape> amr_shape_table()
{
    std::vector<StageShape> v;
    for (int w : {2, 1})
        for (int nt : {64, 128})
            for (int tx : {4, 8, 16, 32}) v.push_back(StageShape{nt, w, tx});
    return v;
}

std::vector<StageShape> plan_shapes(const vp_plan* p)
{
    if (p->p4) return shape_table_4d();
    if (p->a4) return {StageShape{256, 1, 1}};
    return (p->amr || p->hier) ? amr_shape_table() : shape_table(p->dtype);
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

vp_status fail(vp_status code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

vp_status hip_fail(hipError_t e, const char* what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return VP_EHIP;
}

vp_status hier_plan_create(const vp_problem* pb, const vp_box* boxes, int nbox, vp_plan** out, bool tag_only)
{
    if (!pb || !out) return fail(VP_EINVAL, "hier_plan_create: NULL pointer");
    *out = nullptr;
    if (pb->n_levels < 2 || pb->n_levels > VP_MAX_LEVELS) return fail(VP_EINVAL, "n_levels must be 2 .. 4");
    if (!pb->veq[0][0]) return fail(VP_EINVAL, "veq[0][0] (equilibrium with ghosts) is required");
    return create_multi_level(pb, boxes, nbox, out, true, tag_only);
}

}  // namespace vp

using namespace vp;

extern "C" {

const char* vp_last_error(void) { return g_last_error.c_str(); }

vp_status vp_plan_create(const vp_problem* pb, const vp_box* boxes, int32_t nbox, vp_plan** out)
{
    if (!pb || !out) return fail(VP_EINVAL, "vp_plan_create: NULL problem or output pointer");
    *out = nullptr;
    if (pb->ndim != 1 && pb->ndim != 2) return fail(VP_EINVAL, "ndim must be 1 or 2");
    if (pb->dtype != VP_F64 && pb->dtype != VP_F32) return fail(VP_EDTYPE, "dtype must be VP_F64 or VP_F32");
    if (pb->n_levels < 1 || pb->n_levels > VP_MAX_LEVELS) return fail(VP_EINVAL, "n_levels must be 1 .. 4");
    if (nbox < 0 || (nbox > 0 && !boxes)) return fail(VP_EINVAL, "bad box list");
    const int nd = 2 * pb->ndim;
    for (int d = 0; d < nd; ++d)
        if (pb->cells[d] < 1) return fail(VP_EINVAL, "cells must be positive");
    for (int d = 0; d < pb->ndim; ++d) {
        if (!(pb->x_len[d] > 0.0)) return fail(VP_EINVAL, "x_len must be positive");
        if (!(pb->v_hi[d] > pb->v_lo[d])) return fail(VP_EINVAL, "v_hi must exceed v_lo");
        if (!pb->veq[0][d]) return fail(VP_EINVAL, "veq[0][d] (equilibrium with ghosts) is required");
    }
    if (pb->n_levels >= 2 && pb->ndim == 2) return create_amr4d(pb, boxes, nbox, out);
    if (pb->n_levels >= 2) return create_multi_level(pb, boxes, nbox, out, false);
    if (nbox != 0) return fail(VP_EINVAL, "a single-level plan takes no boxes");
    if (pb->ndim == 2) return create_4d(pb, out);

    vp_plan* p = new (std::nothrow) vp_plan();
    if (!p) return fail(VP_ENOMEM, "out of host memory");
    p->pb = *pb;
    p->ndim = pb->ndim;
    p->dtype = pb->dtype;
    p->nlev = pb->n_levels;
    p->esize = pb->dtype == VP_F64 ? 8 : 4;
    p->nx = pb->cells[0];
    p->nv = pb->cells[1];
    p->dx = pb->x_len[0] / p->nx;
    p->dv = (pb->v_hi[0] - pb->v_lo[0]) / p->nv;
    p->v_lo = pb->v_lo[0];
    p->veq[0][0].assign(pb->veq[0][0], pb->veq[0][0] + p->nv + 4);
    p->vg[0] = p->veq[0][0][0];
    p->vg[1] = p->veq[0][0][1];
    p->vg[2] = p->veq[0][0][p->nv + 2];
    p->vg[3] = p->veq[0][0][p->nv + 3];
    for (int l = 0; l < VP_MAX_LEVELS; ++l)
        for (int d = 0; d < 2; ++d) p->pb.veq[l][d] = nullptr;
    if (p->nx > kMaxPoisson1D) {
        delete p;
        return fail(VP_ENOTSUP, "configuration mesh larger than 8192 cells");
    }
    p->shape = p->dtype == VP_F64 ? StageShape{256, 2, 16} : StageShape{128, 4, 16};
    p->state_elems = (size_t)p->nx * p->nv;

    // Poisson tables
    std::vector<double> g = tridiag_green(p->nx, kGreenTaps);
    p->gk = kGreenTaps;
    hipError_t e = hipMalloc(&p->d_green, g.size() * sizeof(double));
    if (e == hipSuccess)
        e = hipMemcpy(p->d_green, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = poisson1d_prepare();
    if (e != hipSuccess) {
        vp_status st = hip_fail(e, "vp_plan_create: Poisson tables");
        if (p->d_green) (void)hipFree(p->d_green);
        delete p;
        return st;
    }

    // workspace: acc, two predictor buffers, moment partials, config scratch
    const size_t sb = align256(p->state_elems * p->esize);
    const int max_strips = (p->nv + 63) / 64;
    size_t off = 0;
    p->ws_acc = off; off += sb;
    p->ws_fsa = off; off += sb;
    p->ws_fsb = off; off += sb;
    p->ws_part = off; off += align256((size_t)max_strips * p->nx * sizeof(double));
    p->ws_cfg = off; off += align256((size_t)8 * p->nx * sizeof(double));
    p->ws_step = off;
    if (p->dtype == VP_F64) {   // adjoint recompute: copy of f_n and a_n, stage record
        p->ws_tmpf = off; off += sb;
        p->ws_tmpa = off; off += align256((size_t)p->nx * sizeof(double));
        p->ws_stages = off; off += align256(3 * p->state_elems * p->esize + 4 * (size_t)p->nx * sizeof(double));
    }
    p->ws_total = off;
    *out = p;
    return VP_OK;
}

int32_t vp_tile_shape_count(const vp_plan* p)
{
    return p ? (int32_t)plan_shapes(p).size() : 0;
}

vp_status vp_tile_shape_get(const vp_plan* p, int32_t index, int32_t* threads, int32_t* cells, int32_t* rows)
{
    if (vp_status s = check_plan(p)) return s;
    const auto tab = plan_shapes(p);
    if (index < 0 || index >= (int32_t)tab.size()) return fail(VP_EINVAL, "vp_tile_shape_get: index out of range");
    if (threads) *threads = tab[index].nt;
    if (cells) *cells = tab[index].w;
    if (rows) *rows = tab[index].tx;
    return VP_OK;
}

vp_status vp_tile_shape_set(vp_plan* p, int32_t index)
{
    if (vp_status s = check_plan(p)) return s;
    const auto tab = plan_shapes(p);
    if (index < 0 || index >= (int32_t)tab.size()) return fail(VP_EINVAL, "vp_tile_shape_set: index out of range");
    if (p->amr) {
        if (vp_status s = amr_set_shape(p, tab[index].nt, tab[index].w, tab[index].tx)) return s;
    }
    if (p->hier) {
        if (vp_status s = hier_set_shape(p, tab[index].nt, tab[index].w, tab[index].tx)) return s;
    }
    if (p->p4) {
        p->p4->tile_x = tab[index].w;
        p->p4->tile_y = tab[index].tx;
    }
    p->shape = tab[index];
    return VP_OK;
}

vp_status vp_face_scheme_set(vp_plan* p, int32_t scheme)
{
    if (vp_status s = check_plan(p)) return s;
    if (scheme != VP_FACE_CENTERED && scheme != VP_FACE_LIMITED)
        return fail(VP_EINVAL, "vp_face_scheme_set: unknown scheme");
    if (scheme == VP_FACE_LIMITED && (p->hier || p->p4 || p->a4))
        return fail(VP_ENOTSUP, "vp_face_scheme_set: limited faces are built for 1D+1V plans of one or two levels");
    p->face_scheme = scheme;
    return VP_OK;
}

vp_status vp_reduction_set(vp_plan* p, int32_t algorithm)
{
    if (vp_status s = check_plan(p)) return s;
    if (algorithm != VP_REDUCE_SUBPATCH && algorithm != VP_REDUCE_MASK && algorithm != VP_REDUCE_FUSED)
        return fail(VP_EINVAL, "vp_reduction_set: unknown algorithm");
    if (p->hier && algorithm != VP_REDUCE_SUBPATCH)
        return fail(VP_ENOTSUP, "vp_reduction_set: multi-level plans use the Sub-Patch reduction");
    if (p->a4 && algorithm != VP_REDUCE_MASK)
        return fail(VP_ENOTSUP, "vp_reduction_set: two-level 2D+2V plans use the Mask reduction");
    if (p->amr) p->amr->reduce_mode = algorithm;
    return VP_OK;
}

vp_status vp_launch_mode_set(vp_plan* p, int32_t mode)
{
    if (vp_status s = check_plan(p)) return s;
    if (mode != VP_LAUNCH_PERSISTENT && mode != VP_LAUNCH_PER_PATCH)
        return fail(VP_EINVAL, "vp_launch_mode_set: unknown mode");
    if (p->amr) p->amr->mode = mode;
    if ((p->hier || p->a4) && mode != VP_LAUNCH_PERSISTENT)
        return fail(VP_ENOTSUP, "vp_launch_mode_set: multi-level and 2D+2V plans use the persistent launch");
    return VP_OK;
}

vp_status vp_autotune(vp_plan* p, void* f, double* a, double dt, int32_t reps, void* work, hipStream_t stream,
                      int32_t* best_index, float* best_ms)
{
    if (vp_status s = check_plan(p)) return s;
    if (!f || !a || !work) return fail(VP_EINVAL, "vp_autotune: NULL pointer");
    if (reps < 1 || !std::isfinite(dt)) return fail(VP_EINVAL, "vp_autotune: reps must be positive and dt finite");
    const auto tab = plan_shapes(p);
    const StageShape keep = p->shape;
    const bool timing = p->timing.enabled;
    p->timing.enabled = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    VP_HIP(hipEventCreate(&e0));
    VP_HIP(hipEventCreate(&e1));
    // every shape is timed in three interleaved passes and keeps its fastest
    // pass, so that a slow moment of the device does not decide the choice
    constexpr int kPasses = 3;
    std::vector<float> tmin(tab.size(), -1.f);
    vp_status st = VP_OK;
    for (int pass = 0; pass < kPasses && st == VP_OK; ++pass) {
        for (int k = 0; k < (int)tab.size() && st == VP_OK; ++k) {
            if (vp_tile_shape_set(p, k) != VP_OK) continue;      // shape not valid for this plan
            st = vp_rk4_step(p, f, a, dt, work, stream);         // warm-up
            if (st != VP_OK) break;
            hipError_t e = hipEventRecord(e0, stream);
            for (int r = 0; r < reps && st == VP_OK && e == hipSuccess; ++r)
                st = vp_rk4_step(p, f, a, dt, work, stream);
            if (e == hipSuccess) e = hipEventRecord(e1, stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) st = hip_fail(e, "vp_autotune: timing");
            if (st == VP_OK && (tmin[k] < 0.f || t < tmin[k])) tmin[k] = t;
        }
    }
    int best = -1;
    float best_t = 0.f;
    for (int k = 0; k < (int)tab.size(); ++k)
        if (tmin[k] >= 0.f && (best < 0 || tmin[k] < best_t)) { best = k; best_t = tmin[k]; }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->timing.enabled = timing;
    if (st != VP_OK) return st;
    if (best < 0) return fail(VP_ENOTSUP, "vp_autotune: no tile shape is valid for this plan");
    if (vp_status s = vp_tile_shape_set(p, best)) return s;
    (void)keep;
    if (best_index) *best_index = best;
    if (best_ms) *best_ms = best_t / reps;
    return VP_OK;
}

vp_status vp_timing_enable(vp_plan* p, int32_t enable)
{
    if (vp_status s = check_plan(p)) return s;
    Timing& T = p->timing;
    if (enable && T.ev.empty()) {
        T.ev.resize(2 * Timing::kMaxRecords, nullptr);
        T.cls.resize(Timing::kMaxRecords, 0);
        for (auto& e : T.ev) VP_HIP(hipEventCreate(&e));
    }
    T.enabled = enable != 0;
    T.used = 0;
    return VP_OK;
}

vp_status vp_timing_read(vp_plan* p, double* ms, int64_t* counts, int32_t nclass)
{
    if (vp_status s = check_plan(p)) return s;
    if (!ms || !counts || nclass < 1) return fail(VP_EINVAL, "vp_timing_read: bad output arrays");
    for (int c = 0; c < nclass; ++c) { ms[c] = 0.0; counts[c] = 0; }
    Timing& T = p->timing;
    for (int r = 0; r < T.used; ++r) {
        VP_HIP(hipEventSynchronize(T.ev[2 * r + 1]));
        float t = 0.f;
        VP_HIP(hipEventElapsedTime(&t, T.ev[2 * r], T.ev[2 * r + 1]));
        const int c = T.cls[r];
        if (c < nclass) { ms[c] += t; counts[c] += 1; }
    }
    T.used = 0;
    return VP_OK;
}

vp_status vp_plan_destroy(vp_plan* p)
{
    if (!p) return VP_OK;
    for (auto& e : p->timing.ev)
        if (e) (void)hipEventDestroy(e);
    if (p->d_green) (void)hipFree(p->d_green);
    amr_destroy(p);
    hier_destroy(p);
    p4_destroy(p);
    a4_destroy(p);
    delete p;
    return VP_OK;
}

size_t vp_state_elems(const vp_plan* p) { return p ? p->state_elems : 0; }

int64_t vp_patch_offset(const vp_plan* p, int32_t patch)
{
    if (!p) return -1;
    if (patch == -1) return 0;
    if (p->amr && patch >= 0 && patch < (int32_t)p->amr->patches.size()) return p->amr->patches[patch].off;
    if (p->hier && patch >= 0 && patch + 1 < (int32_t)p->hier->patches.size()) return p->hier->patches[patch + 1].off;
    if (p->a4 && patch >= 0 && patch + 1 < (int32_t)p->a4->patches.size()) return p->a4->patches[patch + 1].off;
    return -1;
}

size_t vp_config_elems(const vp_plan* p) { return p ? (size_t)p->nx : 0; }
size_t vp_field_elems(const vp_plan* p)
{
    if (!p) return 0;
    if (p->p4) return 2 * (size_t)p->nx;
    if (p->a4) return 2 * (size_t)(p->a4->nc[0] * p->a4->nc[1] + p->nx);
    if (p->hier) return (size_t)p->hier->na;
    return p->amr ? (size_t)(p->amr->ncx + p->amr->nfx) : (size_t)p->nx;
}
size_t vp_workspace_bytes(const vp_plan* p) { return p ? p->ws_total : 0; }

size_t vp_stage_elems(const vp_plan* p)
{
    if (!p || p->amr || p->hier || p->p4 || p->a4) return 0;
    const size_t a_bytes = 4 * (size_t)p->nx * sizeof(double);
    return 3 * p->state_elems + (a_bytes + p->esize - 1) / p->esize;
}

vp_status vp_rhs(const vp_plan* p, const void* f, const double* a, void* k, hipStream_t stream)
{
    if (vp_status s = check_plan(p)) return s;
    if (!f || !a || !k) return fail(VP_EINVAL, "vp_rhs: NULL pointer");
    if (f == k) return fail(VP_EINVAL, "vp_rhs: k must not alias f");
    if (p->amr) return amr_rhs(p, f, a, k, stream);
    if (p->hier) return hier_rhs(p, f, a, k, stream);
    if (p->p4) return p4_rhs(p, f, a, k, stream);
    if (p->a4) return a4_rhs(p, f, a, k, stream);
    const StageShape sh = pick_shape(p, {f, k});
    Stage1DArgs A = base_args(p, sh);
    A.fs = f;
    A.fout = k;
    A.a = a;
    VP_HIP(timed(p, kTStage, stream, [&] { return launch_stage1d(p->dtype, sh, kRhs, A, stream); }));
    return VP_OK;
}

vp_status vp_reduce_moment(const vp_plan* p, const void* f, double* n, void* work, hipStream_t stream)
{
    if (vp_status s = check_plan(p)) return s;
    if (!f || !n) return fail(VP_EINVAL, "vp_reduce_moment: NULL pointer");
    if (p->amr) {
        if (!work) return fail(VP_EINVAL, "vp_reduce_moment: a two-level plan needs the workspace");
        return amr_reduce(p, f, n, work, stream);
    }
    if (p->hier) {
        if (!work) return fail(VP_EINVAL, "vp_reduce_moment: a multi-level plan needs the workspace");
        return hier_reduce(p, f, n, work, stream);
    }
    if (p->p4) return p4_reduce(p, f, n, stream);
    if (p->a4) {
        if (!work) return fail(VP_EINVAL, "vp_reduce_moment: a two-level plan needs the workspace");
        return a4_reduce(p, f, n, work, stream);
    }
    VP_HIP(timed(p, kTMoment, stream, [&] { return launch_moment_rows(p->dtype, f, p->nx, p->nv, p->dv, n, stream); }));
    return VP_OK;
}

vp_status vp_poisson_periodic(const vp_plan* p, const double* n, double* phi, double* E, void* work,
                              hipStream_t stream)
{
    (void)work;
    if (vp_status s = check_plan(p)) return s;
    if (!n) return fail(VP_EINVAL, "vp_poisson_periodic: NULL n");
    if (p->p4) return p4_poisson(p, n, phi, E, stream);
    if (p->a4) return a4_poisson(p, n, phi, E, stream);
    VP_HIP(timed(p, kTField, stream, [&] {
        return launch_poisson1d(nullptr, 0, n, p->dv, p->nx, p->dx, p->pb.qm, p->d_green, p->gk, nullptr, phi, E,
                                nullptr, stream);
    }));
    return VP_OK;
}

vp_status vp_inject_field(const vp_plan* p, const double* E, double* a, hipStream_t stream)
{
    if (vp_status s = check_plan(p)) return s;
    if (!E || !a) return fail(VP_EINVAL, "vp_inject_field: NULL pointer");
    if (p->amr) return amr_inject(p, E, a, stream);
    if (p->hier) return hier_inject(p, E, a, stream);
    if (p->a4) return a4_inject(p, E, a, stream);
    if (p->p4) {
        VP_HIP(timed(p, kTOther, stream, [&] { return launch_scale(E, p->pb.qm, a, 2 * p->nx, stream); }));
        return VP_OK;
    }
    VP_HIP(timed(p, kTOther, stream, [&] { return launch_scale(E, p->pb.qm, a, p->nx, stream); }));
    return VP_OK;
}

vp_status vp_rk4_step(const vp_plan* p, void* f, double* a, double dt, void* work, hipStream_t stream)
{
    if (vp_status s = check_plan(p)) return s;
    if (!f || !a || !work) return fail(VP_EINVAL, "vp_rk4_step: NULL pointer");
    if (!std::isfinite(dt)) return fail(VP_EINVAL, "vp_rk4_step: dt is not finite");
    if (p->amr) return amr_rk4(p, f, a, dt, work, stream);
    if (p->hier) return hier_rk4(p, f, a, dt, work, stream);
    if (p->p4) return p4_rk4(p, f, a, dt, work, stream);
    if (p->a4) return a4_rk4(p, f, a, dt, work, stream);
    return rk4_1d(p, f, a, dt, work, nullptr, nullptr, stream);
}

vp_status vp_rk4_step_noalloc(const vp_plan* p, void* f, double* a, double dt, hipStream_t stream)
{
    if (vp_status s = check_plan(p)) return s;
    if (!f || !a) return fail(VP_EINVAL, "vp_rk4_step_noalloc: NULL pointer");
    if (!std::isfinite(dt)) return fail(VP_EINVAL, "vp_rk4_step_noalloc: dt is not finite");
    if (p->amr || p->hier || p->p4 || p->a4) return fail(VP_ENOTSUP, "vp_rk4_step_noalloc: single-level 1D+1V plans only");
    if (p->ws_step > kScratchBytes)
        return fail(VP_ESHAPE, "vp_rk4_step_noalloc: the step needs " + std::to_string(p->ws_step) +
                                   " bytes of scratch, more than the " + std::to_string(kScratchBytes) +
                                   " bytes of the static scratch array");
    void* work = nullptr;
    if (vp_status s = scratch_address(&work)) return s;
    return rk4_1d(p, f, a, dt, work, nullptr, nullptr, stream);
}

vp_status vp_amr_subcycle_step(const vp_plan* p, void* f, double* a, double dt, void* work, hipStream_t stream)
{
    if (vp_status s = check_plan(p)) return s;
    if (!f || !a || !work) return fail(VP_EINVAL, "vp_amr_subcycle_step: NULL pointer");
    if (!std::isfinite(dt)) return fail(VP_EINVAL, "vp_amr_subcycle_step: dt is not finite");
    if (!p->amr) return fail(VP_EINVAL, "vp_amr_subcycle_step: needs a two-level plan");
    return amr_subcycle(p, f, a, dt, work, stream);
}

vp_status vp_rk4_step_record(const vp_plan* p, void* f, double* a, double dt, void* stages, void* work,
                             hipStream_t stream)
{
    if (vp_status s = check_plan(p)) return s;
    if (!f || !a || !work || !stages) return fail(VP_EINVAL, "vp_rk4_step_record: NULL pointer");
    if (!std::isfinite(dt)) return fail(VP_EINVAL, "vp_rk4_step_record: dt is not finite");
    if (p->amr || p->hier || p->p4 || p->a4) return fail(VP_ENOTSUP, "vp_rk4_step_record: single-level 1D+1V plans only");
    if (p->face_scheme != VP_FACE_CENTERED)
        return fail(VP_ENOTSUP, "vp_rk4_step_record: the adjoint is built for the centred (unlimited) scheme");
    double* st_a = reinterpret_cast<double*>(static_cast<char*>(stages) + 3 * p->state_elems * p->esize);
    if (reinterpret_cast<uintptr_t>(st_a) % 8) return fail(VP_EINVAL, "stage record misaligned");
    return rk4_1d(p, f, a, dt, work, stages, st_a, stream);
}

vp_status vp_field_adjoint(const vp_plan* p, const double* abar, void* fbar, void* work, hipStream_t stream)
{
    if (vp_status s = check_plan(p)) return s;
    if (!abar || !fbar || !work) return fail(VP_EINVAL, "vp_field_adjoint: NULL pointer");
    if (p->dtype != VP_F64) return fail(VP_ENOTSUP, "vp_field_adjoint: FP64 only");
    if (p->amr || p->hier || p->p4 || p->a4) return fail(VP_ENOTSUP, "vp_field_adjoint: single-level 1D+1V plans only");
    double* cfg = reinterpret_cast<double*>(wsp(work, p->ws_cfg));
    double* ab = cfg;
    double* z = cfg + p->nx;
    VP_HIP(hipMemcpyAsync(ab, abar, sizeof(double) * p->nx, hipMemcpyDeviceToDevice, stream));
    VP_HIP(timed(p, kTField, stream, [&] {
        return launch_poisson1d_adjoint(nullptr, 0, p->nx, p->dx, p->dv, p->pb.qm, p->d_green, p->gk, ab, z, stream);
    }));
    VP_HIP(timed(p, kTOther, stream, [&] {
        return launch_row_broadcast(z, p->nx, p->nv, static_cast<double*>(fbar), stream);
    }));
    return VP_OK;
}

vp_status vp_adjoint_step(const vp_plan* p, const void* f_n, const double* a_n, const void* stages,
                          const void* lam_np1, void* lam_n, double dt, void* work, hipStream_t stream)
{
    if (vp_status s = check_plan(p)) return s;
    if (!f_n || !a_n || !lam_np1 || !lam_n || !work) return fail(VP_EINVAL, "vp_adjoint_step: NULL pointer");
    if (p->dtype != VP_F64) return fail(VP_ENOTSUP, "vp_adjoint_step: the adjoint is FP64 only");
    if (p->amr || p->hier || p->p4 || p->a4 || p->nlev != 1 || p->ndim != 1)
        return fail(VP_ENOTSUP, "vp_adjoint_step: single-level 1D+1V only");
    if (p->face_scheme != VP_FACE_CENTERED)
        return fail(VP_ENOTSUP, "vp_adjoint_step: the adjoint is built for the centred (unlimited) scheme");
    if (!std::isfinite(dt)) return fail(VP_EINVAL, "vp_adjoint_step: dt is not finite");
    const size_t N = p->state_elems;
    const int nx = p->nx, nv = p->nv;
    // stage states f(1..4) and accelerations a(1..4)
    const double* st = static_cast<const double*>(stages);
    if (!st) {
        double* tf = reinterpret_cast<double*>(wsp(work, p->ws_tmpf));
        double* ta = reinterpret_cast<double*>(wsp(work, p->ws_tmpa));
        double* rec = reinterpret_cast<double*>(wsp(work, p->ws_stages));
        VP_HIP(hipMemcpyAsync(tf, f_n, N * sizeof(double), hipMemcpyDeviceToDevice, stream));
        VP_HIP(hipMemcpyAsync(ta, a_n, nx * sizeof(double), hipMemcpyDeviceToDevice, stream));
        if (vp_status s = rk4_1d(p, tf, ta, dt, work, rec, rec + 3 * N, stream)) return s;
        st = rec;
    }
    const double* fst[4] = {static_cast<const double*>(f_n), st, st + N, st + 2 * N};
    const double* ast[4] = {st + 3 * N, st + 3 * N + nx, st + 3 * N + 2 * nx, st + 3 * N + 3 * nx};

    double* mu = reinterpret_cast<double*>(wsp(work, p->ws_acc));
    double* gbuf[2] = {reinterpret_cast<double*>(wsp(work, p->ws_fsa)), reinterpret_cast<double*>(wsp(work, p->ws_fsb))};
    double* part = reinterpret_cast<double*>(wsp(work, p->ws_part));
    double* cfg = reinterpret_cast<double*>(wsp(work, p->ws_cfg));
    double* abar = cfg;
    double* zbuf[2] = {cfg + nx, cfg + 2 * nx};

    const bool al = aligned16(f_n) && aligned16(lam_np1) && aligned16(st) && aligned16(mu) && nv % 2 == 0 &&
                    (N * sizeof(double)) % 16 == 0;
    const int w = al ? 2 : 1;
    Adjoint1DArgs A{};
    A.nx = nx;
    A.nv = nv;
    A.nstrip = (nv + 128 * w - 1) / (128 * w);
    // rows per tile: 16, halved (down to 4) while the grid has fewer than
    // 512 tiles, so that small meshes still give every CU work
    A.tx = 16;
    while (A.tx > 4 && (size_t)A.nstrip * ((nx + A.tx - 1) / A.tx) < 512) A.tx /= 2;
    A.dxi = 1.0 / p->dx;
    A.dvi = 1.0 / p->dv;
    A.dv24 = p->dv / 24.0;
    A.v_lo = p->v_lo;
    A.dv = p->dv;
    for (int q = 0; q < 4; ++q) A.vg[q] = p->vg[q];
    A.lam = static_cast<const double*>(lam_np1);
    A.part = part;
    const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    for (int s = 3; s >= 0; --s) {
        const int cur = s & 1, prev = (s + 1) & 1;
        A.fs = fst[s];
        A.a = ast[s];
        A.g_out = gbuf[cur];
        A.c1 = dt * b[s];
        A.c2 = s < 3 ? dt * alpha[s + 1] : 0.0;
        A.g_prev = s < 3 ? gbuf[prev] : nullptr;
        A.z_prev = s < 3 ? zbuf[prev] : nullptr;
        A.mu_in = (s < 2) ? mu : nullptr;     // s = 2 (third from the top) starts from lam
        A.mu_out = mu;
        const bool first = (s == 3);
        VP_HIP(timed(p, kTAdjoint, stream, [&] { return launch_adjoint_stage1d(w, first, A, stream); }));
        VP_HIP(timed(p, kTField, stream, [&] {
            return launch_poisson1d_adjoint(part, A.nstrip, nx, p->dx, p->dv, p->pb.qm, p->d_green, p->gk, abar,
                                            zbuf[cur], stream);
        }));
    }
    VP_HIP(timed(p, kTOther, stream, [&] {
        return launch_adjoint_final(mu, gbuf[0], zbuf[0], nx, nv, static_cast<double*>(lam_n), stream);
    }));
    return VP_OK;
}

}  // extern "C"
