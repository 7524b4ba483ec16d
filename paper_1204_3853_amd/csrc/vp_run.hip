// Adaptive two-level run (section 3, Alg. smsvphu with regridding; the time
// step control of the numerical results of section 4): a run object owns
// the plan of the current hierarchy and the device buffers of its state,
// advances RK4 steps with a time step held below a fraction of the
// stability limit, and regrids every regrid_interval steps (tag level 0,
// cluster the tags, build the plan of the new hierarchy, transfer the
// state, recompute the field).  Host code only: every operation on the
// state goes through the library's entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "vp_internal.hpp"

struct vp_amr_run {
    vp_amr_params prm{};
    vp_plan* plan = nullptr;
    void* f = nullptr;                 // current state, room for f_cap elements
    void* f_spare = nullptr;           // the other state buffer (target of the next transfer)
    size_t f_cap = 0, spare_cap = 0;
    double* a = nullptr;
    double* n = nullptr;
    double* phi = nullptr;
    double* E = nullptr;
    void* work = nullptr;
    size_t work_bytes = 0;
    uint8_t* d_tags = nullptr;
    std::vector<uint8_t> tags;
    std::vector<double> a_host;
    std::vector<vp_box> boxes;
    double t = 0.0, dt = 0.0;
    long long steps = 0;
    int regrids = 0;
    double regrid_seconds = 0.0;
};

namespace vp {
namespace {

template <class T>
void free_dev(T*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

void run_free(vp_amr_run* r)
{
    free_dev(r->f);
    free_dev(r->f_spare);
    free_dev(r->a);
    free_dev(r->n);
    free_dev(r->phi);
    free_dev(r->E);
    free_dev(r->work);
    free_dev(r->d_tags);
    if (r->plan) vp_plan_destroy(r->plan);
    r->plan = nullptr;
}

// workspace of at least `bytes` (grown, never shrunk)
vp_status ensure_work(vp_amr_run* r, size_t bytes)
{
    if (bytes <= r->work_bytes && r->work) return VP_OK;
    free_dev(r->work);
    r->work_bytes = 0;
    VP_HIP(hipMalloc(&r->work, std::max<size_t>(bytes, 256)));
    r->work_bytes = std::max<size_t>(bytes, 256);
    return VP_OK;
}

// a = (q/m) E(f): moment, Poisson, injection
vp_status run_field(vp_amr_run* r, hipStream_t s)
{
    vp_status st = vp_reduce_moment(r->plan, r->f, r->n, r->work, s);
    if (st == VP_OK) st = vp_poisson_periodic(r->plan, r->n, r->phi, r->E, r->work, s);
    if (st == VP_OK) st = vp_inject_field(r->plan, r->E, r->a, s);
    return st;
}

// the largest step with dt (max|v|/dx + max|a|/dv) <= 1 on every level: on
// level 0 over the whole mesh, on level 1 per patch over its own velocity
// faces and configuration columns; reads a back (synchronises the stream)
vp_status stability_limit(vp_amr_run* r, hipStream_t s, double* lim)
{
    const AmrPlan& M = *r->plan->amr;
    const size_t na = (size_t)M.ncx + (size_t)M.nfx;
    r->a_host.resize(na);
    VP_HIP(hipMemcpyAsync(r->a_host.data(), r->a, na * sizeof(double), hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));
    const double* ac = r->a_host.data();
    const double* af = ac + M.ncx;
    const double v_hi = M.v_lo + M.ncv * M.dvc;
    double amax = 0.0;
    for (int i = 0; i < M.ncx; ++i) amax = std::max(amax, std::fabs(ac[i]));
    double rate = std::max(std::fabs(M.v_lo), std::fabs(v_hi)) / M.dxc + amax / M.dvc;
    for (const AmrPatch& P : M.patches) {
        const double v0 = M.v_lo + P.gv0 * M.dvf, v1 = M.v_lo + (P.gv0 + P.nv) * M.dvf;
        double ap = 0.0;
        for (int i = P.gx0; i < P.gx0 + P.nx; ++i) ap = std::max(ap, std::fabs(af[i]));
        rate = std::max(rate, std::max(std::fabs(v0), std::fabs(v1)) / M.dxf + ap / M.dvf);
    }
    *lim = 1.0 / rate;
    return VP_OK;
}

vp_status regrid(vp_amr_run* r, hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    const AmrPlan& M = *r->plan->amr;
    const int ncx = M.ncx, ncv = M.ncv, R = M.R;
    vp_status st = vp_tag_cells(r->plan, r->f, r->prm.tol, r->d_tags, nullptr, s);
    if (st != VP_OK) return st;
    r->tags.resize((size_t)ncx * ncv);
    VP_HIP(hipMemcpyAsync(r->tags.data(), r->d_tags, r->tags.size(), hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));
    // boxes at least one cell apart: at most ceil(ncx/2) ceil(ncv/2) of them
    std::vector<vp_box> bx((size_t)((ncx + 1) / 2) * ((ncv + 1) / 2) + 1);
    int32_t nb = 0;
    st = vp_cluster_tags(r->tags.data(), ncx, ncv, R, r->prm.efficiency, r->prm.min_width, r->prm.buffer, bx.data(),
                         (int32_t)bx.size(), &nb);
    if (st != VP_OK) return st;
    bx.resize((size_t)nb);
    vp_problem pb = r->plan->pb;
    pb.veq[0][0] = r->plan->veq[0][0].data();
    pb.veq[1][0] = r->plan->veq[1][0].data();
    vp_plan* np = nullptr;
    st = vp_plan_create(&pb, bx.data(), nb, &np);
    if (st != VP_OK) return st;
    // the new state goes into the spare buffer (grown when too small); the
    // old one becomes the spare
    const size_t ne = std::max<size_t>(vp_state_elems(np), 1);
    hipError_t e = hipSuccess;
    if (ne > r->spare_cap) {
        free_dev(r->f_spare);
        r->spare_cap = 0;
        e = hipMalloc(&r->f_spare, ne * sizeof(double));
        if (e != hipSuccess) {
            vp_plan_destroy(np);
            return hip_fail(e, "vp_amr_run_advance: state of the new hierarchy");
        }
        r->spare_cap = ne;
    }
    st = ensure_work(r, vp_workspace_bytes(np));
    if (st == VP_OK) st = vp_regrid_transfer(r->plan, r->f, np, r->f_spare, s);
    if (st == VP_OK) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "vp_amr_run_advance: transfer");
    }
    if (st != VP_OK) {
        vp_plan_destroy(np);
        return st;
    }
    vp_plan_destroy(r->plan);
    std::swap(r->f, r->f_spare);
    std::swap(r->f_cap, r->spare_cap);
    r->plan = np;
    r->boxes = bx;
    st = run_field(r, s);
    if (st != VP_OK) return st;
    VP_HIP(hipStreamSynchronize(s));
    ++r->regrids;
    r->regrid_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return VP_OK;
}

}  // namespace
}  // namespace vp

using namespace vp;

extern "C" {

vp_status vp_amr_run_create(const vp_problem* problem, const vp_box* boxes, int32_t nbox, const void* f0,
                            const vp_amr_params* params, vp_amr_run** out, hipStream_t stream)
{
    if (!problem || !params || !out || !f0) return fail(VP_EINVAL, "vp_amr_run_create: NULL pointer");
    *out = nullptr;
    const vp_amr_params& q = *params;
    if (!(q.tol >= 0.0) || !std::isfinite(q.tol) || q.regrid_interval < 1 || !(q.efficiency > 0.0 && q.efficiency <= 1.0) ||
        q.min_width < 1 || q.buffer < 0 || !(q.cfl > 0.0) || !(q.dt_growth >= 1.0) || !(q.dt_initial > 0.0))
        return fail(VP_EINVAL, "vp_amr_run_create: bad parameters");
    if (problem->n_levels != 2) return fail(VP_EINVAL, "vp_amr_run_create: the problem must have two levels");
    vp_amr_run* r = new (std::nothrow) vp_amr_run();
    if (!r) return fail(VP_ENOMEM, "out of host memory");
    r->prm = q;
    vp_status st = vp_plan_create(problem, boxes, nbox, &r->plan);
    if (st != VP_OK) {
        delete r;
        return st;
    }
    const AmrPlan& M = *r->plan->amr;
    auto dev = [&](auto** p, size_t bytes) -> vp_status {
        VP_HIP(hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(bytes, 256)));
        return VP_OK;
    };
    const size_t nf = (size_t)M.nfx;
    st = dev(&r->f, vp_state_elems(r->plan) * sizeof(double));
    r->f_cap = std::max<size_t>(vp_state_elems(r->plan), 1);
    if (st == VP_OK) st = dev(&r->a, vp_field_elems(r->plan) * sizeof(double));
    if (st == VP_OK) st = dev(&r->n, nf * sizeof(double));
    if (st == VP_OK) st = dev(&r->phi, nf * sizeof(double));
    if (st == VP_OK) st = dev(&r->E, nf * sizeof(double));
    if (st == VP_OK) st = dev(&r->d_tags, (size_t)M.ncx * M.ncv);
    if (st == VP_OK) st = ensure_work(r, vp_workspace_bytes(r->plan));
    if (st == VP_OK) {
        const hipError_t e = hipMemcpyAsync(r->f, f0, vp_state_elems(r->plan) * sizeof(double),
                                            hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) st = hip_fail(e, "vp_amr_run_create: initial state");
    }
    if (st == VP_OK) st = run_field(r, stream);
    if (st != VP_OK) {
        run_free(r);
        delete r;
        return st;
    }
    r->boxes.assign(boxes, boxes + nbox);
    *out = r;
    return VP_OK;
}

vp_status vp_amr_run_advance(vp_amr_run* r, int32_t steps, hipStream_t stream)
{
    if (!r) return fail(VP_EINVAL, "vp_amr_run_advance: run is NULL");
    if (steps < 0) return fail(VP_EINVAL, "vp_amr_run_advance: negative step count");
    for (int32_t k = 0; k < steps; ++k) {
        double lim = 0.0;
        vp_status st = stability_limit(r, stream, &lim);
        if (st != VP_OK) return st;
        const double cap = r->steps == 0 ? r->prm.dt_initial : r->prm.dt_growth * r->dt;
        const double dt = std::min(cap, r->prm.cfl * lim);
        st = vp_rk4_step(r->plan, r->f, r->a, dt, r->work, stream);
        if (st != VP_OK) return st;
        r->dt = dt;
        r->t += dt;
        ++r->steps;
        if (r->steps % r->prm.regrid_interval == 0) {
            st = regrid(r, stream);
            if (st != VP_OK) return st;
        }
    }
    VP_HIP(hipStreamSynchronize(stream));
    return VP_OK;
}

vp_status vp_amr_run_info(const vp_amr_run* r, vp_amr_info* info)
{
    if (!r || !info) return fail(VP_EINVAL, "vp_amr_run_info: NULL pointer");
    std::memset(info, 0, sizeof(*info));
    info->t = r->t;
    info->dt = r->dt;
    info->steps = r->steps;
    info->regrids = r->regrids;
    info->npatch = (int32_t)r->boxes.size();
    info->state_elems = (int64_t)vp_state_elems(r->plan);
    info->regrid_seconds = r->regrid_seconds;
    return VP_OK;
}

const vp_plan* vp_amr_run_plan(const vp_amr_run* r) { return r ? r->plan : nullptr; }

vp_status vp_amr_run_boxes(const vp_amr_run* r, vp_box* boxes, int32_t max_boxes, int32_t* nbox)
{
    if (!r || !nbox || (max_boxes > 0 && !boxes)) return fail(VP_EINVAL, "vp_amr_run_boxes: NULL pointer");
    *nbox = (int32_t)r->boxes.size();
    if (*nbox > max_boxes) return fail(VP_EINVAL, "vp_amr_run_boxes: more boxes than max_boxes");
    std::copy(r->boxes.begin(), r->boxes.end(), boxes);
    return VP_OK;
}

vp_status vp_amr_run_read_state(const vp_amr_run* r, void* dst, size_t elems, hipStream_t stream)
{
    if (!r || !dst) return fail(VP_EINVAL, "vp_amr_run_read_state: NULL pointer");
    if (elems != vp_state_elems(r->plan)) return fail(VP_ESHAPE, "vp_amr_run_read_state: wrong element count");
    VP_HIP(hipMemcpyAsync(dst, r->f, elems * sizeof(double), hipMemcpyDeviceToDevice, stream));
    return VP_OK;
}

vp_status vp_amr_run_destroy(vp_amr_run* r)
{
    if (!r) return VP_OK;
    (void)hipDeviceSynchronize();
    run_free(r);
    delete r;
    return VP_OK;
}

}  // extern "C"
