// Adaptive two-level run (section 3, Alg. smsvphu with regridding; the time
// step control of the numerical results of section 4): a run object owns
// the plans of the current hierarchies and the device buffers of their
// states, advances RK4 steps with a time step held below a fraction of the
// stability limit, and regrids every regrid_interval steps (tag level 0,
// cluster the tags, build the plan of the new hierarchy, transfer the
// state, recompute the field).  A run carries one species (its plan's own
// field: rho = 1 - n) or several, each on its own hierarchy that it regrids
// from its own tags, coupled through the field of a species group (section
// 1: one hierarchy per species).  Host code only: every operation on the
// states goes through the library's entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "vp_internal.hpp"

namespace vp {
namespace {

struct RunSpecies {
    vp_plan* plan = nullptr;
    void* f = nullptr;                 // current state, room for f_cap elements
    void* f_spare = nullptr;           // the other state buffer (target of the next transfer)
    size_t f_cap = 0, spare_cap = 0;
    double* a = nullptr;               // [coarse][fine] acceleration
    void* work = nullptr;
    size_t work_bytes = 0;
    uint8_t* d_tags = nullptr;
    std::vector<uint8_t> tags;
    std::vector<double> a_host;
    std::vector<vp_box> boxes;
};

}  // namespace
}  // namespace vp

struct vp_amr_run {
    vp_amr_params prm{};
    int ns = 0;
    bool group_field = false;          // several species: the field of the species group
    vp::RunSpecies sp[vp::kMaxSpecies];
    double charge[vp::kMaxSpecies] = {};
    double background = 0.0;
    vp_species_group* group = nullptr;
    void* gwork = nullptr;
    size_t gwork_bytes = 0;
    double* n = nullptr;               // single species: moment, potential, field
    double* phi = nullptr;
    double* E = nullptr;
    double t = 0.0, dt = 0.0;
    double* d_clock = nullptr;         // [dt, t] on the device (one species on a multi-level hierarchy)
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
    if (r->group) vp_species_group_destroy(r->group);
    r->group = nullptr;
    for (int s = 0; s < r->ns; ++s) {
        RunSpecies& S = r->sp[s];
        free_dev(S.f);
        free_dev(S.f_spare);
        free_dev(S.a);
        free_dev(S.work);
        free_dev(S.d_tags);
        if (S.plan) vp_plan_destroy(S.plan);
        S.plan = nullptr;
    }
    free_dev(r->gwork);
    free_dev(r->d_clock);
    free_dev(r->n);
    free_dev(r->phi);
    free_dev(r->E);
}

// device buffer of at least `bytes` (grown, never shrunk)
vp_status ensure_buf(void** buf, size_t* cap, size_t bytes)
{
    bytes = std::max<size_t>(bytes, 256);
    if (bytes <= *cap && *buf) return VP_OK;
    free_dev(*buf);
    *cap = 0;
    VP_HIP(hipMalloc(buf, bytes));
    *cap = bytes;
    return VP_OK;
}

// the species group over the current plans (rebuilt after every regrid)
vp_status rebuild_group(vp_amr_run* r)
{
    if (!r->group_field) return VP_OK;
    if (r->group) vp_species_group_destroy(r->group);
    r->group = nullptr;
    const vp_plan* plans[kMaxSpecies];
    for (int s = 0; s < r->ns; ++s) plans[s] = r->sp[s].plan;
    if (vp_status st = vp_species_group_create(plans, r->charge, r->ns, r->background, &r->group)) return st;
    return ensure_buf(&r->gwork, &r->gwork_bytes, vp_species_workspace_bytes(r->group));
}

// every a_s of the current states
vp_status run_field(vp_amr_run* r, hipStream_t s)
{
    if (r->group_field) {
        void* f[kMaxSpecies];
        double* a[kMaxSpecies];
        void* w[kMaxSpecies];
        for (int q = 0; q < r->ns; ++q) {
            f[q] = r->sp[q].f;
            a[q] = r->sp[q].a;
            w[q] = r->sp[q].work;
        }
        return vp_species_field(r->group, f, a, w, r->gwork, s);
    }
    RunSpecies& S = r->sp[0];
    vp_status st = vp_reduce_moment(S.plan, S.f, r->n, S.work, s);
    if (st == VP_OK) st = vp_poisson_periodic(S.plan, r->n, r->phi, r->E, S.work, s);
    if (st == VP_OK) st = vp_inject_field(S.plan, r->E, S.a, s);
    return st;
}

// Largest Courant number dt (|v|/dx + |a|/dv) of linear stability for RK4
// on the centred fourth-order flux divergence (section 4 takes a fraction of
// this limit): the divergence symbol (8 sin t - sin 2t)/6 peaks at
// cos t = 1 - sqrt(6)/2, and RK4 is stable on the imaginary axis up to
// 2 sqrt(2); about 2.0612.
double linear_stability_courant()
{
    const double c = 1.0 - std::sqrt(6.0) / 2.0;
    const double s_max = std::sqrt(1.0 - c * c) * (4.0 - c) / 3.0;
    return 2.0 * std::sqrt(2.0) / s_max;
}

// the largest linearly stable step, dt (max|v|/dx + max|a|/dv) <=
// linear_stability_courant() on every level of every species: on level 0
// over the whole mesh, on level 1 per patch over its own velocity faces and
// configuration columns; reads a back (synchronises the stream)
vp_status stability_limit(vp_amr_run* r, hipStream_t s, double* lim)
{
    for (int q = 0; q < r->ns; ++q) {
        RunSpecies& S = r->sp[q];
        S.a_host.resize(vp_field_elems(S.plan));
        VP_HIP(hipMemcpyAsync(S.a_host.data(), S.a, S.a_host.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    VP_HIP(hipStreamSynchronize(s));
    double rate = 0.0;
    for (int q = 0; q < r->ns; ++q) {
        const RunSpecies& S = r->sp[q];
        if (S.plan->hier) {
            // every patch of every level (level 0 is patch 0) over its own
            // velocity faces and configuration columns
            const HierPlan& H = *S.plan->hier;
            const double v_lo = S.plan->pb.v_lo[0];
            for (const HPatch& P : H.patches) {
                const HLevel& v = H.lv[P.lev];
                const double* al = S.a_host.data() + v.a_off;
                const double v0 = v_lo + P.gv0 * v.dv, v1 = v_lo + (P.gv0 + P.nv) * v.dv;
                double ap = 0.0;
                for (int i = P.gx0; i < P.gx0 + P.nx; ++i) ap = std::max(ap, std::fabs(al[i]));
                rate = std::max(rate, std::max(std::fabs(v0), std::fabs(v1)) * v.dxi + ap * v.dvi);
            }
            continue;
        }
        const AmrPlan& M = *S.plan->amr;
        const double* ac = S.a_host.data();
        const double* af = ac + M.ncx;
        const double v_hi = M.v_lo + M.ncv * M.dvc;
        double amax = 0.0;
        for (int i = 0; i < M.ncx; ++i) amax = std::max(amax, std::fabs(ac[i]));
        rate = std::max(rate, std::max(std::fabs(M.v_lo), std::fabs(v_hi)) / M.dxc + amax / M.dvc);
        for (const AmrPatch& P : M.patches) {
            const double v0 = M.v_lo + P.gv0 * M.dvf, v1 = M.v_lo + (P.gv0 + P.nv) * M.dvf;
            double ap = 0.0;
            for (int i = P.gx0; i < P.gx0 + P.nx; ++i) ap = std::max(ap, std::fabs(af[i]));
            rate = std::max(rate, std::max(std::fabs(v0), std::fabs(v1)) / M.dxf + ap / M.dvf);
        }
    }
    *lim = linear_stability_courant() / rate;
    return VP_OK;
}

// the boxes of a and b are the same sequence (level and the x, v corners;
// the adaptive run is 1D+1V)
bool same_boxes(const vp_box* a, size_t na, const vp_box* b, size_t nb)
{
    if (na != nb) return false;
    for (size_t q = 0; q < na; ++q)
        if (a[q].level != b[q].level || a[q].lo[0] != b[q].lo[0] || a[q].lo[1] != b[q].lo[1] ||
            a[q].hi[0] != b[q].hi[0] || a[q].hi[1] != b[q].hi[1])
            return false;
    return true;
}

// regrid of a multi-level hierarchy, from the coarsest level up: level l of
// the new hierarchy is tagged (level 0: the old state; finer: a plan of the
// new levels 0 .. l with its transferred state), its tags clustered into
// level-(l+1) boxes nested in it; the final plan's state transferred from the
// old hierarchy.  While the new levels 0 .. l are the old ones, box for box,
// the transfer would copy them unchanged, so level l is tagged on the old
// plan and state; a new hierarchy equal to the old one keeps the old plan
// and state (*changed = false).
vp_status regrid_hier(vp_amr_run* r, RunSpecies& S, hipStream_t s, bool* changed)
{
    const vp_plan* old = S.plan;
    const int L = old->hier->L;
    vp_problem pb = old->pb;
    for (int l = 0; l < L; ++l) pb.veq[l][0] = old->veq[l][0].data();
    std::vector<vp_box> nb;
    vp_plan* P = nullptr;          // the new levels 0 .. l
    void* F = nullptr;             // its state
    size_t fcap = 0;
    bool same = true;              // the new levels 0 .. l are the old ones
    vp_status st = VP_OK;
    for (int l = 0; l + 1 < L && st == VP_OK; ++l) {
        const vp_plan* tp = same ? old : P;
        const void* tf = same ? S.f : F;
        const HLevel& v = tp->hier->lv[l];
        st = ensure_buf(&S.work, &S.work_bytes, vp_workspace_bytes(tp));
        if (st == VP_OK) st = hier_tag_level(tp, static_cast<const double*>(tf), l, r->prm.tol, S.d_tags, nullptr,
                                             S.work, s);
        if (st != VP_OK) break;
        S.tags.resize((size_t)v.nx * v.nv);
        hipError_t e = hipMemcpyAsync(S.tags.data(), S.d_tags, S.tags.size(), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { st = hip_fail(e, "vp_amr_run_advance: tags"); break; }
        std::vector<vp_box> add;
        const int mx = r->prm.max_size[l + 1][0], mv = r->prm.max_size[l + 1][1];
        st = hier_cluster(tp, l, S.tags.data(), pb.ratio[l][0], pb.ratio[l][1], r->prm.efficiency, r->prm.min_width,
                          r->prm.buffer, mx, mv, add);
        if (st != VP_OK || add.empty()) break;
        nb.insert(nb.end(), add.begin(), add.end());
        if (same) {
            std::vector<vp_box> ol;               // the old level-(l+1) boxes
            for (const vp_box& b : S.boxes)
                if (b.level == l + 1) ol.push_back(b);
            same = same_boxes(add.data(), add.size(), ol.data(), ol.size());
        }
        if (l + 2 < L && !same) {             // the new levels 0 .. l+1, to tag level l+1 next
            vp_problem pbi = pb;
            pbi.n_levels = l + 2;
            vp_plan* Pn = nullptr;
            st = hier_plan_create(&pbi, nb.data(), (int)nb.size(), &Pn, true);
            if (st == VP_OK) st = ensure_buf(&F, &fcap, std::max<size_t>(vp_state_elems(Pn), 1) * sizeof(double));
            if (st == VP_OK) st = hier_transfer(old, static_cast<const double*>(S.f), Pn, static_cast<double*>(F), s);
            if (P) vp_plan_destroy(P);
            P = Pn;
        }
    }
    if (P) vp_plan_destroy(P);
    free_dev(F);
    if (st != VP_OK) return st;
    *changed = !same_boxes(nb.data(), nb.size(), S.boxes.data(), S.boxes.size());
    if (!*changed) return VP_OK;
    vp_plan* np = nullptr;
    st = hier_plan_create(&pb, nb.data(), (int)nb.size(), &np);
    if (st != VP_OK) return st;
    size_t spare_bytes = S.spare_cap * sizeof(double);
    st = ensure_buf(&S.f_spare, &spare_bytes, std::max<size_t>(vp_state_elems(np), 1) * sizeof(double));
    S.spare_cap = spare_bytes / sizeof(double);
    if (st == VP_OK) st = ensure_buf(&S.work, &S.work_bytes, vp_workspace_bytes(np));
    if (st == VP_OK) st = hier_transfer(old, static_cast<const double*>(S.f), np, static_cast<double*>(S.f_spare), s);
    if (st != VP_OK) {
        vp_plan_destroy(np);
        return st;
    }
    vp_plan_destroy(S.plan);
    std::swap(S.f, S.f_spare);
    std::swap(S.f_cap, S.spare_cap);
    S.plan = np;
    S.boxes = nb;
    return VP_OK;
}

// regrid of one species' hierarchy from its own tags; *changed = false when
// the new boxes are the old ones (the plan and state are kept)
vp_status regrid_species(vp_amr_run* r, RunSpecies& S, hipStream_t s, bool* changed)
{
    if (S.plan->hier) return regrid_hier(r, S, s, changed);
    const AmrPlan& M = *S.plan->amr;
    const int ncx = M.ncx, ncv = M.ncv, R = M.R;
    vp_status st = vp_tag_cells(S.plan, S.f, r->prm.tol, S.d_tags, nullptr, s);
    if (st != VP_OK) return st;
    S.tags.resize((size_t)ncx * ncv);
    VP_HIP(hipMemcpyAsync(S.tags.data(), S.d_tags, S.tags.size(), hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));
    // boxes at least one cell apart: at most ceil(ncx/2) ceil(ncv/2) of them
    std::vector<vp_box> bx((size_t)((ncx + 1) / 2) * ((ncv + 1) / 2) + 1);
    int32_t nb = 0;
    st = vp_cluster_tags(S.tags.data(), ncx, ncv, R, r->prm.efficiency, r->prm.min_width, r->prm.buffer, bx.data(),
                         (int32_t)bx.size(), &nb);
    if (st != VP_OK) return st;
    bx.resize((size_t)nb);
    *changed = !same_boxes(bx.data(), bx.size(), S.boxes.data(), S.boxes.size());
    if (!*changed) return VP_OK;
    vp_problem pb = S.plan->pb;
    pb.veq[0][0] = S.plan->veq[0][0].data();
    pb.veq[1][0] = S.plan->veq[1][0].data();
    vp_plan* np = nullptr;
    st = vp_plan_create(&pb, bx.data(), nb, &np);
    if (st != VP_OK) return st;
    // the new state goes into the spare buffer (grown when too small); the
    // old one becomes the spare
    size_t spare_bytes = S.spare_cap * sizeof(double);
    st = ensure_buf(&S.f_spare, &spare_bytes, std::max<size_t>(vp_state_elems(np), 1) * sizeof(double));
    S.spare_cap = spare_bytes / sizeof(double);
    if (st == VP_OK) st = ensure_buf(&S.work, &S.work_bytes, vp_workspace_bytes(np));
    if (st == VP_OK) st = vp_regrid_transfer(S.plan, S.f, np, S.f_spare, s);
    if (st == VP_OK) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "vp_amr_run_advance: transfer");
    }
    if (st != VP_OK) {
        vp_plan_destroy(np);
        return st;
    }
    vp_plan_destroy(S.plan);
    std::swap(S.f, S.f_spare);
    std::swap(S.f_cap, S.spare_cap);
    S.plan = np;
    S.boxes = bx;
    return VP_OK;
}

vp_status regrid(vp_amr_run* r, hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    bool any = false;
    for (int q = 0; q < r->ns; ++q) {
        bool changed = true;
        if (vp_status st = regrid_species(r, r->sp[q], s, &changed)) return st;
        any = any || changed;
    }
    if (any)
        if (vp_status st = rebuild_group(r)) return st;
    if (vp_status st = run_field(r, s)) return st;
    VP_HIP(hipStreamSynchronize(s));
    ++r->regrids;
    r->regrid_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return VP_OK;
}

vp_status check_params(const vp_amr_params& q)
{
    if (!(q.tol >= 0.0) || !std::isfinite(q.tol) || q.regrid_interval < 1 || !(q.efficiency > 0.0 && q.efficiency <= 1.0) ||
        q.min_width < 1 || q.buffer < 0 || !(q.cfl > 0.0) || !(q.dt_growth >= 1.0) || !(q.dt_initial > 0.0))
        return fail(VP_EINVAL, "vp_amr_run_create: bad parameters");
    for (int l = 0; l < VP_MAX_LEVELS; ++l)
        if (q.max_size[l][0] < 0 || q.max_size[l][1] < 0) return fail(VP_EINVAL, "vp_amr_run_create: bad patch size limit");
    return VP_OK;
}

// plan, buffers and initial state of species q
vp_status add_species(vp_amr_run* r, int q, const vp_problem* pb, const vp_box* boxes, int32_t nbox, const void* f0,
                      hipStream_t stream)
{
    RunSpecies& S = r->sp[q];
    if (vp_status st = vp_plan_create(pb, boxes, nbox, &S.plan)) return st;
    if (!S.plan->amr && !S.plan->hier) return fail(VP_EINVAL, "vp_amr_run_create: the problem must have two or more levels");
    size_t tag_cells = 0;
    if (S.plan->amr) {
        tag_cells = (size_t)S.plan->amr->ncx * S.plan->amr->ncv;
    } else {
        for (int l = 0; l < S.plan->hier->L; ++l)
            tag_cells = std::max(tag_cells, (size_t)S.plan->hier->lv[l].nx * S.plan->hier->lv[l].nv);
    }
    const size_t ne = std::max<size_t>(vp_state_elems(S.plan), 1);
    size_t fb = 0, ab = 0, tb = 0;
    if (vp_status st = ensure_buf(&S.f, &fb, ne * sizeof(double))) return st;
    S.f_cap = ne;
    void* a = nullptr;
    if (vp_status st = ensure_buf(&a, &ab, vp_field_elems(S.plan) * sizeof(double))) return st;
    S.a = static_cast<double*>(a);
    void* tg = nullptr;
    if (vp_status st = ensure_buf(&tg, &tb, tag_cells)) return st;
    S.d_tags = static_cast<uint8_t*>(tg);
    if (vp_status st = ensure_buf(&S.work, &S.work_bytes, vp_workspace_bytes(S.plan))) return st;
    VP_HIP(hipMemcpyAsync(S.f, f0, vp_state_elems(S.plan) * sizeof(double), hipMemcpyDeviceToDevice, stream));
    S.boxes.assign(boxes, boxes + nbox);
    return VP_OK;
}

// One species on a multi-level hierarchy: the time step is computed on the
// device from the field the previous step (or the regrid) left, and the
// step's kernels read it there, so the steps between two regrids are
// enqueued without waiting for the GPU; dt and t come back to the host at
// the end of the call (or when a regrid synchronises anyway).
vp_status advance_device_clock(vp_amr_run* r, int32_t steps, hipStream_t stream)
{
    RunSpecies& S = r->sp[0];
    if (!r->d_clock) {
        VP_HIP(hipMalloc(&r->d_clock, 2 * sizeof(double)));
        const double c[2] = {r->dt, r->t};
        VP_HIP(hipMemcpy(r->d_clock, c, sizeof(c), hipMemcpyHostToDevice));
    }
    const double courant = linear_stability_courant();
    for (int32_t k = 0; k < steps; ++k) {
        const HierPlan& H = *S.plan->hier;
        VP_HIP(launch_hier_dt(S.a, H.d_patches, (int)H.patches.size(), H.lv, H.L, S.plan->pb.v_lo[0], courant,
                              r->prm.cfl, r->prm.dt_growth, r->prm.dt_initial, r->steps == 0, r->d_clock, stream));
        if (vp_status st = hier_rk4(S.plan, S.f, S.a, 0.0, S.work, stream, r->d_clock)) return st;
        ++r->steps;
        if (r->steps % r->prm.regrid_interval == 0)
            if (vp_status st = regrid(r, stream)) return st;
    }
    double c[2];
    VP_HIP(hipMemcpyAsync(c, r->d_clock, sizeof(c), hipMemcpyDeviceToHost, stream));
    VP_HIP(hipStreamSynchronize(stream));
    r->dt = c[0];
    r->t = c[1];
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
    if (vp_status st = check_params(*params)) return st;
    if (problem->n_levels < 2) return fail(VP_EINVAL, "vp_amr_run_create: the problem must have two or more levels");
    vp_amr_run* r = new (std::nothrow) vp_amr_run();
    if (!r) return fail(VP_ENOMEM, "out of host memory");
    r->prm = *params;
    r->ns = 1;
    vp_status st = add_species(r, 0, problem, boxes, nbox, f0, stream);
    if (st == VP_OK) {
        const size_t nf = vp_config_elems(r->sp[0].plan);
        size_t c1 = 0, c2 = 0, c3 = 0;
        st = ensure_buf(reinterpret_cast<void**>(&r->n), &c1, nf * sizeof(double));
        if (st == VP_OK) st = ensure_buf(reinterpret_cast<void**>(&r->phi), &c2, nf * sizeof(double));
        if (st == VP_OK) st = ensure_buf(reinterpret_cast<void**>(&r->E), &c3, nf * sizeof(double));
    }
    if (st == VP_OK) st = run_field(r, stream);
    if (st != VP_OK) {
        run_free(r);
        delete r;
        return st;
    }
    *out = r;
    return VP_OK;
}

vp_status vp_amr_run_create_species(int32_t nspecies, const vp_problem* const* problems, const vp_box* const* boxes,
                                    const int32_t* nbox, const void* const* f0, const double* charge,
                                    double background, const vp_amr_params* params, vp_amr_run** out,
                                    hipStream_t stream)
{
    if (!problems || !boxes || !nbox || !f0 || !charge || !params || !out)
        return fail(VP_EINVAL, "vp_amr_run_create_species: NULL pointer");
    *out = nullptr;
    if (vp_status st = check_params(*params)) return st;
    if (nspecies < 1 || nspecies > kMaxSpecies)
        return fail(VP_EINVAL, "vp_amr_run_create_species: 1 to " + std::to_string(kMaxSpecies) + " species");
    for (int q = 0; q < nspecies; ++q) {
        if (!problems[q] || !f0[q] || (nbox[q] > 0 && !boxes[q]))
            return fail(VP_EINVAL, "vp_amr_run_create_species: NULL pointer");
        if (problems[q]->n_levels != 2)
            return fail(VP_EINVAL, "vp_amr_run_create_species: every problem must have two levels");
    }
    vp_amr_run* r = new (std::nothrow) vp_amr_run();
    if (!r) return fail(VP_ENOMEM, "out of host memory");
    r->prm = *params;
    r->ns = nspecies;
    r->group_field = true;
    r->background = background;
    vp_status st = VP_OK;
    for (int q = 0; q < nspecies && st == VP_OK; ++q) {
        r->charge[q] = charge[q];
        st = add_species(r, q, problems[q], boxes[q], nbox[q], f0[q], stream);
    }
    if (st == VP_OK) st = rebuild_group(r);
    if (st == VP_OK) st = run_field(r, stream);
    if (st != VP_OK) {
        run_free(r);
        delete r;
        return st;
    }
    *out = r;
    return VP_OK;
}

vp_status vp_amr_run_advance(vp_amr_run* r, int32_t steps, hipStream_t stream)
{
    if (!r) return fail(VP_EINVAL, "vp_amr_run_advance: run is NULL");
    if (steps < 0) return fail(VP_EINVAL, "vp_amr_run_advance: negative step count");
    if (!r->group_field && r->sp[0].plan->hier) return advance_device_clock(r, steps, stream);
    for (int32_t k = 0; k < steps; ++k) {
        double lim = 0.0;
        vp_status st = stability_limit(r, stream, &lim);
        if (st != VP_OK) return st;
        const double cap = r->steps == 0 ? r->prm.dt_initial : r->prm.dt_growth * r->dt;
        const double dt = std::min(cap, r->prm.cfl * lim);
        if (r->group_field) {
            void* f[kMaxSpecies];
            double* a[kMaxSpecies];
            void* w[kMaxSpecies];
            for (int q = 0; q < r->ns; ++q) {
                f[q] = r->sp[q].f;
                a[q] = r->sp[q].a;
                w[q] = r->sp[q].work;
            }
            st = vp_species_rk4_step(r->group, f, a, dt, w, r->gwork, stream);
        } else {
            st = vp_rk4_step(r->sp[0].plan, r->sp[0].f, r->sp[0].a, dt, r->sp[0].work, stream);
        }
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
    for (int q = 0; q < r->ns; ++q) {
        info->npatch += (int32_t)r->sp[q].boxes.size();
        info->state_elems += (int64_t)vp_state_elems(r->sp[q].plan);
    }
    info->regrid_seconds = r->regrid_seconds;
    return VP_OK;
}

int32_t vp_amr_run_species_count(const vp_amr_run* r) { return r ? r->ns : 0; }

const vp_plan* vp_amr_run_plan_of(const vp_amr_run* r, int32_t species)
{
    return (r && species >= 0 && species < r->ns) ? r->sp[species].plan : nullptr;
}

const vp_plan* vp_amr_run_plan(const vp_amr_run* r) { return vp_amr_run_plan_of(r, 0); }

vp_status vp_amr_run_boxes_of(const vp_amr_run* r, int32_t species, vp_box* boxes, int32_t max_boxes, int32_t* nbox)
{
    if (!r || !nbox || (max_boxes > 0 && !boxes)) return fail(VP_EINVAL, "vp_amr_run_boxes: NULL pointer");
    if (species < 0 || species >= r->ns) return fail(VP_EINVAL, "vp_amr_run_boxes: no such species");
    const std::vector<vp_box>& b = r->sp[species].boxes;
    *nbox = (int32_t)b.size();
    if (*nbox > max_boxes) return fail(VP_EINVAL, "vp_amr_run_boxes: more boxes than max_boxes");
    std::copy(b.begin(), b.end(), boxes);
    return VP_OK;
}

vp_status vp_amr_run_boxes(const vp_amr_run* r, vp_box* boxes, int32_t max_boxes, int32_t* nbox)
{
    return vp_amr_run_boxes_of(r, 0, boxes, max_boxes, nbox);
}

vp_status vp_amr_run_read_state_of(const vp_amr_run* r, int32_t species, void* dst, size_t elems,
                                   hipStream_t stream)
{
    if (!r || !dst) return fail(VP_EINVAL, "vp_amr_run_read_state: NULL pointer");
    if (species < 0 || species >= r->ns) return fail(VP_EINVAL, "vp_amr_run_read_state: no such species");
    const RunSpecies& S = r->sp[species];
    if (elems != vp_state_elems(S.plan)) return fail(VP_ESHAPE, "vp_amr_run_read_state: wrong element count");
    VP_HIP(hipMemcpyAsync(dst, S.f, elems * sizeof(double), hipMemcpyDeviceToDevice, stream));
    return VP_OK;
}

vp_status vp_amr_run_read_state(const vp_amr_run* r, void* dst, size_t elems, hipStream_t stream)
{
    return vp_amr_run_read_state_of(r, 0, dst, elems, stream);
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
