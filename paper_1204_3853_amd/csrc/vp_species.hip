// Several kinetic species on one configuration mesh (section 1: every
// species has its own velocity range and its own phase-space hierarchy;
// collisionless species interact only through the field).  A group ties
// 1D+1V plans together, single-level or two-level: each species is advanced
// by its own plan's stage kernels, and after every stage one field solve on
// the shared finest configuration mesh, from the charge density of all
// species, gives every species its acceleration (q/m)_s E (injected onto
// both levels of a two-level species).
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "vp_internal.hpp"

struct vp_species_group {
    int ns = 0;
    const vp_plan* plans[vp::kMaxSpecies] = {};
    double charge[vp::kMaxSpecies] = {};
    double background = 0.0;
    int nx = 0;
    // group workspace layout (byte offsets): per-species moments, n_eff, E,
    // field-solve scratch
    size_t ws_n = 0, ws_neff = 0, ws_E = 0, ws_cfg = 0, ws_total = 0;
};

namespace vp {
namespace {

size_t align256s(size_t x) { return (x + 255) & ~size_t(255); }

double* gptr(void* gwork, size_t off) { return reinterpret_cast<double*>(static_cast<char*>(gwork) + off); }

// the field of the species' moments m, then every a_s.  Meshes of at least
// kFieldSplitMin cells: the split solve takes the charge density straight
// from the moments and writes a_s = (q/m)_s E of every single-level species
// (and E for the two-level ones, which inject it onto their levels).
// Smaller meshes: n_eff = 1 - rho, the one-block solve for E, then a_s.
vp_status species_field_solve(const vp_species_group* g, const SpeciesMoments& m, void* gwork, double* const* a,
                              hipStream_t stream)
{
    const vp_plan* p = g->plans[0];
    double* n_eff = gptr(gwork, g->ws_neff);
    double* E = gptr(gwork, g->ws_E);
    double* cfg = gptr(gwork, g->ws_cfg);
    bool need_E = true;
    if (p->nx >= kFieldSplitMin) {
        FieldOutputs out{};
        bool any_amr = false;
        for (int s = 0; s < g->ns; ++s) {
            if (g->plans[s]->amr) {
                any_amr = true;
                continue;
            }
            out.a[out.n] = a[s];
            out.qm[out.n] = g->plans[s]->pb.qm;
            ++out.n;
        }
        if (any_amr) {
            out.a[out.n] = E;
            out.qm[out.n] = 1.0;
            ++out.n;
        }
        VP_HIP(timed(p, kTField, stream, [&] {
            return launch_field_split_species(m, p->nx, p->dx, p->d_green, cfg, out, stream);
        }));
        need_E = false;
    } else {
        VP_HIP(launch_species_neff(m, g->nx, n_eff, stream));
        VP_HIP(timed(p, kTField, stream, [&] {
            return launch_poisson1d(nullptr, 0, n_eff, 1.0, p->nx, p->dx, 1.0, p->d_green, p->gk, nullptr, nullptr,
                                    nullptr, E, stream);
        }));
    }
    for (int s = 0; s < g->ns; ++s) {
        const vp_plan* q = g->plans[s];
        double* as = a[s];
        if (!q->amr && !need_E) continue;
        VP_HIP(timed(q, kTOther, stream, [&] {
            if (q->amr) return launch_amr_inject(E, q->amr->ncx, q->amr->R, q->pb.qm, as, stream);
            return launch_scale(E, q->pb.qm, as, q->nx, stream);
        }));
    }
    return VP_OK;
}

double* moment_buf(const vp_species_group* g, void* gwork, int s)
{
    return gptr(gwork, g->ws_n + (size_t)s * align256s((size_t)g->nx * sizeof(double)));
}

vp_status check_group_call(const vp_species_group* g, const void* const* f, double* const* a, void* gwork)
{
    if (!g) return fail(VP_EINVAL, "species group is NULL");
    if (!f || !a || !gwork) return fail(VP_EINVAL, "species call: NULL pointer");
    for (int s = 0; s < g->ns; ++s)
        if (!f[s] || !a[s]) return fail(VP_EINVAL, "species call: NULL state or acceleration");
    return VP_OK;
}

}  // namespace
}  // namespace vp

using namespace vp;

extern "C" {

vp_status vp_species_group_create(const vp_plan* const* plans, const double* charge, int32_t nspecies,
                                  double background, vp_species_group** out)
{
    if (!plans || !charge || !out) return fail(VP_EINVAL, "vp_species_group_create: NULL pointer");
    *out = nullptr;
    if (nspecies < 1 || nspecies > kMaxSpecies)
        return fail(VP_EINVAL, "vp_species_group_create: 1 to " + std::to_string(kMaxSpecies) + " species");
    if (!std::isfinite(background)) return fail(VP_EINVAL, "vp_species_group_create: background must be finite");
    const vp_plan* p0 = plans[0];
    for (int s = 0; s < nspecies; ++s) {
        const vp_plan* p = plans[s];
        if (!p) return fail(VP_EINVAL, "vp_species_group_create: NULL plan");
        if (p->p4 || p->ndim != 1) return fail(VP_ENOTSUP, "vp_species_group_create: 1D+1V plans only");
        if (p->hier) return fail(VP_ENOTSUP, "vp_species_group_create: single-level or two-level plans only");
        if (!std::isfinite(charge[s])) return fail(VP_EINVAL, "vp_species_group_create: charges must be finite");
        if (p->dtype != p0->dtype) return fail(VP_EINVAL, "vp_species_group_create: the plans differ in dtype");
        if (p->nx != p0->nx || p->pb.x_lo[0] != p0->pb.x_lo[0] || p->pb.x_len[0] != p0->pb.x_len[0])
            return fail(VP_EINVAL, "vp_species_group_create: the plans differ in their configuration mesh");
    }
    vp_species_group* g = new (std::nothrow) vp_species_group();
    if (!g) return fail(VP_ENOMEM, "out of host memory");
    g->ns = nspecies;
    g->nx = p0->nx;
    g->background = background;
    for (int s = 0; s < nspecies; ++s) {
        g->plans[s] = plans[s];
        g->charge[s] = charge[s];
    }
    const size_t row = align256s((size_t)g->nx * sizeof(double));
    size_t o = 0;
    g->ws_n = o; o += (size_t)nspecies * row;
    g->ws_neff = o; o += row;
    g->ws_E = o; o += row;
    g->ws_cfg = o; o += align256s(((size_t)g->nx + 4 * ((size_t)g->nx / kFieldChunk + 1) + 64) * sizeof(double));
    g->ws_total = o;
    *out = g;
    return VP_OK;
}

vp_status vp_species_group_destroy(vp_species_group* g)
{
    delete g;
    return VP_OK;
}

size_t vp_species_workspace_bytes(const vp_species_group* g) { return g ? g->ws_total : 0; }

vp_status vp_species_field(const vp_species_group* g, const void* const* f, double* const* a, void* const* work,
                           void* gwork, hipStream_t stream)
{
    if (vp_status st = check_group_call(g, f, a, gwork)) return st;
    SpeciesMoments m{};
    m.ns = g->ns;
    m.background = g->background;
    for (int s = 0; s < g->ns; ++s) {
        double* ns = moment_buf(g, gwork, s);
        void* ws = work ? work[s] : nullptr;
        if (g->plans[s]->amr && !ws) return fail(VP_EINVAL, "vp_species_field: a two-level species needs its workspace");
        if (vp_status st = vp_reduce_moment(g->plans[s], f[s], ns, ws, stream)) return st;
        m.part[s] = ns;
        m.nstrip[s] = 1;
        m.w[s] = g->charge[s];
    }
    return species_field_solve(g, m, gwork, a, stream);
}

vp_status vp_species_rk4_step(const vp_species_group* g, void* const* f, double* const* a, double dt,
                              void* const* work, void* gwork, hipStream_t stream)
{
    if (vp_status st = check_group_call(g, f, a, gwork)) return st;
    if (!work) return fail(VP_EINVAL, "vp_species_rk4_step: NULL workspace list");
    for (int s = 0; s < g->ns; ++s)
        if (!work[s]) return fail(VP_EINVAL, "vp_species_rk4_step: NULL workspace");
    Rk4Setup1D R[kMaxSpecies];
    SpeciesMoments m{};
    m.ns = g->ns;
    m.background = g->background;
    for (int s = 0; s < g->ns; ++s) {
        const vp_plan* p = g->plans[s];
        if (p->amr) {
            // the moment on the finest configuration mesh, by the plan's reduction
            m.part[s] = moment_buf(g, gwork, s);
            m.nstrip[s] = 1;
            m.w[s] = g->charge[s];
        } else {
            // the strip partial sums of the fused stage reduction
            R[s] = rk4_setup_1d(p, f[s], work[s], dt, nullptr);
            m.part[s] = R[s].part;
            m.nstrip[s] = R[s].A.nstrip;
            m.w[s] = g->charge[s] * p->dv;
        }
    }
    for (int st = 0; st < 4; ++st) {
        // every species' stage (each reads its a_s of this stage), then one
        // field solve that writes every a_s of the next stage; a two-level
        // species is synchronised (flux correction, average-down) after its
        // last stage, before its moment is taken
        for (int s = 0; s < g->ns; ++s) {
            const vp_plan* p = g->plans[s];
            if (p->amr) {
                const bool partials = amr_stage_partials(p, st);
                if (vp_status e = amr_stage(p, st, f[s], a[s], dt, work[s], stream, partials)) return e;
                if (st == 3)
                    if (vp_status e = amr_end_sync(p, f[s], dt, work[s], stream)) return e;
                const void* out = amr_stage_output(p, st, f[s], work[s]);
                if (vp_status e = amr_reduce(p, out, moment_buf(g, gwork, s), work[s], stream, partials)) return e;
                continue;
            }
            const Stage1DArgs A = rk4_stage_args_1d(R[s], st, a[s]);
            const StageShape sh = R[s].sh;
            const int kind = R[s].kind[st];
            VP_HIP(timed(p, kTStage, stream, [&] { return launch_stage1d(p->dtype, sh, kind, A, stream); }));
        }
        if (vp_status e = species_field_solve(g, m, gwork, a, stream)) return e;
    }
    return VP_OK;
}

}  // extern "C"
