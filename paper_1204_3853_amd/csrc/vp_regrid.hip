// Regridding entry points (section 3): the refinement criterion on level 0,
// the clustering of tagged level-0 cells into level-1 boxes (host), and the
// transfer of a state to a plan with new level-1 patches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "vp_internal.hpp"

namespace vp {

hipError_t launch_tag(const double* f, int nx, int nv, const double* vg, double dx, double dv, double tol,
                      unsigned char* tags, double* values, hipStream_t stream);
hipError_t launch_prolong(const double* fc, int ncx, int ncv, const double* vgc, int R, const AmrPatch* d_patches,
                          int npatch, int max_coarse_cells, double* fnew, hipStream_t stream);
hipError_t launch_copy_old(const double* fold, const AmrPatch* d_old, int nold, const AmrPatch* d_new, int nnew,
                           int max_fine_cells, double* fnew, hipStream_t stream);

namespace {

// level 0 of a 1D+1V plan: the single level, or the coarse level of two
struct Level0 {
    int nx, nv;
    double dx, dv;
    const double* vg;
};

bool level0_of(const vp_plan* p, Level0& L)
{
    if (!p || p->p4 || p->hier || p->ndim != 1) return false;
    if (p->amr) {
        const AmrPlan& M = *p->amr;
        L = Level0{M.ncx, M.ncv, M.dxc, M.dvc, M.vgc};
    } else {
        L = Level0{p->nx, p->nv, p->dx, p->dv, p->vg};
    }
    return true;
}

}  // namespace

TagSums::TagSums(const std::vector<unsigned char>& m, int mx, int mv, bool bounded) : nx(mx), nv(mv)
{
    if (bounded) {
        // the rows holding set cells, and the velocity range of those cells
        int xa = mx, xb = -1, va = mv, vb = -1;
        for (int i = 0; i < mx; ++i) {
            const unsigned char* r = m.data() + (size_t)i * mv;
            const unsigned char* f = std::find_if(r, r + mv, [](unsigned char c) { return c != 0; });
            if (f == r + mv) continue;
            const unsigned char* l = r + mv - 1;
            while (*l == 0) --l;
            xa = std::min(xa, i);
            xb = i;
            va = std::min(va, (int)(f - r));
            vb = std::max(vb, (int)(l - r));
        }
        if (xb < 0) { xa = xb = 0; va = vb = 0; }
        x0 = xa;
        v0 = va;
        nx = xb - xa + 1;
        nv = vb - va + 1;
    }
    s.assign((size_t)(nx + 1) * (nv + 1), 0);
    for (int i = 0; i < nx; ++i) {
        const unsigned char* r = m.data() + (size_t)(x0 + i) * mv + v0;
        int row = 0;
        for (int j = 0; j < nv; ++j) {
            row += r[j] != 0;
            s[(size_t)(i + 1) * (nv + 1) + j + 1] = s[(size_t)i * (nv + 1) + j + 1] + row;
        }
    }
}

namespace {

// Berger-Rigoutsos: split the bounding box of the tags inside B at a hole
// of a signature, else at the strongest inflection of a signature's
// second difference, else in the middle of the longer side, until each
// box holds at least `eff` tagged cells per cell or cannot be split into
// two parts of at least `minw` cells.  The signatures (tagged cells per
// row and per column of B) come from the summed-area table, so a box costs
// the length of its sides, not its area.
void br_split(const TagSums& T, CBox B, double eff, int minw, std::vector<CBox>& out)
{
    const int bwx = B.xhi - B.xlo + 1, bwv = B.vhi - B.vlo + 1;
    std::vector<long long> fx(bwx), fv(bwv);
    long long nt = 0;
    for (int i = 0; i < bwx; ++i) nt += fx[i] = T.count(B.xlo + i, B.vlo, B.xlo + i, B.vhi);
    if (nt == 0) return;
    for (int j = 0; j < bwv; ++j) fv[j] = T.count(B.xlo, B.vlo + j, B.xhi, B.vlo + j);
    // shrink to the tags' bounding box (every tag of B lies in it, so the
    // signatures over B restricted to it are its own)
    int x0 = 0, x1 = bwx - 1, v0 = 0, v1 = bwv - 1;
    while (fx[x0] == 0) ++x0;
    while (fx[x1] == 0) --x1;
    while (fv[v0] == 0) ++v0;
    while (fv[v1] == 0) --v1;
    const std::vector<long long> sx(fx.begin() + x0, fx.begin() + x1 + 1), sv(fv.begin() + v0, fv.begin() + v1 + 1);
    B = CBox{B.xlo + x0, B.vlo + v0, B.xlo + x1, B.vlo + v1};
    const int wx = B.xhi - B.xlo + 1, wv = B.vhi - B.vlo + 1;
    if ((double)nt >= eff * (double)B.area() || (wx < 2 * minw && wv < 2 * minw)) {
        out.push_back(B);
        return;
    }
    // candidate cut: the first cell of the upper part, at offset c of a side
    // of width w (minw <= c <= w - minw); best = (class, score, distance to the middle)
    int best_dir = -1, best_cut = 0;
    long long best_score = -1;
    int best_class = 3;                      // 0 hole, 1 inflection, 2 middle
    int best_dist = 1 << 30;
    auto consider = [&](int dir, int c, int cls, long long score, int w) {
        const int dist = std::abs(2 * c - w);
        if (cls < best_class || (cls == best_class && (score > best_score || (score == best_score && dist < best_dist)))) {
            best_class = cls; best_score = score; best_dist = dist; best_dir = dir; best_cut = c;
        }
    };
    for (int dir = 0; dir < 2; ++dir) {
        const std::vector<long long>& sg = dir == 0 ? sx : sv;
        const int w = (int)sg.size();
        if (w < 2 * minw) continue;
        for (int c = minw; c <= w - minw; ++c)
            if (sg[c - 1] == 0 || sg[c] == 0) consider(dir, c, 0, 0, w);
        for (int c = std::max(minw, 2); c <= std::min(w - minw, w - 2); ++c) {
            // inflection between cells c-1 and c: second differences change sign
            const long long l0 = sg[c - 2] - 2 * sg[c - 1] + sg[c];
            const long long l1 = sg[c - 1] - 2 * sg[c] + sg[c + 1];
            if ((l0 < 0 && l1 > 0) || (l0 > 0 && l1 < 0)) consider(dir, c, 1, std::llabs(l1 - l0), w);
        }
        consider(dir, w / 2, 2, w, w);
    }
    if (best_dir < 0) {
        out.push_back(B);
        return;
    }
    CBox lo = B, hi = B;
    if (best_dir == 0) { lo.xhi = B.xlo + best_cut - 1; hi.xlo = B.xlo + best_cut; }
    else { lo.vhi = B.vlo + best_cut - 1; hi.vlo = B.vlo + best_cut; }
    br_split(T, lo, eff, minw, out);
    br_split(T, hi, eff, minw, out);
}

}  // namespace

void br_cluster(const TagSums& T, CBox B, double eff, int minw, std::vector<CBox>& out) { br_split(T, B, eff, minw, out); }

void br_cluster(const std::vector<unsigned char>& tag, int nv, CBox B, double eff, int minw, std::vector<CBox>& out)
{
    br_split(TagSums(tag, (int)(tag.size() / (size_t)nv), nv, true), B, eff, minw, out);
}

namespace {

bool overlap(const CBox& a, const CBox& b)
{
    return std::max(a.xlo, b.xlo) <= std::min(a.xhi, b.xhi) && std::max(a.vlo, b.vlo) <= std::min(a.vhi, b.vhi);
}

}  // namespace

}  // namespace vp

using namespace vp;

extern "C" {

vp_status vp_tag_cells(const vp_plan* p, const void* f, double tol, uint8_t* tags, double* values,
                       hipStream_t stream)
{
    Level0 L;
    if (!p) return fail(VP_EINVAL, "vp_tag_cells: plan is NULL");
    if (!f || !tags) return fail(VP_EINVAL, "vp_tag_cells: NULL pointer");
    if (p->p4) {
        if (p->dtype != VP_F64) return fail(VP_ENOTSUP, "vp_tag_cells: FP64 plans only");
        const Plan4D& Q = *p->p4;
        Tag4DArgs a{};
        a.f = static_cast<const double*>(f);
        a.nx = Q.nx;
        a.ny = Q.ny;
        a.nvx = Q.nvx;
        a.nvy = Q.nvy;
        a.gx = Q.d_gx;
        a.gy = Q.d_gy;
        a.h[0] = Q.dx;
        a.h[1] = Q.dy;
        a.h[2] = Q.dvx;
        a.h[3] = Q.dvy;
        a.tol = tol;
        a.tags = tags;
        a.values = values;
        VP_HIP(launch_tag4d(a, stream));
        return VP_OK;
    }
    if (!level0_of(p, L)) return fail(VP_ENOTSUP, "vp_tag_cells: 1D+1V plans only");
    if (p->dtype != VP_F64) return fail(VP_ENOTSUP, "vp_tag_cells: FP64 plans only");
    VP_HIP(launch_tag(static_cast<const double*>(f), L.nx, L.nv, L.vg, L.dx, L.dv, tol, tags, values, stream));
    return VP_OK;
}

vp_status vp_cluster_tags(const uint8_t* tags, int32_t ncx, int32_t ncv, int32_t ratio, double efficiency,
                          int32_t min_width, int32_t buffer, vp_box* boxes, int32_t max_boxes, int32_t* nbox)
{
    if (!tags || !nbox || (max_boxes > 0 && !boxes)) return fail(VP_EINVAL, "vp_cluster_tags: NULL pointer");
    if (ncx < 1 || ncv < 1 || ratio < 1 || min_width < 1 || buffer < 0 || !(efficiency > 0.0 && efficiency <= 1.0))
        return fail(VP_EINVAL, "vp_cluster_tags: bad sizes or parameters");
    std::vector<unsigned char> t(tags, tags + (size_t)ncx * ncv);
    std::vector<CBox> bx;
    br_cluster(t, ncv, CBox{0, 0, ncx - 1, ncv - 1}, efficiency, min_width, bx);
    // buffer cells around every box, inside the domain (patches may touch,
    // also across the periodic x boundary, but never wrap)
    for (CBox& b : bx) {
        b.xlo = std::max(b.xlo - buffer, 0); b.xhi = std::min(b.xhi + buffer, ncx - 1);
        b.vlo = std::max(b.vlo - buffer, 0); b.vhi = std::min(b.vhi + buffer, ncv - 1);
    }
    // boxes that overlap after the buffer are replaced by their bounding box
    // until none do
    for (bool merged = true; merged;) {
        merged = false;
        for (size_t a = 0; a < bx.size() && !merged; ++a)
            for (size_t b = a + 1; b < bx.size() && !merged; ++b)
                if (overlap(bx[a], bx[b])) {
                    CBox u{std::min(bx[a].xlo, bx[b].xlo), std::min(bx[a].vlo, bx[b].vlo),
                           std::max(bx[a].xhi, bx[b].xhi), std::max(bx[a].vhi, bx[b].vhi)};
                    bx[a] = u;
                    bx.erase(bx.begin() + (long)b);
                    merged = true;
                }
    }
    std::sort(bx.begin(), bx.end(), [](const CBox& a, const CBox& b) {
        return a.xlo != b.xlo ? a.xlo < b.xlo : a.vlo < b.vlo;
    });
    *nbox = (int32_t)bx.size();
    if ((int32_t)bx.size() > max_boxes)
        return fail(VP_EINVAL, "vp_cluster_tags: " + std::to_string(bx.size()) + " boxes, room for " +
                                   std::to_string(max_boxes));
    for (size_t q = 0; q < bx.size(); ++q) {
        vp_box& o = boxes[q];
        std::memset(&o, 0, sizeof(o));
        o.level = 1;
        o.lo[0] = bx[q].xlo * ratio;
        o.lo[1] = bx[q].vlo * ratio;
        o.hi[0] = (bx[q].xhi + 1) * ratio - 1;
        o.hi[1] = (bx[q].vhi + 1) * ratio - 1;
    }
    return VP_OK;
}

vp_status vp_regrid_transfer(const vp_plan* old_plan, const void* f_old, const vp_plan* new_plan, void* f_new,
                             hipStream_t stream)
{
    Level0 A, B;
    if (!old_plan || !new_plan || !f_old || !f_new) return fail(VP_EINVAL, "vp_regrid_transfer: NULL pointer");
    if (old_plan->hier || new_plan->hier)
        return hier_transfer(old_plan, static_cast<const double*>(f_old), new_plan, static_cast<double*>(f_new), stream);
    if (!level0_of(old_plan, A) || !level0_of(new_plan, B))
        return fail(VP_ENOTSUP, "vp_regrid_transfer: 1D+1V plans only");
    if (old_plan->dtype != VP_F64 || new_plan->dtype != VP_F64)
        return fail(VP_ENOTSUP, "vp_regrid_transfer: FP64 plans only");
    if (A.nx != B.nx || A.nv != B.nv || A.dx != B.dx || A.dv != B.dv || std::memcmp(A.vg, B.vg, 4 * sizeof(double)))
        return fail(VP_EINVAL, "vp_regrid_transfer: the plans have different level-0 meshes");
    if (old_plan->amr && new_plan->amr && old_plan->amr->R != new_plan->amr->R)
        return fail(VP_EINVAL, "vp_regrid_transfer: the plans have different refinement ratios");
    const double* fo = static_cast<const double*>(f_old);
    double* fn = static_cast<double*>(f_new);
    VP_HIP(hipMemcpyAsync(fn, fo, sizeof(double) * (size_t)A.nx * A.nv, hipMemcpyDeviceToDevice, stream));
    if (!new_plan->amr) return VP_OK;
    const AmrPlan& N = *new_plan->amr;
    int max_c = 0, max_f = 0;
    for (const AmrPatch& P : N.patches) {
        max_c = std::max(max_c, (P.nx / N.R) * (P.nv / N.R));
        max_f = std::max(max_f, P.nx * P.nv);
    }
    VP_HIP(launch_prolong(fo, A.nx, A.nv, A.vg, N.R, N.d_patches, (int)N.patches.size(), max_c, fn, stream));
    if (old_plan->amr) {
        const AmrPlan& O = *old_plan->amr;
        VP_HIP(launch_copy_old(fo, O.d_patches, (int)O.patches.size(), N.d_patches, (int)N.patches.size(), max_f, fn,
                               stream));
    }
    return VP_OK;
}

vp_status vp_tag_level(const vp_plan* p, const void* f, int32_t level, double tol, uint8_t* tags, double* values,
                       void* work, hipStream_t stream)
{
    if (!p || !f || !tags || !work) return fail(VP_EINVAL, "vp_tag_level: NULL pointer");
    if (!p->hier) return fail(VP_ENOTSUP, "vp_tag_level: multi-level plans only (vp_tag_cells for the others)");
    return hier_tag_level(p, static_cast<const double*>(f), level, tol, tags, values, work, stream);
}

vp_status vp_cluster_level(const vp_plan* p, int32_t level, const uint8_t* tags, int32_t ratio_x, int32_t ratio_v,
                           double efficiency, int32_t min_width, int32_t buffer, int32_t max_x, int32_t max_v,
                           vp_box* boxes, int32_t max_boxes, int32_t* nbox)
{
    if (!p || !tags || !nbox || (max_boxes > 0 && !boxes)) return fail(VP_EINVAL, "vp_cluster_level: NULL pointer");
    if (!p->hier) return fail(VP_ENOTSUP, "vp_cluster_level: multi-level plans only (vp_cluster_tags for the others)");
    if (min_width < 1 || buffer < 0 || max_x < 0 || max_v < 0 || !(efficiency > 0.0 && efficiency <= 1.0))
        return fail(VP_EINVAL, "vp_cluster_level: bad parameters");
    std::vector<vp_box> out;
    if (vp_status st = hier_cluster(p, level, tags, ratio_x, ratio_v, efficiency, min_width, buffer, max_x, max_v, out))
        return st;
    *nbox = (int32_t)out.size();
    if (*nbox > max_boxes)
        return fail(VP_EINVAL, "vp_cluster_level: " + std::to_string(out.size()) + " boxes, room for " +
                                   std::to_string(max_boxes));
    std::copy(out.begin(), out.end(), boxes);
    return VP_OK;
}

}  // extern "C"
