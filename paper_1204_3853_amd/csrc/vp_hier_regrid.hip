// Regridding of a multi-level hierarchy (section 3: mesh refinement
// criteria, the conservative limited high-order interpolation of new fine
// cells; the hierarchy is rebuilt from the coarsest level up, so every new
// level is nested in the new level below it).  Host code: the criterion and
// the transfer run in the kernels of vp_kernels_regrid.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "vp_internal.hpp"

namespace vp {

namespace {

int rwrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

// dense owner map of level l of a multi-level plan: patch index or -1
std::vector<int> owner_map(const HierPlan& H, int l)
{
    const HLevel& v = H.lv[l];
    std::vector<int> own((size_t)v.nx * v.nv, -1);
    for (size_t q = 0; q < H.patches.size(); ++q) {
        const HPatch& P = H.patches[q];
        if (P.lev != l) continue;
        for (int i = 0; i < P.nx; ++i)
            for (int j = 0; j < P.nv; ++j) own[(size_t)(P.gx0 + i) * v.nv + (P.gv0 + j)] = (int)q;
    }
    return own;
}

// device memory freed at the end of a scope
struct DevMem {
    void* p = nullptr;
    ~DevMem() { if (p) (void)hipFree(p); }
};

}  // namespace

vp_status hier_tag_level(const vp_plan* p, const double* f, int l, double tol, uint8_t* d_tags, double* d_values,
                         void* work, hipStream_t stream)
{
    if (!p || !p->hier) return fail(VP_EINVAL, "hier_tag_level: needs a multi-level plan");
    const HierPlan& H = *p->hier;
    if (l < 0 || l >= H.L) return fail(VP_EINVAL, "hier_tag_level: no such level");
    const HLevel& v = H.lv[l];
    const size_t cells = (size_t)v.nx * v.nv;
    if (vp_status st = hier_fill_frames(p, f, work, stream)) return st;
    VP_HIP(hipMemsetAsync(d_tags, 0, cells, stream));
    if (d_values) VP_HIP(hipMemsetAsync(d_values, 0xff, cells * sizeof(double), stream));     // NaN: no patch
    const int b0 = H.level_begin[l], n = H.level_begin[l + 1] - b0;
    const double* frame = reinterpret_cast<const double*>(static_cast<const char*>(work) + H.ws_frame);
    VP_HIP(launch_hier_tag(f, frame, H.d_patches, H.d_level_list + b0, n, H.level_max_cells[l], v.nv, 1.0 / v.dxi,
                           v.dv, tol, d_tags, d_values, stream));
    return VP_OK;
}

vp_status hier_transfer(const vp_plan* old_plan, const double* f_old, const vp_plan* new_plan, double* f_new,
                        hipStream_t stream)
{
    if (!old_plan || !new_plan || !old_plan->hier || !new_plan->hier)
        return fail(VP_EINVAL, "hier_transfer: needs two multi-level plans");
    const HierPlan& O = *old_plan->hier;
    const HierPlan& N = *new_plan->hier;
    if (O.lv[0].nx != N.lv[0].nx || O.lv[0].nv != N.lv[0].nv)
        return fail(VP_EINVAL, "hier_transfer: the plans have different level-0 meshes");
    for (int l = 1; l < std::min(O.L, N.L); ++l)
        if (O.lv[l].rx != N.lv[l].rx || O.lv[l].rv != N.lv[l].rv)
            return fail(VP_EINVAL, "hier_transfer: the plans have different refinement ratios");
    // every level's records first (host), so that a bad hierarchy is found before any launch
    std::vector<std::vector<int>> win(N.L);
    std::vector<std::vector<HProlongPatch>> pp(N.L);
    std::vector<std::vector<HCopyBlock>> cp(N.L);
    std::vector<int> maxpc(N.L, 0), maxc(N.L, 0);
    for (int l = 1; l < N.L; ++l) {
        const HLevel& v = N.lv[l];
        const HLevel& pv = N.lv[l - 1];
        const std::vector<int> pown = owner_map(N, l - 1);
        // prolongation records: each new level-l patch's parent window, sources in the new state
        for (int b = N.level_begin[l]; b < N.level_begin[l + 1]; ++b) {
            const HPatch& P = N.patches[N.level_list[b]];
            HProlongPatch R{};
            R.off = P.off;
            R.nv = P.nv;
            R.pcx = P.nx / v.rx;
            R.pcv = P.nv / v.rv;
            R.win = (int)win[l].size();
            const int cx0 = P.gx0 / v.rx, cv0 = P.gv0 / v.rv;
            for (int a = -2; a < R.pcx + 2; ++a)
                for (int c = -2; c < R.pcv + 2; ++c) {
                    const int X = cx0 + a, V = cv0 + c;
                    int src;
                    if (V < 0) src = -1 - (4 * (l - 1) + (V + 2));
                    else if (V >= pv.nv) src = -1 - (4 * (l - 1) + 2 + (V - pv.nv));
                    else {
                        const int q = pown[(size_t)rwrap(X, pv.nx) * pv.nv + V];
                        if (q < 0) return fail(VP_EINVAL, "hier_transfer: a new patch is not nested in its new parent level");
                        const HPatch& Q = N.patches[q];
                        src = (int)(Q.off + (long long)(rwrap(X, pv.nx) - Q.gx0) * Q.nv + (V - Q.gv0));
                    }
                    win[l].push_back(src);
                }
            maxpc[l] = std::max(maxpc[l], R.pcx * R.pcv);
            pp[l].push_back(R);
        }
        // old cells of the same level kept
        if (l >= O.L) continue;
        for (int b = N.level_begin[l]; b < N.level_begin[l + 1]; ++b) {
            const HPatch& P = N.patches[N.level_list[b]];
            for (int c = O.level_begin[l]; c < O.level_begin[l + 1]; ++c) {
                const HPatch& Q = O.patches[O.level_list[c]];
                const int x0 = std::max(P.gx0, Q.gx0), x1 = std::min(P.gx0 + P.nx, Q.gx0 + Q.nx) - 1;
                const int v0 = std::max(P.gv0, Q.gv0), v1 = std::min(P.gv0 + P.nv, Q.gv0 + Q.nv) - 1;
                if (x0 > x1 || v0 > v1) continue;
                HCopyBlock B{};
                B.dst = P.off + (long long)(x0 - P.gx0) * P.nv + (v0 - P.gv0);
                B.src = Q.off + (long long)(x0 - Q.gx0) * Q.nv + (v0 - Q.gv0);
                B.dst_stride = P.nv;
                B.src_stride = Q.nv;
                B.nx = x1 - x0 + 1;
                B.nv = v1 - v0 + 1;
                maxc[l] = std::max(maxc[l], B.nx * B.nv);
                cp[l].push_back(B);
            }
        }
    }
    // every level's records in one allocation and one copy
    std::vector<int*> dwin(N.L, nullptr);
    std::vector<HProlongPatch*> dpp(N.L, nullptr);
    std::vector<HCopyBlock*> dcp(N.L, nullptr);
    TableArena T;
    for (int l = 1; l < N.L; ++l) {
        T.add(&dwin[l], win[l]);
        T.add(&dpp[l], pp[l]);
        T.add(&dcp[l], cp[l]);
    }
    DevMem recs;
    VP_HIP(T.commit(&recs.p));
    // level 0 copied, then every level from the coarsest: prolongation from
    // the new parent level, then the old cells of the level
    VP_HIP(hipMemcpyAsync(f_new, f_old, sizeof(double) * (size_t)N.lv[0].nx * N.lv[0].nv, hipMemcpyDeviceToDevice,
                          stream));
    hipError_t e = hipSuccess;
    for (int l = 1; l < N.L && e == hipSuccess; ++l) {
        e = launch_hier_prolong(f_new, dwin[l], dpp[l], (int)pp[l].size(), maxpc[l], N.lv[l].rx, N.lv[l].rv,
                                N.d_eqv, stream);
        if (e == hipSuccess) e = launch_hier_copy(f_new, f_old, dcp[l], (int)cp[l].size(), maxc[l], stream);
    }
    const hipError_t es = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hier_transfer: launch");
    if (es != hipSuccess) return hip_fail(es, "hier_transfer: synchronise");
    return VP_OK;
}

vp_status hier_cluster(const vp_plan* p, int l, const uint8_t* tags, int rx, int rv, double efficiency, int min_width,
                       int buffer, int max_x, int max_v, std::vector<vp_box>& out)
{
    if (!p || !p->hier) return fail(VP_EINVAL, "hier_cluster: needs a multi-level plan");
    const HierPlan& H = *p->hier;
    if (l < 0 || l >= H.L || rx < 1 || rv < 1) return fail(VP_EINVAL, "hier_cluster: no such level or bad ratio");
    const HLevel& v = H.lv[l];
    const int nx = v.nx, nv = v.nv;
    // cells a new level-(l+1) patch may cover: held by level l with every
    // cell within three cells held too (x periodic; outside the velocity box
    // counts as held), so the new level is nested with room for its ghost
    // interpolation (the nesting rule of the multi-level plan)
    const std::vector<int> own = owner_map(H, l);
    // the 7 x 7 erosion of the held cells, one direction at a time: held
    // over the velocity window [j - 3, j + 3] clipped to the box (a prefix
    // count per row), then over the periodic window of rows [i - 3, i + 3]
    std::vector<unsigned char> held_v((size_t)nx * nv), allowed((size_t)nx * nv);
    std::vector<int> pre(nv + 1);
    for (int i = 0; i < nx; ++i) {
        const int* o = own.data() + (size_t)i * nv;
        pre[0] = 0;
        for (int j = 0; j < nv; ++j) pre[j + 1] = pre[j] + (o[j] >= 0);
        for (int j = 0; j < nv; ++j) {
            const int j0 = std::max(j - 3, 0), j1 = std::min(j + 3, nv - 1);
            held_v[(size_t)i * nv + j] = pre[j1 + 1] - pre[j0] == j1 - j0 + 1;
        }
    }
    for (int i = 0; i < nx; ++i) {
        const unsigned char* r[7];
        for (int a = -3; a <= 3; ++a) r[a + 3] = held_v.data() + (size_t)rwrap(i + a, nx) * nv;
        unsigned char* dst = allowed.data() + (size_t)i * nv;
        for (int j = 0; j < nv; ++j)
            dst[j] = r[0][j] & r[1][j] & r[2][j] & r[3][j] & r[4][j] & r[5][j] & r[6][j];
    }
    std::vector<unsigned char> t((size_t)nx * nv);
    for (size_t c = 0; c < t.size(); ++c) t[c] = tags[c] && allowed[c];
    const TagSums st(t, nx, nv, true);
    std::vector<CBox> bx;
    br_cluster(st, CBox{0, 0, nx - 1, nv - 1}, efficiency, min_width, bx);
    for (CBox& b : bx) {
        b.xlo = std::max(b.xlo - buffer, 0); b.xhi = std::min(b.xhi + buffer, nx - 1);
        b.vlo = std::max(b.vlo - buffer, 0); b.vhi = std::min(b.vhi + buffer, nv - 1);
    }
    auto overlap = [](const CBox& a, const CBox& b) {
        return std::max(a.xlo, b.xlo) <= std::min(a.xhi, b.xhi) && std::max(a.vlo, b.vlo) <= std::min(a.vhi, b.vhi);
    };
    for (bool merged = true; merged;) {
        merged = false;
        for (size_t a = 0; a < bx.size() && !merged; ++a)
            for (size_t b = a + 1; b < bx.size() && !merged; ++b)
                if (overlap(bx[a], bx[b])) {
                    bx[a] = CBox{std::min(bx[a].xlo, bx[b].xlo), std::min(bx[a].vlo, bx[b].vlo),
                                 std::max(bx[a].xhi, bx[b].xhi), std::max(bx[a].vhi, bx[b].vhi)};
                    bx.erase(bx.begin() + (long)b);
                    merged = true;
                }
    }
    // a box holding disallowed cells is halved along its longer side until
    // every part is allowed; parts without tags are dropped
    const TagSums sa(allowed, nx, nv);
    std::vector<CBox> todo(bx.begin(), bx.end()), fit;
    while (!todo.empty()) {
        const CBox b = todo.back();
        todo.pop_back();
        if (st.count(b.xlo, b.vlo, b.xhi, b.vhi) == 0) continue;
        if (sa.count(b.xlo, b.vlo, b.xhi, b.vhi) == b.area()) {
            fit.push_back(b);
            continue;
        }
        CBox lo = b, hi = b;
        if (b.xhi - b.xlo >= b.vhi - b.vlo) {
            const int m = (b.xlo + b.xhi) / 2;
            lo.xhi = m; hi.xlo = m + 1;
        } else {
            const int m = (b.vlo + b.vhi) / 2;
            lo.vhi = m; hi.vlo = m + 1;
        }
        todo.push_back(lo);
        todo.push_back(hi);
    }
    // largest patch size (cells of level l + 1): split into near-equal parts
    std::vector<CBox> fin;
    for (const CBox& b : fit) {
        const int wx = b.xhi - b.xlo + 1, wv = b.vhi - b.vlo + 1;
        const int mx = max_x > 0 ? std::max(1, max_x / rx) : wx, mv = max_v > 0 ? std::max(1, max_v / rv) : wv;
        const int kx = (wx + mx - 1) / mx, kv = (wv + mv - 1) / mv;
        for (int a = 0; a < kx; ++a)
            for (int c = 0; c < kv; ++c)
                fin.push_back(CBox{b.xlo + a * wx / kx, b.vlo + c * wv / kv, b.xlo + (a + 1) * wx / kx - 1,
                                   b.vlo + (c + 1) * wv / kv - 1});
    }
    std::sort(fin.begin(), fin.end(), [](const CBox& a, const CBox& b) {
        return a.xlo != b.xlo ? a.xlo < b.xlo : a.vlo < b.vlo;
    });
    out.clear();
    for (const CBox& b : fin) {
        vp_box o{};
        o.level = l + 1;
        o.lo[0] = b.xlo * rx;
        o.lo[1] = b.vlo * rv;
        o.hi[0] = (b.xhi + 1) * rx - 1;
        o.hi[1] = (b.vhi + 1) * rv - 1;
        out.push_back(o);
    }
    return VP_OK;
}

}  // namespace vp
