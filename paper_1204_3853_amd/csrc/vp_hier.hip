// Host runtime of the multi-level path (L <= 4 levels, a refinement ratio
// per level and direction; section 3, the hierarchy of levels with ratio
// vectors; section 4 runs ratios [2,4], [4,2], [2,2]): box validation and
// nesting, the ghost-frame sources of every patch (same-level copy,
// equilibrium, or parent interpolation), the Sub-Patch reduction lists
// (Alg. subdiv against the next finer level, Alg. spreduce), the
// coarse-fine faces of every level pair, the average-down lists, device
// tables, and the enqueue sequence of one synchronous RK4 step
// (Alg. smsvphu without regridding).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "vp_internal.hpp"

namespace vp {

namespace {

struct HBox {
    int xlo, vlo, xhi, vhi;   // inclusive
    bool empty() const { return xlo > xhi || vlo > vhi; }
};

HBox hsect(const HBox& a, const HBox& b)
{
    return HBox{std::max(a.xlo, b.xlo), std::max(a.vlo, b.vlo), std::min(a.xhi, b.xhi), std::min(a.vhi, b.vhi)};
}

int hwrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

char* wsp(void* work, size_t off) { return static_cast<char*>(work) + off; }

constexpr long long kMaxLevelCells = 1LL << 25;   // index-space cells per level (host owner maps)

struct Builder {
    int L = 0;
    HLevel lv[kHierLevels] = {};
    std::vector<HPatch> P;
    std::vector<std::vector<int>> owner;           // per level: patch holding each cell, or -1

    int holder(int l, int X, int V) const
    {
        if (V < 0 || V >= lv[l].nv) return -1;
        return owner[l][(size_t)hwrap(X, lv[l].nx) * lv[l].nv + V];
    }
    long long offset(int p, int l, int X, int V) const
    {
        const HPatch& q = P[p];
        return q.off + (long long)(hwrap(X, lv[l].nx) - q.gx0) * q.nv + (V - q.gv0);
    }
    // source code of level-l cell (X, V): state offset, or -1 - equilibrium index; -2^31 when not held
    int source(int l, int X, int V) const
    {
        if (V < 0) return -1 - (4 * l + (V + 2));
        if (V >= lv[l].nv) return -1 - (4 * l + 2 + (V - lv[l].nv));
        const int p = holder(l, X, V);
        if (p < 0) return INT32_MIN;
        return (int)offset(p, l, X, V);
    }
};

void fill_tiles(HierPlan& H)
{
    const int tv = H.nt * H.w;
    H.tiles.clear();
    for (size_t p = 0; p < H.patches.size(); ++p) {
        const HPatch& q = H.patches[p];
        const int ns = (q.nv + tv - 1) / tv, nseg = (q.nx + H.tx - 1) / H.tx;
        for (int g = 0; g < nseg; ++g)
            for (int b = 0; b < ns; ++b) H.tiles.push_back(AmrTile{kTileFine, (int)p, g, b});
    }
    H.face_tile_begin = (int)H.tiles.size();
    for (int f0 = 0; f0 < H.nfaces; f0 += H.nt) H.tiles.push_back(AmrTile{kTileFaces, f0, std::min(H.nt, H.nfaces - f0), 0});
    H.ntiles = (int)H.tiles.size();
}

hipError_t upload_tiles(HierPlan& H)
{
    if (H.d_tiles) (void)hipFree(H.d_tiles);
    H.d_tiles = nullptr;
    if (H.tiles.empty()) return hipSuccess;
    hipError_t e = hipMalloc(&H.d_tiles, H.tiles.size() * sizeof(AmrTile));
    if (e != hipSuccess) return e;
    return hipMemcpy(H.d_tiles, H.tiles.data(), H.tiles.size() * sizeof(AmrTile), hipMemcpyHostToDevice);
}

HierArgs base_args(const vp_plan* p, const double* fs, const double* a, void* work)
{
    const HierPlan& H = *p->hier;
    HierArgs A{};
    for (int l = 0; l < H.L; ++l) A.lv[l] = H.lv[l];
    A.patches = H.d_patches;
    A.tiles = H.d_tiles;
    A.tx = H.tx;
    A.v_lo = p->pb.v_lo[0];
    A.fs = fs;
    A.a = a;
    A.frame = reinterpret_cast<const double*>(wsp(work, H.ws_frame));
    A.eqv = H.d_eqv;
    A.faces = H.d_faces;
    A.cf_acc = reinterpret_cast<double*>(wsp(work, H.ws_cf));
    A.ff_acc = reinterpret_cast<double*>(wsp(work, H.ws_ff));
    return A;
}

vp_status fill_frames(const vp_plan* p, const double* f, void* work, hipStream_t stream)
{
    return hier_fill_frames(p, f, work, stream);
}
}  // namespace

vp_status hier_fill_frames(const vp_plan* p, const double* f, void* work, hipStream_t stream)
{
    const HierPlan& H = *p->hier;
    double* frame = reinterpret_cast<double*>(wsp(work, H.ws_frame));
    VP_HIP(timed(p, kTOther, stream, [&] {
        return launch_hier_fill(f, H.d_desc, H.d_rec, H.d_wts, H.d_wofs, H.d_eqv, frame, H.nframe, stream);
    }));
    return VP_OK;
}

namespace {

// the velocity moment on the finest configuration mesh (Sub-Patch
// reduction); the frames of f must be filled
vp_status reduce_filled(const vp_plan* p, const double* f, double* n, void* work, hipStream_t stream)
{
    const HierPlan& H = *p->hier;
    const double* frame = reinterpret_cast<const double*>(wsp(work, H.ws_frame));
    double* slots = reinterpret_cast<double*>(wsp(work, H.ws_slots));
    VP_HIP(timed(p, kTMoment, stream, [&] {
        hipError_t e = launch_hier_rowsum(f, frame, H.d_task_off, H.d_task_len, H.ntasks, slots, stream);
        if (e != hipSuccess) return e;
        return launch_amr_reduce_finalize(slots, H.d_rowptr, H.d_idx, H.d_w, H.lv[H.L - 1].nx, n, stream);
    }));
    return VP_OK;
}

// reduction -> Poisson and field on the finest configuration mesh -> a on every level
vp_status constraint(const vp_plan* p, const double* f, double* a, void* work, hipStream_t stream)
{
    const HierPlan& H = *p->hier;
    const int nfx = H.lv[H.L - 1].nx;
    double* n = reinterpret_cast<double*>(wsp(work, H.ws_n));
    double* E = reinterpret_cast<double*>(wsp(work, H.ws_E));
    if (vp_status st = reduce_filled(p, f, n, work, stream)) return st;
    VP_HIP(timed(p, kTField, stream, [&] {
        if (nfx >= kFieldSplitMin) {
            SpeciesMoments m{};
            m.part[0] = n;
            m.nstrip[0] = 1;
            m.w[0] = -1.0;
            m.ns = 1;
            m.background = 1.0;
            FieldOutputs out{};
            out.a[0] = E;
            out.qm[0] = 1.0;
            out.n = 1;
            double* scratch = reinterpret_cast<double*>(wsp(work, H.ws_fld));
            return launch_field_split_species(m, nfx, H.dxf, p->d_green, scratch, out, stream);
        }
        // the injection onto every level in the same launch
        int off[kHierLevels], rt[kHierLevels];
        for (int l = 0; l < H.L; ++l) {
            off[l] = H.lv[l].a_off;
            rt[l] = H.lv[l].rt;
        }
        return launch_poisson1d_levels(n, nfx, H.dxf, p->pb.qm, p->d_green, p->gk, E, a, H.L, off, rt, stream);
    }));
    if (nfx >= kFieldSplitMin)
        VP_HIP(timed(p, kTOther, stream, [&] {
            return launch_hier_inject(E, H.lv, H.L, p->pb.qm, a, H.na, stream);
        }));
    return VP_OK;
}

vp_status launch_stage(const vp_plan* p, int kind, const HierArgs& A, hipStream_t stream)
{
    const HierPlan& H = *p->hier;
    const int grid = std::min(std::max(H.ntiles, 1), 256 * 8);
    VP_HIP(timed(p, kTStage, stream, [&] { return launch_hier_stage(H.w, H.nt, kind, A, 0, H.ntiles, grid, stream); }));
    return VP_OK;
}

}  // namespace

vp_status hier_set_shape(vp_plan* p, int nt, int w, int tx)
{
    HierPlan& H = *p->hier;
    if (!((nt == 64 || nt == 128) && (w == 1 || w == 2) && tx >= 1 && tx <= kMaxTx))
        return fail(VP_EINVAL, "hierarchy tile shape must be threads 64|128, cells 1|2, rows 1..128");
    if (w == 2)
        for (const HPatch& q : H.patches)
            if (q.nv % 2) return fail(VP_EINVAL, "two cells per thread needs even velocity widths on every patch");
    VP_HIP(hipDeviceSynchronize());       // the old tile table may still be read by queued launches
    H.nt = nt;
    H.w = w;
    H.tx = tx;
    fill_tiles(H);
    VP_HIP(upload_tiles(H));
    return VP_OK;
}

vp_status hier_create(vp_plan* p, const vp_problem* pb, const vp_box* boxes, int nbox, bool tag_only)
{
    if (pb->ndim != 1) return fail(VP_ENOTSUP, "multi-level hierarchies are supported for 1D+1V");
    if (pb->dtype != VP_F64) return fail(VP_ENOTSUP, "multi-level hierarchies are supported in FP64");
    const int L = pb->n_levels;
    Builder B;
    B.L = L;
    HierPlan* Hp = new HierPlan();
    p->hier = Hp;
    HierPlan& H = *Hp;
    H.L = L;
    H.tag_only = tag_only;
    const double x_len = pb->x_len[0], vspan = pb->v_hi[0] - pb->v_lo[0];
    for (int l = 0; l < L; ++l) {
        HLevel& v = B.lv[l];
        if (l == 0) {
            v.nx = pb->cells[0];
            v.nv = pb->cells[1];
            v.rx = v.rv = 1;
        } else {
            v.rx = pb->ratio[l - 1][0];
            v.rv = pb->ratio[l - 1][1];
            const auto ok = [](int r) { return r == 1 || r == 2 || r == 4 || r == 8; };
            if (!ok(v.rx) || !ok(v.rv) || v.rx * v.rv == 1)
                return fail(VP_ENOTSUP, "refinement ratios must be 1, 2, 4 or 8 per direction (not both 1)");
            v.nx = B.lv[l - 1].nx * v.rx;
            v.nv = B.lv[l - 1].nv * v.rv;
        }
        if ((long long)v.nx * v.nv > kMaxLevelCells) return fail(VP_ENOTSUP, "level index space too large");
        if (!pb->veq[l][0]) return fail(VP_EINVAL, "veq[l][0] (equilibrium with ghosts) is required on every level");
        v.dxi = v.nx / x_len;
        v.dv = vspan / v.nv;
        v.dvi = 1.0 / v.dv;
        v.dv24 = v.dv / 24.0;
    }
    int a_off = 0;
    for (int l = 0; l < L; ++l) {
        B.lv[l].rt = 1;
        for (int m = l + 1; m < L; ++m) B.lv[l].rt *= B.lv[m].rx;
        B.lv[l].a_off = a_off;
        a_off += B.lv[l].nx;
    }
    H.na = a_off;
    const int nfx = B.lv[L - 1].nx;
    H.dxf = x_len / nfx;
    if (nfx > kMaxPoisson1D) return fail(VP_ENOTSUP, "finest configuration mesh larger than 8192 cells");
    for (int l = 0; l < L; ++l) {
        const double* q = pb->veq[l][0];
        const int nv = B.lv[l].nv;
        for (double g : {q[0], q[1], q[nv + 2], q[nv + 3]}) H.eqv.push_back(g);
    }

    // ---- patches: level 0, then the boxes in order; layout of state, frames, boundary fluxes
    B.owner.resize(L);
    for (int l = 0; l < L; ++l) B.owner[l].assign((size_t)B.lv[l].nx * B.lv[l].nv, l == 0 ? 0 : -1);
    std::vector<HBox> bx{HBox{0, 0, B.lv[0].nx - 1, B.lv[0].nv - 1}};
    {
        HPatch q{};
        q.lev = 0;
        q.nx = B.lv[0].nx;
        q.nv = B.lv[0].nv;
        B.P.push_back(q);
    }
    for (int k = 0; k < nbox; ++k) {
        const vp_box& b = boxes[k];
        const int l = b.level;
        if (l < 1 || l >= L) return fail(VP_EINVAL, "box " + std::to_string(k) + ": level must be 1 .. n_levels-1");
        const HLevel& v = B.lv[l];
        HBox X{b.lo[0], b.lo[1], b.hi[0], b.hi[1]};
        if (X.empty() || X.xlo < 0 || X.vlo < 0 || X.xhi >= v.nx || X.vhi >= v.nv)
            return fail(VP_EINVAL, "box " + std::to_string(k) + " is empty or outside its level");
        if (X.xlo % v.rx || (X.xhi + 1) % v.rx || X.vlo % v.rv || (X.vhi + 1) % v.rv)
            return fail(VP_EINVAL, "box " + std::to_string(k) + " is not aligned to its level's refinement ratio");
        const int pid = (int)B.P.size();
        for (size_t r = 1; r < bx.size(); ++r)
            if (B.P[r].lev == l && !hsect(bx[r], X).empty())
                return fail(VP_EINVAL, "boxes " + std::to_string(r - 1) + " and " + std::to_string(k) + " overlap");
        for (int i = X.xlo; i <= X.xhi; ++i)
            std::fill_n(B.owner[l].begin() + (size_t)i * v.nv + X.vlo, X.vhi - X.vlo + 1, pid);
        HPatch q{};
        q.lev = l;
        q.gx0 = X.xlo;
        q.gv0 = X.vlo;
        q.nx = X.xhi - X.xlo + 1;
        q.nv = X.vhi - X.vlo + 1;
        B.P.push_back(q);
        bx.push_back(X);
    }
    size_t off = 0, foff = 0, fro = 0;
    for (HPatch& q : B.P) {
        q.off = (long long)off;
        q.frame = (long long)fro;
        q.foff = (long long)foff;
        off += (size_t)q.nx * q.nv;
        fro += 4 * (size_t)(q.nv + 4) + 4 * (size_t)q.nx;
        foff += 2 * (size_t)(q.nx + q.nv);
    }
    if (off >= (size_t)INT32_MAX) return fail(VP_ENOTSUP, "hierarchy state larger than 2^31 elements");
    H.total = off;
    H.frame_elems = fro;
    H.fflux = foff;

    // ---- ghost frames: copy, equilibrium, or interpolation from the parent level
    std::vector<int2> desc;
    std::vector<HInterp> rec;
    desc.reserve(fro);
    for (size_t pi = 0; pi < B.P.size(); ++pi) {
        const HPatch& q = B.P[pi];
        const int l = q.lev;
        // the parent cells a frame reads, each one's 25 sources found once:
        // the record that first used it, per parent cell of the frame's
        // bounding box (x unwrapped)
        const int rxl = l > 0 ? B.lv[l].rx : 1, rvl = l > 0 ? B.lv[l].rv : 1;
        const int pc0 = (q.gx0 - 2 - (rxl - 1)) / rxl - 1, pv0 = std::max(q.gv0 - 2, 0) / rvl;
        const int pcn = (q.gx0 + q.nx + 2) / rxl - pc0 + 2, pvn = (q.gv0 + q.nv + 2) / rvl - pv0 + 2;
        std::vector<int> first_rec(l > 0 ? (size_t)pcn * pvn : 0, -1);
        auto add = [&](int r, int c) -> bool {
            const int X = q.gx0 + r, V = q.gv0 + c;
            const int s = B.source(l, X, V);
            if (s != INT32_MIN) {
                desc.push_back(s >= 0 ? int2{s, 0} : int2{-1, -1 - s});
                return true;
            }
            const HLevel& v = B.lv[l];
            const int Xw = hwrap(X, v.nx);
            HInterp R{};
            R.lev = l;
            const int ci = Xw / v.rx, cj = V / v.rv;
            R.s = Xw - ci * v.rx;
            R.t = V - cj * v.rv;
            const int cu = (X >= 0 ? X : X - v.rx + 1) / v.rx;          // parent cell, x unwrapped
            int* cached = nullptr;
            if (l > 0 && cu >= pc0 && cu < pc0 + pcn && cj >= pv0 && cj < pv0 + pvn)
                cached = &first_rec[(size_t)(cu - pc0) * pvn + (cj - pv0)];
            if (cached && *cached >= 0) {
                std::memcpy(R.src, rec[*cached].src, sizeof(R.src));
            } else {
                for (int a = -2; a <= 2; ++a)
                    for (int b = -2; b <= 2; ++b) {
                        const int src = B.source(l - 1, ci + a, cj + b);
                        if (src == INT32_MIN) return false;
                        R.src[(a + 2) * 5 + b + 2] = src;
                    }
                if (cached) *cached = (int)rec.size();
            }
            desc.push_back(int2{-2, (int)rec.size()});
            rec.push_back(R);
            return true;
        };
        bool ok = true;
        for (int r : {-2, -1, q.nx, q.nx + 1})
            for (int c = -2; c < q.nv + 2 && ok; ++c) ok = add(r, c);
        for (int r = 0; r < q.nx && ok; ++r)
            for (int c : {-2, -1, q.nv, q.nv + 1})
                if (ok) ok = add(r, c);
        if (!ok)
            return fail(VP_EINVAL, "box " + std::to_string((int)pi - 1) +
                                       ": a ghost cell interpolates from parent cells no patch of the parent level holds "
                                       "(the level is not nested inside its parent with three cells to spare)");
    }
    H.nframe = (int)desc.size();
    std::vector<double> wts;
    std::vector<int> wofs(2 * kHierLevels, 0);
    for (int l = 1; l < L; ++l) {
        wofs[2 * l] = (int)wts.size();
        const std::vector<double> bxw = interp_table(B.lv[l].rx);
        wts.insert(wts.end(), bxw.begin(), bxw.end());
        wofs[2 * l + 1] = (int)wts.size();
        const std::vector<double> bvw = interp_table(B.lv[l].rv);
        wts.insert(wts.end(), bvw.begin(), bvw.end());
    }

    // ---- coarse-fine faces of every level pair, their corrections, average-down lists
    std::vector<HFace> faces;
    std::vector<long long> corr_fine;
    std::vector<int> corr_nfine;
    std::vector<std::pair<long long, int>> corr;     // (corrected cell, encoded face), in the order found
    std::vector<std::vector<long long>> avg_dst(L), avg_src(L);
    std::vector<std::vector<int>> avg_stride(L);
    bool nested = true;
    auto covered = [&](int l, int i, int j) {
        if (j < 0 || j >= B.lv[l].nv) return false;
        return B.holder(l + 1, hwrap(i, B.lv[l].nx) * B.lv[l + 1].rx, j * B.lv[l + 1].rv) >= 0;
    };
    auto stencil = [&](int l, int i, int j, int dir, HFace& F) {
        for (int m = -1; m <= 1; ++m)
            for (int q = 0; q < 4; ++q) {
                const int X = dir == 0 ? i - 1 + q : i + m, V = dir == 0 ? j + m : j - 1 + q;
                const int s = B.source(l, X, V);
                if (s == INT32_MIN) nested = false;
                F.src[(m + 1) * 4 + q] = s == INT32_MIN ? 0 : s;
            }
    };
    auto cell_off = [&](int l, int i, int j) -> long long {
        const int q = B.holder(l, i, j);
        if (q < 0) { nested = false; return 0; }
        return B.offset(q, l, i, j);
    };
    for (size_t gi = 1; gi < (tag_only ? 1 : B.P.size()); ++gi) {
        const HPatch& G = B.P[gi];
        const int l = G.lev - 1;
        const int rx = B.lv[l + 1].rx, rv = B.lv[l + 1].rv;
        const int cx0 = G.gx0 / rx, cx1 = (G.gx0 + G.nx) / rx - 1, cv0 = G.gv0 / rv, cv1 = (G.gv0 + G.nv) / rv - 1;
        const int ncx = B.lv[l].nx;
        for (int cj = cv0; cj <= cv1; ++cj) {
            // lower x side: face between (cx0 - 1, cj) and (cx0, cj)
            if (!covered(l, cx0 - 1, cj)) {
                HFace F{};
                F.dir = 0;
                F.lev = l;
                F.vb = pb->v_lo[0] + (cj + 0.5) * B.lv[l].dv;
                stencil(l, cx0 - 1, cj, 0, F);
                corr.emplace_back(cell_off(l, cx0 - 1, cj), (int)faces.size());         // its upper face
                corr_fine.push_back(G.foff + (cj * rv - G.gv0));
                corr_nfine.push_back(rv);
                faces.push_back(F);
            }
            // upper x side: face between (cx1, cj) and (cx1 + 1, cj)
            if (!covered(l, cx1 + 1, cj)) {
                HFace F{};
                F.dir = 0;
                F.lev = l;
                F.vb = pb->v_lo[0] + (cj + 0.5) * B.lv[l].dv;
                stencil(l, cx1, cj, 0, F);
                corr.emplace_back(cell_off(l, cx1 + 1, cj), -1 - (int)faces.size());    // its lower face
                corr_fine.push_back(G.foff + G.nv + (cj * rv - G.gv0));
                corr_nfine.push_back(rv);
                faces.push_back(F);
            }
        }
        for (int ci = cx0; ci <= cx1; ++ci) {
            const int aim = B.lv[l].a_off + hwrap(ci - 1, ncx), ai0 = B.lv[l].a_off + hwrap(ci, ncx),
                      aip = B.lv[l].a_off + hwrap(ci + 1, ncx);
            // lower v side: face between (ci, cv0 - 1) and (ci, cv0), inside the velocity box
            if (cv0 > 0 && !covered(l, ci, cv0 - 1)) {
                HFace F{};
                F.dir = 1;
                F.lev = l;
                F.ai[0] = aim; F.ai[1] = ai0; F.ai[2] = aip;
                stencil(l, ci, cv0 - 1, 1, F);
                corr.emplace_back(cell_off(l, ci, cv0 - 1), (int)faces.size());
                corr_fine.push_back(G.foff + 2 * G.nv + (ci * rx - G.gx0));
                corr_nfine.push_back(rx);
                faces.push_back(F);
            }
            if (cv1 + 1 < B.lv[l].nv && !covered(l, ci, cv1 + 1)) {
                HFace F{};
                F.dir = 1;
                F.lev = l;
                F.ai[0] = aim; F.ai[1] = ai0; F.ai[2] = aip;
                stencil(l, ci, cv1, 1, F);
                corr.emplace_back(cell_off(l, ci, cv1 + 1), -1 - (int)faces.size());
                corr_fine.push_back(G.foff + 2 * G.nv + G.nx + (ci * rx - G.gx0));
                corr_nfine.push_back(rx);
                faces.push_back(F);
            }
            const int* own_row = B.owner[l].data() + (size_t)hwrap(ci, ncx) * B.lv[l].nv;
            for (int cj = cv0; cj <= cv1; ++cj) {
                const int q = own_row[cj];
                if (q < 0) { nested = false; continue; }
                avg_dst[l].push_back(B.P[q].off + (long long)(hwrap(ci, ncx) - B.P[q].gx0) * B.P[q].nv + (cj - B.P[q].gv0));
                avg_src[l].push_back(G.off + (long long)(ci * rx - G.gx0) * G.nv + (cj * rv - G.gv0));
                avg_stride[l].push_back(G.nv);
            }
        }
    }
    if (!nested) return fail(VP_EINVAL, "a coarse-fine face or a covered cell lies outside the parent level");
    H.nfaces = (int)faces.size();
    // grouped by cell in increasing order, each cell's faces in the order found
    std::stable_sort(corr.begin(), corr.end(),
                     [](const std::pair<long long, int>& a, const std::pair<long long, int>& b) { return a.first < b.first; });
    std::vector<int> corr_ptr{0}, corr_face;
    std::vector<long long> corr_cell;
    for (size_t e = 0; e < corr.size(); ++e) {
        if (e > 0 && corr[e].first != corr[e - 1].first) corr_ptr.push_back((int)corr_face.size());
        if (e == 0 || corr[e].first != corr[e - 1].first) corr_cell.push_back(corr[e].first);
        corr_face.push_back(corr[e].second);
    }
    if (!corr.empty()) corr_ptr.push_back((int)corr_face.size());
    H.ncorr = (int)corr_cell.size();

    // ---- Sub-Patch reduction: each patch minus the next finer level (Alg. subdiv),
    // each sub-patch grown by two columns in x (patch rows or frame rows), its
    // rows summed over its velocity range, refined in x to the finest mesh
    std::vector<long long> task_off;
    std::vector<int> task_len;
    struct Contrib {
        int I, slot;
        double w;
    };
    std::vector<Contrib> contrib;                    // (fine cell, slot, weight), in the order found
    for (size_t pi = 0; pi < (tag_only ? 0 : B.P.size()); ++pi) {
        const HPatch& q = B.P[pi];
        const int l = q.lev;
        const HBox box{q.gx0, q.gv0, q.gx0 + q.nx - 1, q.gv0 + q.nv - 1};
        std::vector<HBox> S{box};
        if (l + 1 < L) {
            const int rx = B.lv[l + 1].rx, rv = B.lv[l + 1].rv;
            for (size_t gi = 1; gi < B.P.size(); ++gi) {
                const HPatch& G = B.P[gi];
                if (G.lev != l + 1) continue;
                const HBox Pc{G.gx0 / rx, G.gv0 / rv, (G.gx0 + G.nx) / rx - 1, (G.gv0 + G.nv) / rv - 1};
                if (hsect(Pc, box).empty()) continue;
                const HBox ext{Pc.xlo, box.vlo, Pc.xhi, box.vhi};
                std::vector<HBox> S2;
                for (const HBox& s : S) {
                    const HBox in = hsect(s, ext);
                    if (in.empty()) { S2.push_back(s); continue; }
                    if (s.xlo < in.xlo) S2.push_back(HBox{s.xlo, s.vlo, in.xlo - 1, s.vhi});
                    if (in.xhi < s.xhi) S2.push_back(HBox{in.xhi + 1, s.vlo, s.xhi, s.vhi});
                    const HBox below{in.xlo, in.vlo, in.xhi, std::min(in.vhi, Pc.vlo - 1)};
                    const HBox above{in.xlo, std::max(in.vlo, Pc.vhi + 1), in.xhi, in.vhi};
                    if (!below.empty()) S2.push_back(below);
                    if (!above.empty()) S2.push_back(above);
                }
                S.swap(S2);
            }
        }
        const int rt = B.lv[l].rt;
        const std::vector<double> Br = interp_table(rt);
        for (const HBox& s : S) {
            const int base = (int)task_off.size();
            for (int i = s.xlo - 2; i <= s.xhi + 2; ++i) {
                long long o;
                if (i >= box.xlo && i <= box.xhi) {
                    o = q.off + (long long)(i - box.xlo) * q.nv + (s.vlo - box.vlo);
                } else {
                    const int r = i < box.xlo ? i - box.xlo + 2 : i - box.xhi + 1;   // frame row 0, 1 | 2, 3
                    o = -1 - (q.frame + (long long)r * (q.nv + 4) + (s.vlo - box.vlo + 2));
                }
                task_off.push_back(o);
                task_len.push_back(s.vhi - s.vlo + 1);
            }
            for (int i = s.xlo; i <= s.xhi; ++i)
                for (int sx = 0; sx < rt; ++sx)
                    for (int a = -2; a <= 2; ++a)
                        contrib.push_back(Contrib{i * rt + sx, base + (i + a - (s.xlo - 2)), Br[sx * 5 + a + 2] * B.lv[l].dv});
        }
    }
    H.ntasks = (int)task_off.size();
    // per fine cell, its terms in the order found (a counting sort)
    std::vector<int> rowptr(tag_only ? 1 : (size_t)nfx + 1, 0), idx(contrib.size());
    std::vector<double> w(contrib.size());
    if (!tag_only) {
        for (const Contrib& c : contrib) ++rowptr[c.I + 1];
        for (int I = 0; I < nfx; ++I) rowptr[I + 1] += rowptr[I];
        std::vector<int> fill(rowptr.begin(), rowptr.end() - 1);
        for (const Contrib& c : contrib) {
            const int e = fill[c.I]++;
            idx[e] = c.slot;
            w[e] = c.w;
        }
    }

    // ---- device tables
    for (int l = 0; l < L; ++l) H.lv[l] = B.lv[l];
    H.patches = B.P;
    H.w = std::all_of(H.patches.begin(), H.patches.end(), [](const HPatch& q) { return q.nv % 2 == 0; }) ? 2 : 1;
    H.nt = 64;
    H.tx = 8;
    if (!tag_only) {
        fill_tiles(H);
        VP_HIP(upload_tiles(H));
    }
    std::vector<HLevel> lvv(H.lv, H.lv + L);
    for (int l = 0; l < L; ++l) {
        H.level_begin[l] = (int)H.level_list.size();
        for (size_t q = 0; q < H.patches.size(); ++q)
            if (H.patches[q].lev == l) {
                H.level_list.push_back((int)q);
                H.level_max_cells[l] = std::max(H.level_max_cells[l], H.patches[q].nx * H.patches[q].nv);
            }
    }
    H.level_begin[L] = (int)H.level_list.size();
    TableArena T;
    T.add(&H.d_patches, H.patches);
    T.add(&H.d_desc, desc);
    T.add(&H.d_rec, rec);
    T.add(&H.d_wts, wts);
    T.add(&H.d_wofs, wofs);
    T.add(&H.d_eqv, H.eqv);
    T.add(&H.d_faces, faces);
    T.add(&H.d_lv, lvv);
    T.add(&H.d_task_off, task_off);
    T.add(&H.d_task_len, task_len);
    T.add(&H.d_rowptr, rowptr);
    T.add(&H.d_idx, idx);
    T.add(&H.d_w, w);
    T.add(&H.d_corr_ptr, corr_ptr);
    T.add(&H.d_corr_face, corr_face);
    T.add(&H.d_corr_cell, corr_cell);
    T.add(&H.d_corr_fine, corr_fine);
    T.add(&H.d_corr_nfine, corr_nfine);
    T.add(&H.d_level_list, H.level_list);
    for (int l = 0; l + 1 < L; ++l) {
        H.avg[l].rx = B.lv[l + 1].rx;
        H.avg[l].rv = B.lv[l + 1].rv;
        H.avg[l].n = (int)avg_dst[l].size();
        T.add(&H.avg[l].d_dst, avg_dst[l]);
        T.add(&H.avg[l].d_src, avg_src[l]);
        T.add(&H.avg[l].d_stride, avg_stride[l]);
    }
    VP_HIP(T.commit(&H.d_tables));
    if (!tag_only) VP_HIP(hipMalloc(&H.d_rhs_frame, std::max<size_t>(H.frame_elems, 1) * sizeof(double)));

    // ---- workspace: acc, two predictors, frames, accumulated fluxes, row sums, n, E, field scratch
    const size_t sb = a256(H.total * sizeof(double));
    size_t o = 0;
    p->ws_acc = o; o += sb;
    p->ws_fsa = o; o += sb;
    p->ws_fsb = o; o += sb;
    H.ws_frame = o; o += a256(std::max<size_t>(H.frame_elems, 1) * sizeof(double));
    H.ws_cf = o; o += a256(std::max<size_t>(faces.size(), 1) * sizeof(double));
    H.ws_ff = o; o += a256(std::max<size_t>(H.fflux, 1) * sizeof(double));
    H.ws_slots = o; o += a256(std::max<size_t>(H.ntasks, 1) * sizeof(double));
    H.ws_n = o; o += a256((size_t)nfx * sizeof(double));
    H.ws_E = o; o += a256((size_t)nfx * sizeof(double));
    H.ws_fld = o; o += a256(((size_t)nfx + 4 * ((size_t)nfx / kFieldChunk + 1) + 64) * sizeof(double));
    p->ws_total = o;
    p->state_elems = H.total;
    return VP_OK;
}

void hier_destroy(vp_plan* p)
{
    HierPlan* H = p->hier;
    if (!H) return;
    if (H->d_tables) (void)hipFree(H->d_tables);
    if (H->d_tiles) (void)hipFree(H->d_tiles);
    if (H->d_rhs_frame) (void)hipFree(H->d_rhs_frame);
    delete H;
    p->hier = nullptr;
}

vp_status hier_rhs(const vp_plan* p, const void* f, const double* a, void* k, hipStream_t stream)
{
    const HierPlan& H = *p->hier;
    const double* fs = static_cast<const double*>(f);
    double* frame = H.d_rhs_frame;
    VP_HIP(timed(p, kTOther, stream, [&] {
        return launch_hier_fill(fs, H.d_desc, H.d_rec, H.d_wts, H.d_wofs, H.d_eqv, frame, H.nframe, stream);
    }));
    HierArgs A{};
    for (int l = 0; l < H.L; ++l) A.lv[l] = H.lv[l];
    A.patches = H.d_patches;
    A.tiles = H.d_tiles;
    A.tx = H.tx;
    A.v_lo = p->pb.v_lo[0];
    A.fs = fs;
    A.a = a;
    A.frame = frame;
    A.eqv = H.d_eqv;
    A.fout = static_cast<double*>(k);
    return launch_stage(p, kRhs, A, stream);
}

vp_status hier_reduce(const vp_plan* p, const void* f, double* n, void* work, hipStream_t stream)
{
    const double* fs = static_cast<const double*>(f);
    if (vp_status st = fill_frames(p, fs, work, stream)) return st;
    return reduce_filled(p, fs, n, work, stream);
}

vp_status hier_inject(const vp_plan* p, const double* E, double* a, hipStream_t stream)
{
    const HierPlan& H = *p->hier;
    VP_HIP(timed(p, kTOther, stream, [&] { return launch_hier_inject(E, H.lv, H.L, p->pb.qm, a, H.na, stream); }));
    return VP_OK;
}

vp_status hier_rk4(const vp_plan* p, void* f, double* a, double dt, void* work, hipStream_t stream,
                   const double* dt_dev)
{
    const HierPlan& H = *p->hier;
    double* fd = static_cast<double*>(f);
    double* acc = reinterpret_cast<double*>(wsp(work, p->ws_acc));
    double* sa = reinterpret_cast<double*>(wsp(work, p->ws_fsa));
    double* sb = reinterpret_cast<double*>(wsp(work, p->ws_fsb));
    const double* in[4] = {fd, sa, sb, sa};
    double* out[4] = {sa, sb, sa, fd};
    const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    // with the time step in device memory the kernels multiply it in (dt b_s, dt/2, dt: the same products)
    const double sc = dt_dev ? 1.0 : dt;
    const double cnext[3] = {0.5 * sc, 0.5 * sc, sc};
    if (vp_status st = fill_frames(p, fd, work, stream)) return st;
    for (int s = 0; s < 4; ++s) {
        const int kind = s == 0 ? kStage1 : (s == 3 ? kStage4 : kStage23);
        HierArgs A = base_args(p, in[s], a, work);
        A.fn = fd;
        A.acc = acc;
        A.fout = out[s];
        A.c_acc = dt_dev ? b[s] : dt * b[s];
        A.c_next = s < 3 ? cnext[s] : 0.0;
        A.dt = dt_dev;
        A.c_flux = b[s];
        A.first = s == 0;
        if (vp_status st = launch_stage(p, kind, A, stream)) return st;
        if (s < 3) {
            if (vp_status st = fill_frames(p, out[s], work, stream)) return st;
            if (vp_status st = constraint(p, out[s], a, work, stream)) return st;
        }
    }
    // end of step: the coarse-fine flux correction on every level, then the
    // average-down from the finest level (Alg. msfduc)
    HierSyncArgs S{};
    S.f = fd;
    for (int l = 0; l < H.L; ++l) S.lv[l] = H.lv[l];
    S.dt = dt;
    S.dt_dev = dt_dev;
    S.faces = H.d_faces;
    S.cf_acc = reinterpret_cast<const double*>(wsp(work, H.ws_cf));
    S.ff_acc = reinterpret_cast<const double*>(wsp(work, H.ws_ff));
    S.corr_ptr = H.d_corr_ptr;
    S.corr_face = H.d_corr_face;
    S.corr_cell = H.d_corr_cell;
    S.corr_fine = H.d_corr_fine;
    S.corr_nfine = H.d_corr_nfine;
    S.ncorr = H.ncorr;
    VP_HIP(timed(p, kTSync, stream, [&] { return launch_hier_reflux(S, stream); }));
    for (int l = H.L - 2; l >= 0; --l) {
        HierAvgArgs G{};
        G.f = fd;
        G.dst = H.avg[l].d_dst;
        G.src = H.avg[l].d_src;
        G.stride = H.avg[l].d_stride;
        G.rx = H.avg[l].rx;
        G.rv = H.avg[l].rv;
        G.n = H.avg[l].n;
        VP_HIP(timed(p, kTSync, stream, [&] { return launch_hier_average(G, stream); }));
    }
    if (vp_status st = fill_frames(p, fd, work, stream)) return st;
    return constraint(p, fd, a, work, stream);
}

}  // namespace vp
