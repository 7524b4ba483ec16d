// Host runtime of the two-level path: box validation and box calculus
// (section 3: coverage, coarse-fine faces, the Sub-Patch decomposition of
// Alg. subdiv), device tables, and the enqueue sequence of one synchronous
// RK4 step (Alg. smsvphu without regridding).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "vp_internal.hpp"

namespace vp {

// b_j(s) of the fifth-order conservative sub-cell interpolation (section 3),
// with p_k(s) = ((s+1)^{k+1} - s^{k+1}) / R^k
std::vector<double> interp_table(int R)
{
    std::vector<double> B((size_t)R * 5);
    for (int s = 0; s < R; ++s) {
        double p[5];
        p[0] = 1.0;
        for (int k = 1; k <= 4; ++k) p[k] = (std::pow(s + 1.0, k + 1) - std::pow((double)s, k + 1)) / std::pow((double)R, k);
        B[s * 5 + 0] = (p[4] - 5 * p[3] + 5 * p[2] + 5 * p[1] - 6) / 120.0;
        B[s * 5 + 1] = (-4 * p[4] + 15 * p[3] + 10 * p[2] - 75 * p[1] + 54) / 120.0;
        B[s * 5 + 2] = (6 * p[4] - 15 * p[3] - 40 * p[2] + 75 * p[1] + 94) / 120.0;
        B[s * 5 + 3] = (-4 * p[4] + 5 * p[3] + 30 * p[2] - 5 * p[1] - 26) / 120.0;
        B[s * 5 + 4] = (p[4] - 5 * p[2] + 4) / 120.0;
    }
    return B;
}

namespace {

struct Box {
    int xlo, vlo, xhi, vhi;   // inclusive
    bool empty() const { return xlo > xhi || vlo > vhi; }
};

Box intersect(const Box& a, const Box& b)
{
    return Box{std::max(a.xlo, b.xlo), std::max(a.vlo, b.vlo), std::min(a.xhi, b.xhi), std::min(a.vhi, b.vhi)};
}

template <typename T>
hipError_t upload(T** dst, const std::vector<T>& v)
{
    if (*dst) (void)hipFree(*dst);
    *dst = nullptr;
    if (v.empty()) return hipSuccess;
    hipError_t e = hipMalloc(dst, v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

char* wsp(void* work, size_t off) { return static_cast<char*>(work) + off; }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// tile table for the shape (nt, w, tx)
void build_tiles(AmrPlan& A)
{
    const int tv = A.nt * A.w;
    A.tiles.clear();
    A.patch_tile_begin.clear();
    A.nstrip_c = (A.ncv + tv - 1) / tv;
    const int nseg_c = (A.ncx + A.tx - 1) / A.tx;
    A.ncoarse_tiles = A.nstrip_c * nseg_c;
    for (int t = 0; t < A.ncoarse_tiles; ++t) A.tiles.push_back(AmrTile{kTileCoarse, 0, t, 0});
    for (size_t p = 0; p < A.patches.size(); ++p) {
        A.patch_tile_begin.push_back((int)A.tiles.size());
        const AmrPatch& P = A.patches[p];
        const int ns = (P.nv + tv - 1) / tv, nseg = (P.nx + A.tx - 1) / A.tx;
        for (int g = 0; g < nseg; ++g)
            for (int b = 0; b < ns; ++b) A.tiles.push_back(AmrTile{kTileFine, (int)p, g, b});
    }
    A.face_tile_begin = (int)A.tiles.size();
    A.patch_tile_begin.push_back(A.face_tile_begin);
    const int nf = (int)A.faces.size();
    for (int f0 = 0; f0 < nf; f0 += A.nt) A.tiles.push_back(AmrTile{kTileFaces, f0, std::min(A.nt, nf - f0), 0});
    A.ntiles = (int)A.tiles.size();
}

// the tile table on the device: the table, then the same tiles in the order
// the one-launch stage takes them.  One block per tile: the longer fine tiles
// (their halo is interpolated from the coarse level first) are dispatched
// first, and the short coarse and face tiles fill the CUs as blocks finish.
hipError_t upload_tiles(AmrPlan& A)
{
    std::vector<AmrTile> v(A.tiles);
    v.insert(v.end(), A.tiles.begin() + A.ncoarse_tiles, A.tiles.begin() + A.face_tile_begin);
    v.insert(v.end(), A.tiles.begin(), A.tiles.begin() + A.ncoarse_tiles);
    v.insert(v.end(), A.tiles.begin() + A.face_tile_begin, A.tiles.end());
    hipError_t e = upload(&A.d_tiles, v);
    A.d_tiles_run = A.d_tiles ? A.d_tiles + A.ntiles : nullptr;
    return e;
}

// the fine strip partials of each coarse column's R fine cells, for the
// Mask reduction from the stage kernel's row sums: fine cell by fine cell,
// patch by patch (patch order), strip by strip (the tiles' strips)
hipError_t upload_fused_lists(AmrPlan& A)
{
    const int tv = A.nt * A.w;
    std::vector<int> ptr{0};
    std::vector<int2> ent;
    for (int i = 0; i < A.ncx; ++i) {
        for (int s = 0; s < A.R; ++s) {
            const int I = i * A.R + s;
            for (int e = A.fcol_ptr[I]; e < A.fcol_ptr[I + 1]; ++e) {
                const AmrPatch& P = A.patches[A.fcol_patch[e]];
                const int ns = (P.nv + tv - 1) / tv;
                for (int b = 0; b < ns; ++b)
                    ent.push_back(make_int2((int)(P.fpart + (long long)b * P.nx + (I - P.gx0)), s));
            }
        }
        ptr.push_back((int)ent.size());
    }
    if (A.d_fz) (void)hipFree(A.d_fz);
    A.d_fz = nullptr;
    TableArena T;
    T.add(&A.d_fz_ptr, ptr);
    T.add(&A.d_fz_entry, ent);
    return T.commit(&A.d_fz);
}

AmrArgs stage_args(const vp_plan* p, const void* fs, const void* fn, void* acc, void* fout, const double* a,
                   double c_acc, double c_next, double c_flux, int first, void* work)
{
    const AmrPlan& M = *p->amr;
    AmrArgs A{};
    Stage1DArgs& C = A.coarse;
    C.nx = M.ncx;
    C.nv = M.ncv;
    C.tx = M.tx;
    C.nstrip = M.nstrip_c;
    C.dxi = 1.0 / M.dxc;
    C.dvi = 1.0 / M.dvc;
    C.dv24 = M.dvc / 24.0;
    C.v_lo = M.v_lo;
    C.dv = M.dvc;
    for (int q = 0; q < 4; ++q) C.vg[q] = M.vgc[q];
    C.fs = fs;
    C.fn = fn;
    C.acc = acc;
    C.fout = fout;
    C.a = a;
    C.part = nullptr;
    C.c_acc = c_acc;
    C.c_next = c_next;
    A.patches = M.d_patches;
    A.tiles = M.d_tiles;
    A.ntiles = M.ntiles;
    A.lim = p->face_scheme == VP_FACE_LIMITED;
    A.nfx = M.nfx;
    A.nfv = M.nfv;
    A.R = M.R;
    A.lr = M.lr;
    A.tx = M.tx;
    A.dxfi = 1.0 / M.dxf;
    A.dvfi = 1.0 / M.dvf;
    A.dvf24 = M.dvf / 24.0;
    A.dvf = M.dvf;
    A.v_lo = M.v_lo;
    for (int q = 0; q < 4; ++q) A.vgf[q] = M.vgf[q];
    A.a_f = a + M.ncx;
    A.B = M.d_B;
    A.faces = M.d_faces;
    A.nb = M.d_nb;
    A.cf_acc = work ? reinterpret_cast<double*>(wsp(work, M.ws_cf)) : nullptr;
    A.ff_acc = work ? reinterpret_cast<double*>(wsp(work, M.ws_ff)) : nullptr;
    A.c_flux = c_flux;
    A.first = first;
    return A;
}

hipError_t launch_stage_all(const vp_plan* p, int kind, const AmrArgs& A, hipStream_t stream)
{
    const AmrPlan& M = *p->amr;
    const int cap = 256 * 8;
    if (M.mode == 0) {
        AmrArgs B = A;
        B.tiles = M.d_tiles_run;
        return launch_amr_stage(M.w, M.nt, kind, B, 0, M.ntiles, std::min(M.ntiles, 1 << 16), stream);
    }
    // baseline: the coarse level, each patch and the face chunks as separate launches
    hipError_t e = launch_amr_stage(M.w, M.nt, kind, A, 0, M.ncoarse_tiles, std::min(M.ncoarse_tiles, cap), stream);
    if (e != hipSuccess) return e;
    for (size_t q = 0; q + 1 < M.patch_tile_begin.size(); ++q) {
        const int t0 = M.patch_tile_begin[q], t1 = M.patch_tile_begin[q + 1];
        e = launch_amr_stage(M.w, M.nt, kind, A, t0, t1, std::min(t1 - t0, cap), stream);
        if (e != hipSuccess) return e;
    }
    if (M.ntiles > M.face_tile_begin)
        e = launch_amr_stage(M.w, M.nt, kind, A, M.face_tile_begin, M.ntiles,
                             std::min(M.ntiles - M.face_tile_begin, cap), stream);
    return e;
}

// velocity moment on the finest configuration mesh, by the plan's reduction algorithm
hipError_t reduce_launch(const AmrPlan& M, const double* f, double* n, void* work, hipStream_t stream)
{
    if (M.reduce_mode == VP_REDUCE_MASK) {
        double* sm = reinterpret_cast<double*>(wsp(work, M.ws_slots_m));
        hipError_t e = launch_amr_mask_rows(f, M.d_mask, M.ncx, M.ncv, sm, stream);
        if (e != hipSuccess) return e;
        e = launch_amr_rowsum(f, M.d_task_off + M.fine_task0, M.d_task_len + M.fine_task0, M.ntasks - M.fine_task0,
                              sm + 5 * M.ncx, stream);
        if (e != hipSuccess) return e;
        return launch_amr_reduce_finalize(sm, M.d_rowptr_m, M.d_idx_m, M.d_w_m, M.nfx, n, stream);
    }
    double* slots = reinterpret_cast<double*>(wsp(work, M.ws_slots));
    hipError_t e = launch_amr_rowsum(f, M.d_task_off, M.d_task_len, M.ntasks, slots, stream);
    if (e != hipSuccess) return e;
    return launch_amr_reduce_finalize(slots, M.d_rowptr, M.d_idx, M.d_w, M.nfx, n, stream);
}

// the Mask reduction of the stage state f from the strip partials the
// stage kernel wrote for it
hipError_t reduce_fused_launch(const AmrPlan& M, const double* f, double* n, void* work, hipStream_t stream)
{
    AmrMaskFusedArgs R{};
    R.f = f;
    R.part_c = reinterpret_cast<const double*>(wsp(work, M.ws_pc));
    R.part_f = reinterpret_cast<const double*>(wsp(work, M.ws_pf));
    R.patches = M.d_patches;
    R.cov_ptr = M.d_covc_ptr;
    R.cov_j = M.d_covc_j;
    R.fz_ptr = M.d_fz_ptr;
    R.fz_entry = M.d_fz_entry;
    R.B = M.d_B;
    R.ncx = M.ncx;
    R.ncv = M.ncv;
    R.nstrip = M.nstrip_c;
    R.R = M.R;
    R.tv = M.nt * M.w;
    R.dvc = M.dvc;
    R.dvf = M.dvf;
    R.n = n;
    return launch_amr_mask_fused(R, stream);
}

// reduction -> Poisson on the finest configuration mesh -> injection (the
// Poisson block also injects the field onto both levels); partials: the
// stage kernel that wrote f also wrote its strip partials
vp_status constraint(const vp_plan* p, const double* f, double* a, void* work, hipStream_t stream,
                     bool partials = false)
{
    const AmrPlan& M = *p->amr;
    double* n = reinterpret_cast<double*>(wsp(work, M.ws_n));
    double* E = reinterpret_cast<double*>(wsp(work, M.ws_E));
    VP_HIP(timed(p, kTMoment, stream, [&] {
        return partials ? reduce_fused_launch(M, f, n, work, stream) : reduce_launch(M, f, n, work, stream);
    }));
    if (M.nfx >= kFieldSplitMin) {
        // the split solve over many blocks; its last kernel also injects
        SpeciesMoments m{};
        m.part[0] = n;
        m.nstrip[0] = 1;
        m.w[0] = -1.0;
        m.ns = 1;
        m.background = 1.0;
        FieldOutputs out{};
        out.a[0] = a + M.ncx;
        out.qm[0] = p->pb.qm;
        out.a[1] = E;
        out.qm[1] = 1.0;
        out.n = 2;
        out.inject_a = a;
        out.inject_qm = p->pb.qm;
        out.inject_R = M.R;
        double* scratch = reinterpret_cast<double*>(wsp(work, M.ws_fld));
        VP_HIP(timed(p, kTField, stream, [&] {
            return launch_field_split_species(m, M.nfx, M.dxf, p->d_green, scratch, out, stream);
        }));
        return VP_OK;
    }
    const PoissonExtra X{nullptr, nullptr, nullptr, nullptr, M.R};
    VP_HIP(timed(p, kTField, stream, [&] {
        return launch_poisson1d_inject(n, X, M.nfx, M.dxf, p->pb.qm, p->d_green, p->gk, E, a, stream);
    }));
    return VP_OK;
}

}  // namespace

vp_status amr_set_shape(vp_plan* p, int nt, int w, int tx)
{
    AmrPlan& M = *p->amr;
    if (!((nt == 64 || nt == 128) && (w == 1 || w == 2) && tx >= 1 && tx <= kMaxTx))
        return fail(VP_EINVAL, "two-level tile shape must be threads 64|128, cells 1|2, rows 1..128");
    if (w == 2) {
        if (M.ncv % 2) return fail(VP_EINVAL, "two cells per thread needs an even coarse velocity count");
        for (const AmrPatch& P : M.patches)
            if (P.nv % 2) return fail(VP_EINVAL, "two cells per thread needs even patch widths");
    }
    VP_HIP(hipDeviceSynchronize());       // the old tile table may still be read by queued launches
    M.nt = nt;
    M.w = w;
    M.tx = tx;
    build_tiles(M);
    VP_HIP(upload_tiles(M));
    VP_HIP(upload_fused_lists(M));
    return VP_OK;
}

vp_status amr_create(vp_plan* p, const vp_problem* pb, const vp_box* boxes, int nbox)
{
    if (pb->ndim != 1) return fail(VP_ENOTSUP, "two levels are supported for 1D+1V");
    if (pb->dtype != VP_F64) return fail(VP_ENOTSUP, "two levels are supported in FP64");
    const int R = pb->ratio[0][0];
    if (pb->ratio[0][1] != R || (R != 2 && R != 4)) return fail(VP_ENOTSUP, "refinement ratio must be 2 or 4, equal in x and v");
    if (!pb->veq[1][0]) return fail(VP_EINVAL, "veq[1][0] (level-1 equilibrium with ghosts) is required");
    AmrPlan* M = new AmrPlan();
    p->amr = M;
    M->ncx = pb->cells[0];
    M->ncv = pb->cells[1];
    M->R = R;
    M->lr = R == 4 ? 2 : 1;
    M->nfx = M->ncx * R;
    M->nfv = M->ncv * R;
    M->dxc = pb->x_len[0] / M->ncx;
    M->dvc = (pb->v_hi[0] - pb->v_lo[0]) / M->ncv;
    M->dxf = M->dxc / R;
    M->dvf = M->dvc / R;
    M->v_lo = pb->v_lo[0];
    const double* vc = pb->veq[0][0];
    const double* vf = pb->veq[1][0];
    M->vgc[0] = vc[0]; M->vgc[1] = vc[1]; M->vgc[2] = vc[M->ncv + 2]; M->vgc[3] = vc[M->ncv + 3];
    M->vgf[0] = vf[0]; M->vgf[1] = vf[1]; M->vgf[2] = vf[M->nfv + 2]; M->vgf[3] = vf[M->nfv + 3];
    if (M->nfx > kMaxPoisson1D) return fail(VP_ENOTSUP, "finest configuration mesh larger than 8192 cells");

    // ---- boxes: level 1, inside the domain, aligned to R, disjoint (touching allowed)
    std::vector<Box> bx;
    for (int q = 0; q < nbox; ++q) {
        const vp_box& b = boxes[q];
        if (b.level != 1) return fail(VP_EINVAL, "boxes must be on level 1");
        Box B{b.lo[0], b.lo[1], b.hi[0], b.hi[1]};
        if (B.empty() || B.xlo < 0 || B.vlo < 0 || B.xhi >= M->nfx || B.vhi >= M->nfv)
            return fail(VP_EINVAL, "box " + std::to_string(q) + " is empty or outside the level-1 domain");
        if (B.xlo % R || B.vlo % R || (B.xhi + 1) % R || (B.vhi + 1) % R)
            return fail(VP_EINVAL, "box " + std::to_string(q) + " is not aligned to the refinement ratio");
        for (size_t r = 0; r < bx.size(); ++r)
            if (!intersect(B, bx[r]).empty())
                return fail(VP_EINVAL, "boxes " + std::to_string(r) + " and " + std::to_string(q) + " overlap");
        bx.push_back(B);
    }

    // ---- patches and state layout
    size_t off = (size_t)M->ncx * M->ncv, foff = 0, fpart = 0;
    for (const Box& B : bx) {
        AmrPatch P{};
        P.off = (long long)off;
        P.foff = (long long)foff;
        P.gx0 = B.xlo;
        P.gv0 = B.vlo;
        P.nx = B.xhi - B.xlo + 1;
        P.nv = B.vhi - B.vlo + 1;
        P.fpart = (long long)fpart;
        off += (size_t)P.nx * P.nv;
        foff += 2 * (size_t)(P.nx + P.nv);
        fpart += (size_t)((P.nv + kMinStripCells - 1) / kMinStripCells) * P.nx;
        M->patches.push_back(P);
    }
    M->total = off;
    M->fflux = foff;

    // ---- neighbour lists: the patches (the patch itself included when its x
    // range wraps onto it) holding cells of the two-cell ghost frame of each
    // patch, x periodic; those ghost cells are copied, not interpolated
    std::vector<int> nb;
    for (size_t q = 0; q < bx.size(); ++q) {
        const Box g{bx[q].xlo - 2, bx[q].vlo - 2, bx[q].xhi + 2, bx[q].vhi + 2};
        M->patches[q].nb0 = (int)nb.size();
        for (size_t r = 0; r < bx.size(); ++r)
            for (int sh : {-M->nfx, 0, M->nfx}) {
                if (r == q && sh == 0) continue;
                const Box o{bx[r].xlo + sh, bx[r].vlo, bx[r].xhi + sh, bx[r].vhi};
                if (!intersect(g, o).empty()) {
                    nb.push_back((int)r);
                    break;
                }
            }
        M->patches[q].nb1 = (int)nb.size();
    }

    // ---- coverage of coarse cells, coarse-fine faces, corrections, restriction
    const int ncx = M->ncx, ncv = M->ncv;
    // per coarse column the velocity runs the patches cover, in increasing
    // velocity (patches are disjoint): the owner of a coarse cell
    struct Run {
        int i, j0, j1, q;
    };
    std::vector<Run> runs;
    for (size_t q = 0; q < bx.size(); ++q)
        for (int i = bx[q].xlo / R; i <= bx[q].xhi / R; ++i) runs.push_back(Run{i, bx[q].vlo / R, bx[q].vhi / R, (int)q});
    std::sort(runs.begin(), runs.end(), [](const Run& a, const Run& b) { return a.i != b.i ? a.i < b.i : a.j0 < b.j0; });
    std::vector<int> run_ptr((size_t)ncx + 1, 0);
    for (const Run& u : runs) ++run_ptr[u.i + 1];
    for (int i = 0; i < ncx; ++i) run_ptr[i + 1] += run_ptr[i];
    auto own = [&](int i, int j) {
        const int iw = ((i % ncx) + ncx) % ncx;
        for (int e = run_ptr[iw]; e < run_ptr[iw + 1]; ++e)
            if (j >= runs[e].j0 && j <= runs[e].j1) return runs[e].q;
        return -1;
    };
    // a coarse face with one covered side lies on a patch's boundary: the
    // candidates from every patch's four sides, each named by its low cell,
    // in the order of a row-major scan of the low cells (x face before v face)
    struct FaceAt {
        int i, j, dir;
    };
    std::vector<FaceAt> cand;
    for (const Box& X : bx) {
        const int cx0 = X.xlo / R, cx1 = X.xhi / R, cv0 = X.vlo / R, cv1 = X.vhi / R;
        for (int j = cv0; j <= cv1; ++j) {
            if (own(cx0 - 1, j) < 0) cand.push_back(FaceAt{((cx0 - 1) % ncx + ncx) % ncx, j, 0});
            if (own(cx1 + 1, j) < 0) cand.push_back(FaceAt{cx1, j, 0});
        }
        for (int i = cx0; i <= cx1; ++i) {
            if (cv0 > 0 && own(i, cv0 - 1) < 0) cand.push_back(FaceAt{i, cv0 - 1, 1});
            if (cv1 + 1 < ncv && own(i, cv1 + 1) < 0) cand.push_back(FaceAt{i, cv1, 1});
        }
    }
    std::sort(cand.begin(), cand.end(), [](const FaceAt& a, const FaceAt& b) {
        return a.i != b.i ? a.i < b.i : (a.j != b.j ? a.j < b.j : a.dir < b.dir);
    });
    std::vector<std::pair<int, int>> corr;           // (corrected cell, encoded face), in face order
    for (const FaceAt& c : cand) {
        const int i = c.i, j = c.j;
        const int a = own(i, j);
        if (c.dir == 0) {            // x face between (i, j) and (i + 1, j)
            const int b = own(i + 1, j);
            AmrFace F{i, j, 0, 0};
            const AmrPatch& P = M->patches[a >= 0 ? a : b];
            // covered on the high side: the patch's lower x face; else its upper x face
            F.fine = (int)(P.foff + (a < 0 ? 0 : P.nv) + (j * R - P.gv0));
            const int fi = (int)M->faces.size();
            M->faces.push_back(F);
            if (a < 0) corr.emplace_back(i * ncv + j, fi);                                    // face above cell (i, j)
            else corr.emplace_back(((i + 1) % ncx) * ncv + j, -fi - 1);                     // face below cell (i+1, j)
        } else {                     // v face between (i, j) and (i, j + 1)
            const int b = own(i, j + 1);
            AmrFace F{i, j, 1, 0};
            const AmrPatch& P = M->patches[a >= 0 ? a : b];
            F.fine = (int)(P.foff + 2 * P.nv + (a < 0 ? 0 : P.nx) + (i * R - P.gx0));
            const int fi = (int)M->faces.size();
            M->faces.push_back(F);
            if (a < 0) corr.emplace_back(i * ncv + j, fi);
            else corr.emplace_back(i * ncv + j + 1, -fi - 1);
        }
    }
    // per corrected cell (increasing), its faces in face order
    std::stable_sort(corr.begin(), corr.end(),
                     [](const std::pair<int, int>& x, const std::pair<int, int>& y) { return x.first < y.first; });
    std::vector<int> corr_ptr{0}, corr_face, corr_cell;
    for (size_t e = 0; e < corr.size(); ++e) {
        if (e == 0 || corr[e].first != corr[e - 1].first) {
            if (e > 0) corr_ptr.push_back((int)corr_face.size());
            corr_cell.push_back(corr[e].first);
        }
        corr_face.push_back(corr[e].second);
    }
    if (!corr.empty()) corr_ptr.push_back((int)corr_face.size());
    M->ncorr = (int)corr_cell.size();
    // covered coarse cells in row-major order
    std::vector<int> cov_cell, cov_nv;
    std::vector<long long> cov_fine;
    for (const Run& u : runs) {
        const AmrPatch& P = M->patches[u.q];
        for (int j = u.j0; j <= u.j1; ++j) {
            cov_cell.push_back(u.i * ncv + j);
            cov_fine.push_back(P.off + (long long)(u.i * R - P.gx0) * P.nv + (j * R - P.gv0));
            cov_nv.push_back(P.nv);
        }
    }
    M->ncov = (int)cov_cell.size();
    // the patches over each fine configuration column, in patch order
    M->fcol_ptr.assign((size_t)M->nfx + 1, 0);
    for (const AmrPatch& P : M->patches)
        for (int I = P.gx0; I < P.gx0 + P.nx; ++I) ++M->fcol_ptr[I + 1];
    for (int I = 0; I < M->nfx; ++I) M->fcol_ptr[I + 1] += M->fcol_ptr[I];
    M->fcol_patch.assign(M->fcol_ptr.back(), 0);
    {
        std::vector<int> at(M->fcol_ptr.begin(), M->fcol_ptr.end() - 1);
        for (size_t q = 0; q < M->patches.size(); ++q)
            for (int I = M->patches[q].gx0; I < M->patches[q].gx0 + M->patches[q].nx; ++I) M->fcol_patch[at[I]++] = (int)q;
    }

    // ---- Sub-Patch reduction: Alg. subdiv on the coarse level, then the
    // row-sum tasks (each sub-patch grown by two columns in x) and the
    // fixed-order contribution list of every fine configuration cell
    std::vector<Box> S{Box{0, 0, ncx - 1, ncv - 1}};
    for (const Box& B : bx) {
        const Box P{B.xlo / R, B.vlo / R, B.xhi / R, B.vhi / R};
        const Box ext{P.xlo, 0, P.xhi, ncv - 1};
        std::vector<Box> S2;
        for (const Box& s : S) {
            const Box in = intersect(s, ext);
            if (in.empty()) { S2.push_back(s); continue; }
            if (s.xlo < in.xlo) S2.push_back(Box{s.xlo, s.vlo, in.xlo - 1, s.vhi});
            if (in.xhi < s.xhi) S2.push_back(Box{in.xhi + 1, s.vlo, s.xhi, s.vhi});
            const Box below{in.xlo, in.vlo, in.xhi, std::min(in.vhi, P.vlo - 1)};
            const Box above{in.xlo, std::max(in.vlo, P.vhi + 1), in.xhi, in.vhi};
            if (!below.empty()) S2.push_back(below);
            if (!above.empty()) S2.push_back(above);
        }
        S.swap(S2);
    }
    M->nsub = (int)S.size();
    std::vector<long long> task_off;
    std::vector<int> task_len, sub_base, fine_base;
    for (const Box& s : S) {
        sub_base.push_back((int)task_off.size());
        for (int i = s.xlo - 2; i <= s.xhi + 2; ++i) {
            task_off.push_back((long long)(((i % ncx) + ncx) % ncx) * ncv + s.vlo);
            task_len.push_back(s.vhi - s.vlo + 1);
        }
    }
    for (const AmrPatch& P : M->patches) {
        fine_base.push_back((int)task_off.size());
        for (int r = 0; r < P.nx; ++r) {
            task_off.push_back(P.off + (long long)r * P.nv);
            task_len.push_back(P.nv);
        }
    }
    M->ntasks = (int)task_off.size();
    M->fine_task0 = fine_base.empty() ? M->ntasks : fine_base[0];
    const std::vector<double> B = interp_table(R);
    // the sub-patches over each coarse column, in sub-patch order
    std::vector<int> scol_ptr((size_t)ncx + 1, 0), scol;
    for (const Box& b : S)
        for (int i = b.xlo; i <= b.xhi; ++i) ++scol_ptr[i + 1];
    for (int i = 0; i < ncx; ++i) scol_ptr[i + 1] += scol_ptr[i];
    scol.resize(scol_ptr.back());
    {
        std::vector<int> at(scol_ptr.begin(), scol_ptr.end() - 1);
        for (size_t q = 0; q < S.size(); ++q)
            for (int i = S[q].xlo; i <= S[q].xhi; ++i) scol[at[i]++] = (int)q;
    }
    std::vector<int> rowptr{0}, idx;
    std::vector<double> w;
    for (int I = 0; I < M->nfx; ++I) {
        const int i = I / R, s = I % R;
        for (int e = scol_ptr[i]; e < scol_ptr[i + 1]; ++e) {
            const int q = scol[e];
            for (int a = -2; a <= 2; ++a) {
                idx.push_back(sub_base[q] + (i + a - (S[q].xlo - 2)));
                w.push_back(B[s * 5 + a + 2] * M->dvc);
            }
        }
        for (int e = M->fcol_ptr[I]; e < M->fcol_ptr[I + 1]; ++e) {
            const int q = M->fcol_patch[e];
            idx.push_back(fine_base[q] + (I - M->patches[q].gx0));
            w.push_back(M->dvf);
        }
        rowptr.push_back((int)idx.size());
    }

    // ---- Mask reduction lists: the masked, x-refined coarse sums S[i][a] and the fine row sums
    std::vector<unsigned char> mask((size_t)ncx * ncv, 0);
    for (const Run& u : runs) std::fill_n(mask.begin() + (size_t)u.i * ncv + u.j0, u.j1 - u.j0 + 1, 1);
    std::vector<int> rowptr_m{0}, idx_m;
    std::vector<double> w_m;
    for (int I = 0; I < M->nfx; ++I) {
        const int i = I / R, s = I % R;
        for (int a = -2; a <= 2; ++a) {
            idx_m.push_back(i * 5 + a + 2);
            w_m.push_back(B[s * 5 + a + 2] * M->dvc);
        }
        for (int e = M->fcol_ptr[I]; e < M->fcol_ptr[I + 1]; ++e) {
            const int q = M->fcol_patch[e];
            idx_m.push_back(5 * ncx + (fine_base[q] - M->fine_task0) + (I - M->patches[q].gx0));
            w_m.push_back(M->dvf);
        }
        rowptr_m.push_back((int)idx_m.size());
    }

    // ---- the Mask reduction from strip partials: each coarse column's
    // covered cells
    std::vector<int> covc_ptr((size_t)ncx + 1, 0), covc_j;
    for (const Run& u : runs) {
        for (int j = u.j0; j <= u.j1; ++j) covc_j.push_back(j);
        covc_ptr[u.i + 1] = (int)covc_j.size();
    }
    for (int i = 0; i < ncx; ++i) covc_ptr[i + 1] = std::max(covc_ptr[i + 1], covc_ptr[i]);

    // ---- device tables
    M->w = (M->ncv % 2 == 0 && std::all_of(M->patches.begin(), M->patches.end(),
                                           [](const AmrPatch& P) { return P.nv % 2 == 0; })) ? 2 : 1;
    M->nt = 64;
    M->tx = 8;
    build_tiles(*M);
    VP_HIP(upload_tiles(*M));
    VP_HIP(upload_fused_lists(*M));
    TableArena T;
    T.add(&M->d_patches, M->patches);
    T.add(&M->d_faces, M->faces);
    T.add(&M->d_nb, nb);
    T.add(&M->d_B, B);
    T.add(&M->d_task_off, task_off);
    T.add(&M->d_task_len, task_len);
    T.add(&M->d_rowptr, rowptr);
    T.add(&M->d_idx, idx);
    T.add(&M->d_w, w);
    T.add(&M->d_corr_ptr, corr_ptr);
    T.add(&M->d_corr_face, corr_face);
    T.add(&M->d_corr_cell, corr_cell);
    T.add(&M->d_cov_cell, cov_cell);
    T.add(&M->d_cov_fine, cov_fine);
    T.add(&M->d_cov_nv, cov_nv);
    T.add(&M->d_mask, mask);
    T.add(&M->d_rowptr_m, rowptr_m);
    T.add(&M->d_idx_m, idx_m);
    T.add(&M->d_w_m, w_m);
    T.add(&M->d_covc_ptr, covc_ptr);
    T.add(&M->d_covc_j, covc_j);
    const std::vector<double> green_c = poisson_green_table(ncx);     // add() keeps a pointer until commit()
    T.add(&M->d_green_c, green_c);
    VP_HIP(T.commit(&M->d_tables));

    // ---- workspace: acc, two predictors, accumulated face fluxes, reduction slots, n, E
    const size_t sb = align256(M->total * sizeof(double));
    size_t o = 0;
    p->ws_acc = o; o += sb;
    p->ws_fsa = o; o += sb;
    p->ws_fsb = o; o += sb;
    M->ws_cf = o; o += align256(std::max<size_t>(M->faces.size(), 1) * sizeof(double));
    M->ws_ff = o; o += align256(std::max<size_t>(M->fflux, 1) * sizeof(double));
    M->ws_slots = o; o += align256(std::max(M->ntasks, 1) * sizeof(double));
    M->ws_slots_m = o; o += align256((size_t)(5 * ncx + (M->ntasks - M->fine_task0)) * sizeof(double));
    M->ws_pc = o; o += align256((size_t)((ncv + kMinStripCells - 1) / kMinStripCells) * ncx * sizeof(double));
    M->ws_pf = o; o += align256(std::max<size_t>(fpart, 1) * sizeof(double));
    M->ws_n = o; o += align256((size_t)M->nfx * sizeof(double));
    M->ws_E = o; o += align256((size_t)M->nfx * sizeof(double));
    M->ws_fld = o; o += align256(((size_t)M->nfx + 4 * ((size_t)M->nfx / kFieldChunk + 1) + 64) * sizeof(double));
    M->hist_stride = align256((size_t)ncx * ncv * sizeof(double)) / sizeof(double);
    M->ws_hist = o; o += 5 * M->hist_stride * sizeof(double);
    M->ws_nc = o; o += align256((size_t)ncx * sizeof(double));
    p->ws_total = o;
    p->state_elems = M->total;
    return VP_OK;
}

void amr_destroy(vp_plan* p)
{
    AmrPlan* M = p->amr;
    if (!M) return;
    if (M->d_tables) (void)hipFree(M->d_tables);
    if (M->d_tiles) (void)hipFree(M->d_tiles);
    if (M->d_fz) (void)hipFree(M->d_fz);
    delete M;
    p->amr = nullptr;
}

vp_status amr_rhs(const vp_plan* p, const void* f, const double* a, void* k, hipStream_t stream)
{
    AmrArgs A = stage_args(p, f, nullptr, nullptr, k, a, 0.0, 0.0, 0.0, 0, nullptr);
    VP_HIP(timed(p, kTStage, stream, [&] { return launch_stage_all(p, kRhs, A, stream); }));
    return VP_OK;
}

vp_status amr_reduce(const vp_plan* p, const void* f, double* n, void* work, hipStream_t stream, bool partials)
{
    const AmrPlan& M = *p->amr;
    const double* fd = static_cast<const double*>(f);
    VP_HIP(timed(p, kTMoment, stream, [&] {
        return partials ? reduce_fused_launch(M, fd, n, work, stream) : reduce_launch(M, fd, n, work, stream);
    }));
    return VP_OK;
}

bool amr_stage_partials(const vp_plan* p, int s) { return s < 3 && p->amr->reduce_mode == VP_REDUCE_FUSED; }

vp_status amr_inject(const vp_plan* p, const double* E, double* a, hipStream_t stream)
{
    const AmrPlan& M = *p->amr;
    VP_HIP(timed(p, kTOther, stream, [&] { return launch_amr_inject(E, M.ncx, M.R, p->pb.qm, a, stream); }));
    return VP_OK;
}

void* amr_stage_output(const vp_plan* p, int s, void* f, void* work)
{
    void* out[4] = {wsp(work, p->ws_fsa), wsp(work, p->ws_fsb), wsp(work, p->ws_fsa), f};
    return out[s];
}

vp_status amr_stage(const vp_plan* p, int s, void* f, const double* a, double dt, void* work, hipStream_t stream,
                    bool partials)
{
    void* acc = wsp(work, p->ws_acc);
    const void* in[4] = {f, amr_stage_output(p, 0, f, work), amr_stage_output(p, 1, f, work),
                         amr_stage_output(p, 2, f, work)};
    const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const double cnext[3] = {0.5 * dt, 0.5 * dt, dt};
    const int kind = s == 0 ? kStage1 : (s == 3 ? kStage4 : kStage23);
    AmrArgs A = stage_args(p, in[s], f, acc, amr_stage_output(p, s, f, work), a, dt * b[s], s < 3 ? cnext[s] : 0.0,
                           b[s], s == 0, work);
    if (partials) {
        const AmrPlan& M = *p->amr;
        A.coarse.part = reinterpret_cast<double*>(wsp(work, M.ws_pc));
        A.fpart = reinterpret_cast<double*>(wsp(work, M.ws_pf));
    }
    VP_HIP(timed(p, kTStage, stream, [&] { return launch_stage_all(p, kind, A, stream); }));
    return VP_OK;
}

vp_status amr_rk4(const vp_plan* p, void* f, double* a, double dt, void* work, hipStream_t stream)
{
    for (int s = 0; s < 4; ++s) {
        const bool partials = amr_stage_partials(p, s);
        if (vp_status st = amr_stage(p, s, f, a, dt, work, stream, partials)) return st;
        if (s < 3)
            if (vp_status st = constraint(p, static_cast<const double*>(amr_stage_output(p, s, f, work)), a, work,
                                          stream, partials))
                return st;
    }
    if (vp_status st = amr_end_sync(p, f, dt, work, stream)) return st;
    return constraint(p, static_cast<const double*>(f), a, work, stream);
}

vp_status amr_end_sync(const vp_plan* p, void* f, double dt, void* work, hipStream_t stream)
{
    const AmrPlan& M = *p->amr;
    AmrSyncArgs S{};
    S.f = static_cast<double*>(f);
    S.ncv = M.ncv;
    S.R = M.R;
    S.cf_acc = reinterpret_cast<const double*>(wsp(work, M.ws_cf));
    S.ff_acc = reinterpret_cast<const double*>(wsp(work, M.ws_ff));
    S.faces = M.d_faces;
    S.corr_ptr = M.d_corr_ptr;
    S.corr_face = M.d_corr_face;
    S.corr_cell = M.d_corr_cell;
    S.ncorr = M.ncorr;
    S.cov_cell = M.d_cov_cell;
    S.cov_fine = M.d_cov_fine;
    S.cov_nv = M.d_cov_nv;
    S.ncov = M.ncov;
    S.dtx = dt / M.dxc;
    S.dtv = dt / M.dvc;
    VP_HIP(timed(p, kTSync, stream, [&] { return launch_amr_sync(S, stream); }));
    return VP_OK;
}

// Substep weights: the coarse data of fine stage s of the substep
// [theta0, theta0 + eta] (units of the coarse step) are f^n + dt sum_q w_q K_q.
// They are the classical RK4 stage values taken on the Taylor expansion at
// theta0 of the continuous extension P(theta) = f^n + dt sum_q b_q(theta) K_q
// of the coarse step, b_1 = theta - 3/2 theta^2 + 2/3 theta^3,
// b_2 = b_3 = theta^2 - 2/3 theta^3, b_4 = -1/2 theta^2 + 2/3 theta^3
// (asynchronous stepping, future work of section 5, after McCorquodale and
// Colella).  With P(theta0 + x) = d0 + d1 x + d2 x^2 + d3 x^3 the four stage
// values are d0; d0 + eta/2 d1; d0 + eta/2 d1 + eta^2/2 d2;
// d0 + eta d1 + eta^2 d2 + 3/2 eta^3 d3.
static void substage_weights(double theta0, double eta, int s, double w[4])
{
    // b_q(theta) = sum_j p[q][j] theta^j
    static const double p[4][4] = {{0.0, 1.0, -1.5, 2.0 / 3.0},
                                   {0.0, 0.0, 1.0, -2.0 / 3.0},
                                   {0.0, 0.0, 1.0, -2.0 / 3.0},
                                   {0.0, 0.0, -0.5, 2.0 / 3.0}};
    // stage s: coefficient of eta^k d_k
    static const double g[4][4] = {{1.0, 0.0, 0.0, 0.0},
                                   {1.0, 0.5, 0.0, 0.0},
                                   {1.0, 0.5, 0.5, 0.0},
                                   {1.0, 1.0, 1.0, 1.5}};
    static const double binom[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
    for (int q = 0; q < 4; ++q) {
        double sum = 0.0, e = 1.0;
        for (int k = 0; k < 4; ++k) {
            double dk = 0.0;             // Taylor coefficient k of b_q at theta0
            for (int j = 3; j >= k; --j) dk = dk * theta0 + p[q][j] * binom[j][k];
            sum += g[s][k] * e * dk;
            e *= eta;
        }
        w[q] = sum;
    }
}

vp_status amr_subcycle(const vp_plan* p, void* f, double* a, double dt, void* work, hipStream_t stream)
{
    const AmrPlan& M = *p->amr;
    const size_t nc = (size_t)M.ncx * M.ncv;
    double* hist = reinterpret_cast<double*>(wsp(work, M.ws_hist));
    double* H[5];
    for (int q = 0; q < 5; ++q) H[q] = hist + q * M.hist_stride;
    double* nmom = reinterpret_cast<double*>(wsp(work, M.ws_nc));
    void* acc = wsp(work, p->ws_acc);
    const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const double cnext[4] = {0.5, 0.5, 1.0, 0.0};
    const int kinds[4] = {kStage1, kStage23, kStage23, kStage4};
    const int cap = 256 * 8;
    auto range = [&](int kind, const AmrArgs& A, int t0, int t1) {
        return launch_amr_stage(M.w, M.nt, kind, A, t0, t1, std::min(std::max(t1 - t0, 1), cap), stream);
    };

    // 1. the coarse level: one RK4 step of dt with the field of its own
    // moment on the coarse configuration mesh; its stage states go to H[1..4]
    VP_HIP(hipMemcpyAsync(H[0], f, nc * sizeof(double), hipMemcpyDeviceToDevice, stream));
    for (int s = 0; s < 4; ++s) {
        const void* in = s == 0 ? f : static_cast<const void*>(H[s]);
        VP_HIP(timed(p, kTMoment, stream, [&] {
            return launch_moment_rows(VP_F64, in, M.ncx, M.ncv, M.dvc, nmom, stream);
        }));
        VP_HIP(timed(p, kTField, stream, [&] {
            return launch_poisson1d(nullptr, 0, nmom, 1.0, M.ncx, M.dxc, p->pb.qm, M.d_green_c, p->gk, nullptr,
                                    nullptr, nullptr, a, stream);
        }));
        AmrArgs A = stage_args(p, in, f, acc, H[s + 1], a, dt * b[s], dt * cnext[s], b[s], s == 0, work);
        VP_HIP(timed(p, kTStage, stream, [&] {
            hipError_t e = range(kinds[s], A, 0, M.ncoarse_tiles);
            return e == hipSuccess ? range(kinds[s], A, M.face_tile_begin, M.ntiles) : e;
        }));
    }

    // 2. the patches: R substeps of dt / R; the coarse part of each stage
    // input holds that stage's coarse data
    const double h = dt / M.R, eta = 1.0 / M.R;
    for (int m = 0; m < M.R; ++m)
        for (int s = 0; s < 4; ++s) {
            void* in = s == 0 ? f : amr_stage_output(p, s - 1, f, work);
            void* out = amr_stage_output(p, s, f, work);
            double w[4];
            substage_weights(m * eta, eta, s, w);
            // in terms of the stored states: dt K_1 = 2 (H1 - H0), dt K_2 = 2 (H2 - H0),
            // dt K_3 = H3 - H0, dt K_4 = 6 (H4 - H0) - 2 (H1 - H0) - 4 (H2 - H0) - 2 (H3 - H0)
            const double c[4] = {2.0 * w[0] - 2.0 * w[3], 2.0 * w[1] - 4.0 * w[3], w[2] - 2.0 * w[3], 6.0 * w[3]};
            VP_HIP(timed(p, kTOther, stream, [&] {
                return launch_amr_substage(H[0], nc, M.hist_stride, c, static_cast<double*>(in), stream);
            }));
            if (vp_status st = constraint(p, static_cast<const double*>(in), a, work, stream)) return st;
            AmrArgs A = stage_args(p, in, f, acc, out, a, h * b[s], h * cnext[s], b[s] / M.R, m == 0 && s == 0, work);
            VP_HIP(timed(p, kTStage, stream, [&] { return range(kinds[s], A, M.ncoarse_tiles, M.face_tile_begin); }));
        }

    // 3. the coarse level's end state, the fine fluxes on coarse-fine faces
    // (averaged over the substeps), the average-down, and the field
    VP_HIP(hipMemcpyAsync(f, H[4], nc * sizeof(double), hipMemcpyDeviceToDevice, stream));
    if (vp_status st = amr_end_sync(p, f, dt, work, stream)) return st;
    return constraint(p, static_cast<const double*>(f), a, work, stream);
}

}  // namespace vp
