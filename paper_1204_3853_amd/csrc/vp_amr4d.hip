// Host runtime of the two-level 2D+2V path (the AMR of section 3 carried to
// the 2D+2V phase space): box validation, padded copies and their
// neighbour lists, the stage tile table, the coarse-fine faces of level 0
// with their fine faces, the Mask reduction lists onto the fine 2D
// configuration mesh (Alg. mreduce: masked coarse plane sums refined in x
// and y, patch plane sums), the Fourier tables of the fine configuration
// mesh, the average-down lists, and the enqueue sequence of one synchronous
// RK4 step (Alg. smsvphu without regridding).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "vp_internal.hpp"

namespace vp {

namespace {

int w4(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }
size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
char* wp(void* work, size_t off) { return static_cast<char*>(work) + off; }

A4Args base_args(const vp_plan* p, const double* pad, const double* a)
{
    const Amr4DPlan& M = *p->a4;
    A4Args A{};
    A.lv[0] = M.lv[0];
    A.lv[1] = M.lv[1];
    A.patches = M.d_patches;
    A.nb = M.d_nb;
    A.tiles = M.d_tiles;
    A.ntiles = M.ntiles;
    A.pad = pad;
    A.a = a;
    return A;
}

vp_status pad_launch(const vp_plan* p, const double* f, double* pad, double* scratch, hipStream_t stream)
{
    const Amr4DPlan& M = *p->a4;
    VP_HIP(timed(p, kTOther, stream, [&] {
        return launch_a4_pad(f, M.d_patches, M.d_list, (int)M.patches.size(), (long long)M.pad_total, M.d_nb, M.lv,
                             M.d_B, M.R, M.d_gxc, M.d_gyc, M.d_gxf, M.d_gyf, M.d_interp, M.ptiles, scratch, pad, stream);
    }));
    return VP_OK;
}

vp_status moment(const vp_plan* p, const double* f, double* n, void* work, hipStream_t stream)
{
    const Amr4DPlan& M = *p->a4;
    double* slots = reinterpret_cast<double*>(wp(work, M.ws_slots));
    VP_HIP(timed(p, kTMoment, stream, [&] {
        hipError_t e = launch_a4_moment_sums(f, M.d_rect_ptr, M.d_rects, M.nc, M.d_task_off, M.d_task_len, M.ntasks,
                                             slots, stream);
        if (e == hipSuccess) e = launch_amr_reduce_finalize(slots, M.d_rowptr, M.d_idx, M.d_w, M.ncfg, n, stream);
        return e;
    }));
    return VP_OK;
}

// moment -> 2D Poisson on the fine configuration mesh -> a on both levels
vp_status constraint(const vp_plan* p, const double* f, double* a, void* work, hipStream_t stream)
{
    const Amr4DPlan& M = *p->a4;
    double* n = reinterpret_cast<double*>(wp(work, M.ws_n));
    double* g = reinterpret_cast<double*>(wp(work, M.ws_g));
    if (vp_status st = moment(p, f, n, work, stream)) return st;
    const int nc = M.nc[0] * M.nc[1];
    VP_HIP(timed(p, kTField, stream, [&] {
        // small fine meshes: the inverse transform also forms the coarse a
        if (M.nf[0] <= kPoisson2DSmall && M.nf[1] <= kPoisson2DSmall)
            return launch_poisson2d_coarse(n, M.nf[0], M.nf[1], M.lv[1].h[0], M.lv[1].h[1], p->pb.qm, M.d_Qx, M.d_Qy,
                                           M.d_inv, g, nullptr, nullptr, a + 2 * nc, M.R, a, stream);
        hipError_t e = launch_poisson2d(n, M.nf[0], M.nf[1], M.lv[1].h[0], M.lv[1].h[1], p->pb.qm, M.d_Qx, M.d_Qy,
                                        M.d_inv, g, nullptr, nullptr, a + 2 * nc, stream);
        if (e == hipSuccess) e = launch_a4_inject(a, M.nc[0], M.nc[1], M.R, stream);
        return e;
    }));
    return VP_OK;
}

}  // namespace

vp_status a4_create(vp_plan* p, const vp_problem* pb, const vp_box* boxes, int nbox)
{
    if (pb->dtype != VP_F64) return fail(VP_ENOTSUP, "two-level 2D+2V is supported in FP64");
    const int R = pb->ratio[0][0];
    if ((R != 2 && R != 4) || pb->ratio[0][1] != R || pb->ratio[0][2] != R || pb->ratio[0][3] != R)
        return fail(VP_ENOTSUP, "two-level 2D+2V needs one refinement ratio, 2 or 4, in every direction");
    if (pb->v_lo[0] != pb->v_lo[1] || pb->v_hi[0] != pb->v_hi[1])
        return fail(VP_ENOTSUP, "2D+2V needs the same velocity interval in vx and vy");
    for (int l = 0; l < 2; ++l)
        for (int d = 0; d < 2; ++d)
            if (!pb->veq[l][d]) return fail(VP_EINVAL, "veq[l][d] (equilibria with ghosts) are required on both levels");
    Amr4DPlan* Mp = new Amr4DPlan();
    p->a4 = Mp;
    Amr4DPlan& M = *Mp;
    M.R = R;
    for (int d = 0; d < 4; ++d) {
        M.nc[d] = pb->cells[d];
        M.nf[d] = pb->cells[d] * R;
    }
    if (M.nf[0] > kMaxPoisson2D || M.nf[1] > kMaxPoisson2D)
        return fail(VP_ENOTSUP, "two-level 2D+2V: the fine configuration mesh is limited to 256 x 256 cells");
    const double len[4] = {pb->x_len[0], pb->x_len[1], pb->v_hi[0] - pb->v_lo[0], pb->v_hi[1] - pb->v_lo[1]};
    for (int l = 0; l < 2; ++l) {
        A4Level& L = M.lv[l];
        for (int d = 0; d < 4; ++d) {
            L.n[d] = l == 0 ? M.nc[d] : M.nf[d];
            L.h[d] = len[d] / L.n[d];
            L.hi[d] = 1.0 / L.h[d];
        }
        L.v_lo = pb->v_lo[0];
        L.a_off = l == 0 ? 0 : 2 * M.nc[0] * M.nc[1];
    }

    // ---- patches: level 0, then the boxes (level 1, aligned, inside, disjoint)
    std::vector<A4Patch>& P = M.patches;
    {
        A4Patch q{};
        for (int d = 0; d < 4; ++d) q.sz[d] = M.nc[d];
        q.lev = 0;
        P.push_back(q);
    }
    for (int k = 0; k < nbox; ++k) {
        const vp_box& b = boxes[k];
        if (b.level != 1) return fail(VP_EINVAL, "two-level 2D+2V: boxes must be on level 1");
        A4Patch q{};
        q.lev = 1;
        for (int d = 0; d < 4; ++d) {
            q.lo[d] = b.lo[d];
            q.sz[d] = b.hi[d] - b.lo[d] + 1;
            if (q.sz[d] < 1 || b.lo[d] < 0 || b.hi[d] >= M.nf[d])
                return fail(VP_EINVAL, "box " + std::to_string(k) + " is empty or outside the level-1 domain");
            if (b.lo[d] % R || (b.hi[d] + 1) % R)
                return fail(VP_EINVAL, "box " + std::to_string(k) + " is not aligned to the refinement ratio");
        }
        for (size_t r = 1; r < P.size(); ++r) {
            bool meet = true;
            for (int d = 0; d < 4; ++d)
                meet = meet && std::max(q.lo[d], P[r].lo[d]) <= std::min(q.lo[d] + q.sz[d], P[r].lo[d] + P[r].sz[d]) - 1;
            if (meet) return fail(VP_EINVAL, "boxes " + std::to_string(r - 1) + " and " + std::to_string(k) + " overlap");
        }
        P.push_back(q);
    }
    size_t off = 0, pad = 0, foff = 0;
    for (A4Patch& q : P) {
        for (int d = 0; d < 4; ++d) {
            q.isz[d] = 1.0 / q.sz[d];
            q.ipz[d] = 1.0 / (q.sz[d] + 4);
        }
        const long long n0 = q.sz[0], n1 = q.sz[1], n2 = q.sz[2], n3 = q.sz[3];
        q.off = (long long)off;
        q.pad = (long long)pad;
        q.foff = (long long)foff;
        off += (size_t)(n0 * n1 * n2 * n3);
        pad += (size_t)((n0 + 4) * (n1 + 4) * (n2 + 4) * (n3 + 4));
        if (q.lev == 1) foff += (size_t)(2 * (n1 * n2 * n3 + n0 * n2 * n3 + n0 * n1 * n3 + n0 * n1 * n2));
    }
    M.total = off;
    M.pad_total = pad;
    M.fflux = foff;

    // ---- neighbour lists of level-1 patches: patches holding cells of the two-deep frame (x, y periodic)
    std::vector<int> nb;
    for (size_t q = 1; q < P.size(); ++q) {
        P[q].nb0 = (int)nb.size();
        for (size_t r = 1; r < P.size(); ++r) {
            bool found = false;
            for (int sx = -1; sx <= 1 && !found; ++sx)
                for (int sy = -1; sy <= 1 && !found; ++sy) {
                    if (r == q && sx == 0 && sy == 0) continue;
                    const int sh[4] = {sx * M.nf[0], sy * M.nf[1], 0, 0};
                    bool meet = true;
                    for (int d = 0; d < 4; ++d)
                        meet = meet && std::max(P[q].lo[d] - 2, P[r].lo[d] + sh[d]) <=
                                           std::min(P[q].lo[d] + P[q].sz[d] + 1, P[r].lo[d] + sh[d] + P[r].sz[d] - 1);
                    found = meet;
                }
            if (found) nb.push_back((int)r);
        }
        P[q].nb1 = (int)nb.size();
    }
    std::vector<int> list(P.size());
    for (size_t q = 0; q < P.size(); ++q) list[q] = (int)q;

    for (const A4Patch& q : P)     // kernels index a patch's cells, and its padded copy, in 32 bits
        if ((long long)(q.sz[0] + 4) * (q.sz[1] + 4) * (q.sz[2] + 4) * (q.sz[3] + 4) >= (1LL << 31))
            return fail(VP_ENOTSUP, "two-level 2D+2V: a patch (or level 0) of 2^31 cells or more");
    // ---- stage tiles: 256 threads of one patch each (a thread per run of
    // kA4VxRun cells along vx)
    std::vector<int> tiles;
    for (size_t q = 0; q < P.size(); ++q) {
        const long long n = (long long)P[q].sz[0] * P[q].sz[1] * ((P[q].sz[2] + kA4VxRun - 1) / kA4VxRun) * P[q].sz[3];
        for (long long c = 0; c < n; c += 256) {
            tiles.push_back((int)q);
            tiles.push_back((int)c);
        }
    }
    M.ntiles = (int)(tiles.size() / 2);

    // ---- coverage of level-0 cells
    const int* n = M.nc;
    const long long ncells0 = (long long)n[0] * n[1] * n[2] * n[3];
    std::vector<int> own((size_t)ncells0, -1);
    auto cidx = [&](int i, int j, int k, int l) {
        return (((long long)w4(i, n[0]) * n[1] + w4(j, n[1])) * n[2] + k) * n[3] + l;
    };
    for (size_t q = 1; q < P.size(); ++q)
        for (int i = P[q].lo[0] / R; i < (P[q].lo[0] + P[q].sz[0]) / R; ++i)
            for (int j = P[q].lo[1] / R; j < (P[q].lo[1] + P[q].sz[1]) / R; ++j)
                for (int k = P[q].lo[2] / R; k < (P[q].lo[2] + P[q].sz[2]) / R; ++k)
                    for (int l = P[q].lo[3] / R; l < (P[q].lo[3] + P[q].sz[3]) / R; ++l) own[cidx(i, j, k, l)] = (int)q;
    // per level-0 configuration column, the velocity rectangles level 1 covers in it
    std::vector<int> rect_ptr{0};
    std::vector<int4> rects;
    for (int i = 0; i < n[0]; ++i)
        for (int j = 0; j < n[1]; ++j) {
            for (size_t q = 1; q < P.size(); ++q) {
                const A4Patch& G = P[q];
                if (i < G.lo[0] / R || i >= (G.lo[0] + G.sz[0]) / R || j < G.lo[1] / R || j >= (G.lo[1] + G.sz[1]) / R)
                    continue;
                rects.push_back(make_int4(G.lo[2] / R, (G.lo[2] + G.sz[2]) / R - 1, G.lo[3] / R,
                                          (G.lo[3] + G.sz[3]) / R - 1));
            }
            rect_ptr.push_back((int)rects.size());
        }

    // ---- coarse-fine faces of level 0: every side of every patch, where the
    // level-0 cell outside is not covered (velocity sides inside the box only)
    std::vector<A4Face> faces;
    std::vector<int> fine;
    std::map<long long, std::vector<int>> corr;
    for (size_t q = 1; q < P.size(); ++q) {
        const A4Patch& G = P[q];
        int c0[4], c1[4];
        for (int d = 0; d < 4; ++d) {
            c0[d] = G.lo[d] / R;
            c1[d] = (G.lo[d] + G.sz[d]) / R - 1;
        }
        const long long n0 = G.sz[0], n1 = G.sz[1], n2 = G.sz[2], n3 = G.sz[3];
        const long long S[4] = {n1 * n2 * n3, n0 * n2 * n3, n0 * n1 * n3, n0 * n1 * n2};
        long long blk[4];
        blk[0] = 0;
        for (int d = 1; d < 4; ++d) blk[d] = blk[d - 1] + 2 * S[d - 1];
        for (int d = 0; d < 4; ++d)
            for (int side = 0; side < 2; ++side) {
                const int out = side == 0 ? c0[d] - 1 : c1[d] + 1;
                if (d >= 2 && (out < 0 || out >= n[d])) continue;          // the velocity boundary
                // transverse coarse cells of the side
                int t[3], tlo[3], thi[3], m = 0;
                for (int e = 0; e < 4; ++e)
                    if (e != d) { t[m] = e; tlo[m] = c0[e]; thi[m] = c1[e]; ++m; }
                for (int u0 = tlo[0]; u0 <= thi[0]; ++u0)
                    for (int u1 = tlo[1]; u1 <= thi[1]; ++u1)
                        for (int u2 = tlo[2]; u2 <= thi[2]; ++u2) {
                            int cc[4];
                            cc[t[0]] = u0; cc[t[1]] = u1; cc[t[2]] = u2;
                            cc[d] = out;
                            if (own[cidx(cc[0], cc[1], cc[2], cc[3])] >= 0) continue;     // both sides covered
                            A4Face F{};
                            F.dir = d;
                            for (int e = 0; e < 4; ++e) F.cell[e] = e < 2 ? w4(cc[e], n[e]) : cc[e];
                            if (side == 1) F.cell[d] = w4(c1[d], n[d]);          // low cell: the covered one
                            const int fi = (int)faces.size();
                            faces.push_back(F);
                            // the R^3 fine faces: G's lower (side 0) or upper face along d
                            const long long base = G.foff + blk[d] + side * S[d];
                            int fl[4];
                            for (int a0 = 0; a0 < R; ++a0)
                                for (int a1 = 0; a1 < R; ++a1)
                                    for (int a2 = 0; a2 < R; ++a2) {
                                        fl[t[0]] = u0 * R + a0 - G.lo[t[0]];
                                        fl[t[1]] = u1 * R + a1 - G.lo[t[1]];
                                        fl[t[2]] = u2 * R + a2 - G.lo[t[2]];
                                        // the block of direction d is indexed by the other three in order
                                        long long idx = 0;
                                        for (int e = 0; e < 4; ++e)
                                            if (e != d) idx = idx * G.sz[e] + fl[e];
                                        fine.push_back((int)(base + idx));
                                    }
                            // the uncovered cell: below the face (side 0, the face is its upper face)
                            // or above it (side 1, its lower face)
                            corr[cidx(cc[0], cc[1], cc[2], cc[3])].push_back(side == 0 ? fi : -fi - 1);
                        }
            }
    }
    M.nfaces = (int)faces.size();
    std::vector<long long> corr_cell;
    std::vector<int> corr_ptr{0}, corr_code;
    for (const auto& kv : corr) {
        corr_cell.push_back(kv.first);
        for (int e : kv.second) corr_code.push_back(e);
        corr_ptr.push_back((int)corr_code.size());
    }
    M.ncorr = (int)corr_cell.size();

    // ---- Mask reduction lists: slots [masked coarse plane sums (25 per
    // coarse configuration cell)][patch plane sums]
    const std::vector<double> B = interp_table(R);
    const int ncx = n[0], ncy = n[1], nfx = M.nf[0], nfy = M.nf[1];
    const double dvc = M.lv[0].h[2] * M.lv[0].h[3], dvf = M.lv[1].h[2] * M.lv[1].h[3];
    std::vector<long long> task_off;
    std::vector<int> task_len;
    std::vector<int> task_base(P.size(), 0);
    for (size_t q = 1; q < P.size(); ++q) {
        task_base[q] = (int)task_off.size();
        const long long plane = (long long)P[q].sz[2] * P[q].sz[3];
        for (int i = 0; i < P[q].sz[0]; ++i)
            for (int j = 0; j < P[q].sz[1]; ++j) {
                task_off.push_back(P[q].off + ((long long)i * P[q].sz[1] + j) * plane);
                task_len.push_back((int)plane);
            }
    }
    M.ntasks = (int)task_off.size();
    M.ncfg = nfx * nfy;
    const int m0 = 25 * ncx * ncy;
    std::vector<int> rowptr{0}, idx;
    std::vector<double> wts;
    for (int I = 0; I < nfx; ++I)
        for (int J = 0; J < nfy; ++J) {
            const int i = I / R, s = I % R, j = J / R, t = J % R;
            for (int a = -2; a <= 2; ++a)
                for (int b = -2; b <= 2; ++b) {
                    idx.push_back((i * ncy + j) * 25 + (a + 2) * 5 + (b + 2));
                    wts.push_back(B[s * 5 + a + 2] * B[t * 5 + b + 2] * dvc);
                }
            for (size_t q = 1; q < P.size(); ++q) {
                if (I < P[q].lo[0] || I >= P[q].lo[0] + P[q].sz[0] || J < P[q].lo[1] || J >= P[q].lo[1] + P[q].sz[1])
                    continue;
                idx.push_back(m0 + task_base[q] + (I - P[q].lo[0]) * P[q].sz[1] + (J - P[q].lo[1]));
                wts.push_back(dvf);
            }
            rowptr.push_back((int)idx.size());
        }

    // ---- average-down lists
    std::vector<long long> avg_dst, avg_src;
    std::vector<int> avg_str;
    for (size_t q = 1; q < P.size(); ++q) {
        const A4Patch& G = P[q];
        const int s2 = G.sz[3], s1 = G.sz[2] * s2, s0 = G.sz[1] * s1;
        for (int i = G.lo[0] / R; i < (G.lo[0] + G.sz[0]) / R; ++i)
            for (int j = G.lo[1] / R; j < (G.lo[1] + G.sz[1]) / R; ++j)
                for (int k = G.lo[2] / R; k < (G.lo[2] + G.sz[2]) / R; ++k)
                    for (int l = G.lo[3] / R; l < (G.lo[3] + G.sz[3]) / R; ++l) {
                        avg_dst.push_back(cidx(i, j, k, l));
                        avg_src.push_back(G.off + (long long)(i * R - G.lo[0]) * s0 + (long long)(j * R - G.lo[1]) * s1 +
                                          (long long)(k * R - G.lo[2]) * s2 + (l * R - G.lo[3]));
                        avg_str.push_back(s0);
                        avg_str.push_back(s1);
                        avg_str.push_back(s2);
                    }
    }
    M.navg = (int)avg_dst.size();

    // ---- Fourier tables of the fine configuration mesh
    const std::vector<double> Qx = fourier_basis(nfx), Qy = fourier_basis_and_transpose(nfy);
    const std::vector<double> lx = fourier_symbol(nfx, M.lv[1].h[0]), ly = fourier_symbol(nfy, M.lv[1].h[1]);
    std::vector<double> inv((size_t)nfx * nfy);
    for (int l = 0; l < nfy; ++l)
        for (int k = 0; k < nfx; ++k) inv[(size_t)l * nfx + k] = (k == 0 && l == 0) ? 0.0 : 1.0 / (lx[k] + ly[l]);
    const std::vector<double> gxc(pb->veq[0][0], pb->veq[0][0] + n[2] + 4), gyc(pb->veq[0][1], pb->veq[0][1] + n[3] + 4);
    const std::vector<double> gxf(pb->veq[1][0], pb->veq[1][0] + M.nf[2] + 4),
        gyf(pb->veq[1][1], pb->veq[1][1] + M.nf[3] + 4);

    // ---- separable interpolation passes over every level-1 patch's padded box
    std::vector<A4Interp> ip;
    auto fdiv = [](int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
    for (size_t q = 1; q < P.size(); ++q) {
        A4Interp Q{};
        for (int d = 0; d < 4; ++d) {
            Q.plo[d] = P[q].lo[d] - 2;
            Q.pn[d] = P[q].sz[d] + 4;
            Q.clo[d] = fdiv(Q.plo[d], R) - 2;
            Q.cn[d] = fdiv(Q.plo[d] + Q.pn[d] - 1, R) + 2 - Q.clo[d] + 1;
            Q.ipn[d] = 1.0 / Q.pn[d];
            Q.icn[d] = 1.0 / Q.cn[d];
        }
        ip.push_back(Q);
    }
    long long acc_o = 0;
    for (int dir = 0; dir < 3; ++dir)
        for (A4Interp& Q : ip) {
            long long n = 1;
            for (int d = 0; d < 4; ++d) n *= d <= dir ? Q.pn[d] : Q.cn[d];
            Q.o[dir] = acc_o;
            acc_o += n;
        }
    const size_t scratch_elems = (size_t)std::max<long long>(acc_o, 1);
    // block tables of the padded copies (every patch) and of the passes
    std::vector<int2> ptile, itile[3];
    for (size_t q = 0; q < P.size(); ++q) {
        const A4Patch& Pq = P[list[q]];
        const long long n = (long long)(Pq.sz[0] + 4) * (Pq.sz[1] + 4) * (Pq.sz[2] + 4) * (Pq.sz[3] + 4);
        for (long long c = 0; c < n; c += 256) ptile.push_back(make_int2((int)q, (int)c));
    }
    for (int dir = 0; dir < 3; ++dir)
        for (size_t e = 0; e < ip.size(); ++e) {
            long long n = 1;
            for (int d = 0; d < 4; ++d) n *= d <= dir ? ip[e].pn[d] : ip[e].cn[d];
            for (long long c = 0; c < n; c += 256) itile[dir].push_back(make_int2((int)e, (int)c));
        }
    int2* d_pt = nullptr;
    int2* d_it[3] = {nullptr, nullptr, nullptr};

    TableArena T;
    T.add(&d_pt, ptile);
    for (int dir = 0; dir < 3; ++dir) T.add(&d_it[dir], itile[dir]);
    T.add(&M.d_interp, ip);
    T.add(&M.d_patches, P);
    T.add(&M.d_list, list);
    T.add(&M.d_nb, nb);
    T.add(&M.d_tiles, tiles);
    T.add(&M.d_B, B);
    T.add(&M.d_gxc, gxc);
    T.add(&M.d_gyc, gyc);
    T.add(&M.d_gxf, gxf);
    T.add(&M.d_gyf, gyf);
    T.add(&M.d_faces, faces);
    T.add(&M.d_rect_ptr, rect_ptr);
    T.add(&M.d_rects, rects);
    T.add(&M.d_task_off, task_off);
    T.add(&M.d_task_len, task_len);
    T.add(&M.d_rowptr, rowptr);
    T.add(&M.d_idx, idx);
    T.add(&M.d_w, wts);
    T.add(&M.d_corr_cell, corr_cell);
    T.add(&M.d_corr_ptr, corr_ptr);
    T.add(&M.d_corr_code, corr_code);
    T.add(&M.d_fine, fine);
    T.add(&M.d_avg_dst, avg_dst);
    T.add(&M.d_avg_src, avg_src);
    T.add(&M.d_avg_strides, avg_str);
    T.add(&M.d_Qx, Qx);
    T.add(&M.d_Qy, Qy);
    T.add(&M.d_inv, inv);
    VP_HIP(T.commit(&M.d_tables));
    M.ptiles.pad = d_pt;
    M.ptiles.npad = (int)ptile.size();
    for (int dir = 0; dir < 3; ++dir) {
        M.ptiles.pass[dir] = d_it[dir];
        M.ptiles.npass[dir] = (int)itile[dir].size();
    }
    VP_HIP(hipMalloc(&M.d_rhs_pad, std::max<size_t>(M.pad_total, 1) * sizeof(double)));
    VP_HIP(hipMalloc(&M.d_rhs_scratch, scratch_elems * sizeof(double)));
    VP_HIP(hipMalloc(&M.d_g, (size_t)2 * nfx * nfy * sizeof(double)));

    // ---- workspace: acc, two predictors, padded copies, boundary and coarse-fine fluxes, slots, n, g
    const size_t sb = al256(M.total * sizeof(double));
    size_t o = 0;
    p->ws_acc = o; o += sb;
    p->ws_fsa = o; o += sb;
    p->ws_fsb = o; o += sb;
    M.ws_pad = o; o += al256(std::max<size_t>(M.pad_total, 1) * sizeof(double));
    M.ws_interp = o; o += al256(scratch_elems * sizeof(double));
    M.ws_ff = o; o += al256(std::max<size_t>(M.fflux, 1) * sizeof(double));
    M.ws_cf = o; o += al256(std::max<size_t>(faces.size(), 1) * sizeof(double));
    M.ws_slots = o; o += al256((size_t)(m0 + M.ntasks) * sizeof(double));
    M.ws_n = o; o += al256((size_t)nfx * nfy * sizeof(double));
    M.ws_g = o; o += al256((size_t)2 * nfx * nfy * sizeof(double));
    p->ws_total = o;
    p->state_elems = M.total;
    return VP_OK;
}

void a4_destroy(vp_plan* p)
{
    Amr4DPlan* M = p->a4;
    if (!M) return;
    if (M->d_tables) (void)hipFree(M->d_tables);
    if (M->d_rhs_pad) (void)hipFree(M->d_rhs_pad);
    if (M->d_rhs_scratch) (void)hipFree(M->d_rhs_scratch);
    if (M->d_g) (void)hipFree(M->d_g);
    delete M;
    p->a4 = nullptr;
}

vp_status a4_rhs(const vp_plan* p, const void* f, const double* a, void* k, hipStream_t stream)
{
    const Amr4DPlan& M = *p->a4;
    const double* fd = static_cast<const double*>(f);
    if (vp_status st = pad_launch(p, fd, M.d_rhs_pad, M.d_rhs_scratch, stream)) return st;
    A4Args A = base_args(p, M.d_rhs_pad, a);
    A.fout = static_cast<double*>(k);
    VP_HIP(timed(p, kTStage, stream, [&] { return launch_a4_stage(kRhs, A, stream); }));
    return VP_OK;
}

vp_status a4_reduce(const vp_plan* p, const void* f, double* n, void* work, hipStream_t stream)
{
    return moment(p, static_cast<const double*>(f), n, work, stream);
}

vp_status a4_poisson(const vp_plan* p, const double* n, double* phi, double* E, hipStream_t stream)
{
    const Amr4DPlan& M = *p->a4;
    VP_HIP(timed(p, kTField, stream, [&] {
        return launch_poisson2d(n, M.nf[0], M.nf[1], M.lv[1].h[0], M.lv[1].h[1], p->pb.qm, M.d_Qx, M.d_Qy, M.d_inv,
                                M.d_g, phi, E, nullptr, stream);
    }));
    return VP_OK;
}

vp_status a4_inject(const vp_plan* p, const double* E, double* a, hipStream_t stream)
{
    const Amr4DPlan& M = *p->a4;
    const int nc = M.nc[0] * M.nc[1], nf = M.nf[0] * M.nf[1];
    VP_HIP(timed(p, kTOther, stream, [&] {
        hipError_t e = launch_scale(E, p->pb.qm, a + 2 * nc, 2 * nf, stream);
        if (e == hipSuccess) e = launch_a4_inject(a, M.nc[0], M.nc[1], M.R, stream);
        return e;
    }));
    return VP_OK;
}

vp_status a4_rk4(const vp_plan* p, void* f, double* a, double dt, void* work, hipStream_t stream)
{
    const Amr4DPlan& M = *p->a4;
    double* fd = static_cast<double*>(f);
    double* acc = reinterpret_cast<double*>(wp(work, p->ws_acc));
    double* sa = reinterpret_cast<double*>(wp(work, p->ws_fsa));
    double* sb = reinterpret_cast<double*>(wp(work, p->ws_fsb));
    double* pad = reinterpret_cast<double*>(wp(work, M.ws_pad));
    double* ff = reinterpret_cast<double*>(wp(work, M.ws_ff));
    double* cf = reinterpret_cast<double*>(wp(work, M.ws_cf));
    double* scr = reinterpret_cast<double*>(wp(work, M.ws_interp));
    double* out[4] = {sa, sb, sa, fd};
    const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const double cnext[3] = {0.5 * dt, 0.5 * dt, dt};
    if (vp_status st = pad_launch(p, fd, pad, scr, stream)) return st;
    for (int s = 0; s < 4; ++s) {
        const int kind = s == 0 ? kStage1 : (s == 3 ? kStage4 : kStage23);
        A4Args A = base_args(p, pad, a);
        A.fn = fd;
        A.acc = acc;
        A.fout = out[s];
        A.ff_acc = ff;
        A.c_acc = dt * b[s];
        A.c_next = s < 3 ? cnext[s] : 0.0;
        A.c_flux = b[s];
        A.first = s == 0;
        A.faces = M.d_faces;
        A.nfaces = M.nfaces;
        A.cf = cf;
        VP_HIP(timed(p, kTStage, stream, [&] { return launch_a4_stage(kind, A, stream); }));
        if (s < 3) {
            if (vp_status st = pad_launch(p, out[s], pad, scr, stream)) return st;
            if (vp_status st = constraint(p, out[s], a, work, stream)) return st;
        }
    }
    // end of step: coarse cells next to coarse-fine faces take the fine
    // accumulated fluxes, then covered coarse cells the mean of their fine cells
    VP_HIP(timed(p, kTSync, stream, [&] {
        const int nfine = M.R * M.R * M.R;
        hipError_t e = launch_a4_reflux(fd, M.d_corr_cell, M.d_corr_ptr, M.d_corr_code, M.d_fine, nfine, ff, cf,
                                        M.d_faces, M.lv[0].hi, dt, M.ncorr, stream);
        if (e == hipSuccess) e = launch_a4_average(fd, M.d_avg_dst, M.d_avg_src, M.d_avg_strides, M.R, M.navg, stream);
        return e;
    }));
    return constraint(p, fd, a, work, stream);
}

}  // namespace vp
