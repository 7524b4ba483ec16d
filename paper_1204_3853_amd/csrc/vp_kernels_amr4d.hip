// HIP kernels of the two-level 2D+2V path (the AMR of section 3 carried to
// the 2D+2V phase space).  Every patch, level 0 included, is copied each
// stage into a padded array with two ghost layers per direction; only the
// ghost cells the flux stencils read are filled (a cell outside the patch
// along one direction, or along one configuration and one velocity
// direction): on level 0 the periodic wrap and the equilibrium product; on
// level 1 the value of the level-1 patch that holds the cell, the fine
// equilibrium product outside the velocity box, else the conservative
// fifth-order sub-cell interpolation of level 0 as a tensor product over
// x, y, vx, vy.  The stage kernel then evaluates the fluxes of section 2
// direction by direction (the single-level 2D+2V formulas) from the padded
// arrays, one thread per cell.
#include <hip/hip_runtime.h>

#include "vp_internal.hpp"
#include "vp_stage_tile.hpp"

namespace vp {

namespace {

using namespace dev;

__device__ __forceinline__ int wrap4(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

struct A4View {
    const double* p;
    long long s0, s1, s2;      // strides of the padded array (the last is 1)
    __device__ __forceinline__ double operator()(int i, int j, int k, int l) const
    {
        return p[(i + 2) * s0 + (j + 2) * s1 + (k + 2) * s2 + (l + 2)];
    }
};

__device__ __forceinline__ A4View view_of(const double* pad, const A4Patch& P)
{
    A4View v;
    v.p = pad + P.pad;
    v.s2 = P.sz[3] + 4;
    v.s1 = (long long)(P.sz[2] + 4) * v.s2;
    v.s0 = (long long)(P.sz[1] + 4) * v.s1;
    return v;
}

// r % d with r = r / d for 0 <= r < 2^31, from a double reciprocal of d
// (the quotient estimate is off by at most one, which the remainder fixes)
__device__ __forceinline__ int divmod_rcp(int& r, int d, double inv)
{
    int q = (int)((double)r * inv);
    int m = r - q * d;
    if (m < 0) { --q; m += d; }
    else if (m >= d) { ++q; m -= d; }
    r = q;
    return m;
}

// i in [-n, 2n) wrapped into [0, n)
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// the accelerations a velocity-face flux of configuration cell (I, J) needs:
// a at the cell and the differences of its x and y neighbours, per component
struct A4Acc {
    double c[2], dx[2], dy[2];
};

__device__ __forceinline__ A4Acc acc_at(const double* a, const A4Level& L, int I, int J)
{
    const int n0 = L.n[0], n1 = L.n[1];
    const int i = wrap1(I, n0), j = wrap1(J, n1);
    const int ip = wrap1(i + 1, n0), im = wrap1(i - 1, n0), jp = wrap1(j + 1, n1), jm = wrap1(j - 1, n1);
    A4Acc r;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double* ac = a + L.a_off + c * n0 * n1;
        r.c[c] = ac[i * n1 + j];
        r.dx[c] = ac[ip * n1 + j] - ac[im * n1 + j];
        r.dy[c] = ac[i * n1 + jp] - ac[i * n1 + jm];
    }
    return r;
}

// flux through the upper face along `dir` of cell (i, j, k, l) of a patch
// (local indices; the face's other cells come from the padded copy)
__device__ __forceinline__ double face_flux(const A4View& U, const A4Patch& P, const A4Level& L, const A4Acc& ac4, int dir, int i,
                            int j, int k, int l)
{
    if (dir == 0) {
        const double fc = face4<double>(U(i - 1, j, k, l), U(i, j, k, l), U(i + 1, j, k, l), U(i + 2, j, k, l));
        const double fu = face4<double>(U(i - 1, j, k + 1, l), U(i, j, k + 1, l), U(i + 1, j, k + 1, l),
                                        U(i + 2, j, k + 1, l));
        const double fd = face4<double>(U(i - 1, j, k - 1, l), U(i, j, k - 1, l), U(i + 1, j, k - 1, l),
                                        U(i + 2, j, k - 1, l));
        const double vb = L.v_lo + ((double)(P.lo[2] + k) + 0.5) * L.h[2];
        return vb * fc + L.h[2] / 24.0 * (fu - fd);
    }
    if (dir == 1) {
        const double fc = face4<double>(U(i, j - 1, k, l), U(i, j, k, l), U(i, j + 1, k, l), U(i, j + 2, k, l));
        const double fu = face4<double>(U(i, j - 1, k, l + 1), U(i, j, k, l + 1), U(i, j + 1, k, l + 1),
                                        U(i, j + 2, k, l + 1));
        const double fd = face4<double>(U(i, j - 1, k, l - 1), U(i, j, k, l - 1), U(i, j + 1, k, l - 1),
                                        U(i, j + 2, k, l - 1));
        const double vb = L.v_lo + ((double)(P.lo[3] + l) + 0.5) * L.h[3];
        return vb * fc + L.h[3] / 24.0 * (fu - fd);
    }
    const bool c0 = dir == 2;                  // the component along the face's velocity direction
    const double ac = c0 ? ac4.c[0] : ac4.c[1], dax = c0 ? ac4.dx[0] : ac4.dx[1], day = c0 ? ac4.dy[0] : ac4.dy[1];
    auto fv = [&](int ii, int jj) {
        return dir == 2 ? face4<double>(U(ii, jj, k - 1, l), U(ii, jj, k, l), U(ii, jj, k + 1, l), U(ii, jj, k + 2, l))
                        : face4<double>(U(ii, jj, k, l - 1), U(ii, jj, k, l), U(ii, jj, k, l + 1), U(ii, jj, k, l + 2));
    };
    return ac * fv(i, j) + (dax * (fv(i + 1, j) - fv(i - 1, j)) + day * (fv(i, j + 1) - fv(i, j - 1))) / 48.0;
}

struct A4PadArgs {
    const double* f;
    const A4Patch* patches;
    const int* list;
    int npatch;
    const int* nb;
    A4Level lv[2];
    const double* B;           // b_j(s) at B[s * 5 + j + 2]
    int R;
    const double *gxc, *gyc, *gxf, *gyf;
    const A4Interp* ip;        // per level-1 patch (list index - 1)
    int nip;
    double* scratch;           // pass results
    double* pad;
    A4PadTiles tl;
};

// level-0 value with x, y periodic and the coarse equilibrium product outside the velocity box
__device__ __forceinline__ double coarse_at(const A4PadArgs& A, int i, int j, int k, int l)
{
    const A4Level& L = A.lv[0];
    if (k < 0 || k >= L.n[2] || l < 0 || l >= L.n[3]) return A.gxc[k + 2] * A.gyc[l + 2];
    return A.f[(((long long)wrap4(i, L.n[0]) * L.n[1] + wrap4(j, L.n[1])) * L.n[2] + k) * L.n[3] + l];
}

// One pass of the separable sub-cell interpolation of level 0 over every
// level-1 patch's padded box (the tensor product of section 3's
// one-dimensional weights, x innermost as in the definition, then y, vx
// and vy): DIR 0 reads level 0 and interpolates along x, DIR 1 along y,
// DIR 2 along vx; the vy pass is the last step of k_a4_pad.
template <int DIR>
__global__ __launch_bounds__(256) void k_a4_interp(A4PadArgs A)
{
    // the block's patch and first result from the block table
    const int2 tb = A.tl.pass[DIR][blockIdx.x];
    const A4Interp Q = A.ip[tb.x];
    // output extents: fine along x .. DIR, coarse after
    int ext[4];
    double iext[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        ext[d] = d <= DIR ? Q.pn[d] : Q.cn[d];
        iext[d] = d <= DIR ? Q.ipn[d] : Q.icn[d];
    }
    int r = tb.y + (int)threadIdx.x;
    if (r >= ext[0] * ext[1] * ext[2] * ext[3]) return;
    const long long g = Q.o[DIR] + r;
    int idx[4];
    idx[3] = divmod_rcp(r, ext[3], iext[3]);
    idx[2] = divmod_rcp(r, ext[2], iext[2]);
    idx[1] = divmod_rcp(r, ext[1], iext[1]);
    idx[0] = r;
    const int R = A.R;
    const int F = Q.plo[DIR] + idx[DIR];
    const int c = (F >= 0 ? F : F - R + 1) / R;
    const double* b = A.B + (F - c * R) * 5;
    double acc = 0.0;
    if (DIR == 0) {
        // velocity cells of the padded box beyond the velocity ghosts (only
        // read for fine cells outside the velocity box, which take the fine
        // equilibrium instead) use the nearest ghost factor
        const A4Level& L = A.lv[0];
        const int k = Q.clo[2] + idx[2], l = Q.clo[3] + idx[3];
        const bool vin = k >= 0 && k < L.n[2] && l >= 0 && l < L.n[3];
        const double geq = A.gxc[min(max(k + 2, 0), L.n[2] + 3)] * A.gyc[min(max(l + 2, 0), L.n[3] + 3)];
        const int j = wrap4(Q.clo[1] + idx[1], L.n[1]);
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            const double cv = vin ? A.f[(((long long)wrap4(c + t - 2, L.n[0]) * L.n[1] + j) * L.n[2] + (vin ? k : 0)) *
                                            L.n[3] + (vin ? l : 0)]
                                  : geq;
            acc += b[t] * cv;
        }
    } else {
        // the previous pass: extent coarse along DIR
        int pe[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) pe[d] = d < DIR ? Q.pn[d] : Q.cn[d];
        const double* in = A.scratch + Q.o[DIR - 1];
        const long long s3 = 1, s2 = pe[3], s1 = (long long)pe[2] * pe[3], s0 = (long long)pe[1] * pe[2] * pe[3];
        const long long sd = DIR == 1 ? s1 : s2;
        long long base = idx[0] * s0 + idx[3] * s3;
        base += DIR == 1 ? idx[2] * s2 : idx[1] * s1;
        base += (long long)(c - 2 - Q.clo[DIR]) * sd;
#pragma unroll
        for (int t = 0; t < 5; ++t) acc += b[t] * in[base + t * sd];
    }
    A.scratch[g] = acc;
}

__global__ __launch_bounds__(256) void k_a4_pad(A4PadArgs A)
{
    // the block's patch and first padded element from the block table
    const int2 tb = A.tl.pad[blockIdx.x];
    const A4Patch P = A.patches[A.list[tb.x]];
    int r = tb.y + (int)threadIdx.x;
    if (r >= (P.sz[0] + 4) * (P.sz[1] + 4) * (P.sz[2] + 4) * (P.sz[3] + 4)) return;
    const long long g = P.pad + r;
    const int l = divmod_rcp(r, P.sz[3] + 4, P.ipz[3]) - 2;
    const int k = divmod_rcp(r, P.sz[2] + 4, P.ipz[2]) - 2;
    const int j = divmod_rcp(r, P.sz[1] + 4, P.ipz[1]) - 2;
    const int i = r - 2;
    const bool ox = i < 0 || i >= P.sz[0], oy = j < 0 || j >= P.sz[1];
    const bool ok = k < 0 || k >= P.sz[2], ol = l < 0 || l >= P.sz[3];
    const int nout = (int)ox + (int)oy + (int)ok + (int)ol;
    double v;
    if (nout == 0) {
        v = A.f[P.off + (((long long)i * P.sz[1] + j) * P.sz[2] + k) * P.sz[3] + l];
    } else {
        // only the ghost cells the flux stencils read: outside along one
        // direction, or along one configuration and one velocity direction
        if (nout > 2 || (ox && oy) || (ok && ol)) return;
        const A4Level& L = A.lv[P.lev];
        const int I = P.lo[0] + i, J = P.lo[1] + j, K = P.lo[2] + k, Lv = P.lo[3] + l;
        if (P.lev == 0) {
            v = coarse_at(A, I, J, K, Lv);
        } else if (K < 0 || K >= L.n[2] || Lv < 0 || Lv >= L.n[3]) {
            v = A.gxf[K + 2] * A.gyf[Lv + 2];
        } else {
            bool held = false;
            const int Iw = wrap4(I, L.n[0]), Jw = wrap4(J, L.n[1]);
            for (int e = P.nb0; e < P.nb1 && !held; ++e) {
                const A4Patch Q = A.patches[A.nb[e]];
                const int di = Iw - Q.lo[0], dj = Jw - Q.lo[1], dk = K - Q.lo[2], dl = Lv - Q.lo[3];
                if (di >= 0 && di < Q.sz[0] && dj >= 0 && dj < Q.sz[1] && dk >= 0 && dk < Q.sz[2] && dl >= 0 &&
                    dl < Q.sz[3]) {
                    v = A.f[Q.off + (((long long)di * Q.sz[1] + dj) * Q.sz[2] + dk) * Q.sz[3] + dl];
                    held = true;
                }
            }
            if (!held) {
                // the last (vy) pass of the separable interpolation over the
                // results of the x, y and vx passes
                const A4Interp Q = A.ip[A.list[tb.x] - 1];
                const int R = A.R;
                const int cl = Lv / R;
                const double* bl = A.B + (Lv - cl * R) * 5;
                const int X = i + 2, Y = j + 2, Kk = k + 2;
                const double* t3 = A.scratch + Q.o[2] +
                                   (((long long)X * Q.pn[1] + Y) * Q.pn[2] + Kk) * Q.cn[3] + (cl - 2 - Q.clo[3]);
                double acc = 0.0;
#pragma unroll
                for (int d = 0; d < 5; ++d) acc += bl[d] * t3[d];
                v = acc;
            }
        }
    }
    A.pad[g] = v;
}

__device__ __forceinline__ void flux_store(double* p, double v, const A4Args& A)
{
    if (A.first) *p = A.c_flux * v;
    else *p += A.c_flux * v;
}

// level-0 flux through coarse-fine face q, accumulated with the stage's
// weight for the reflux at the end of the step
__device__ __forceinline__ void a4_face(const A4Args& A, int q)
{
    if (q >= A.nfaces) return;
    const A4Face F = A.faces[q];
    const A4Patch P = A.patches[0];
    const A4Acc ac4 = acc_at(A.a, A.lv[0], F.cell[0], F.cell[1]);
    const double G = face_flux(view_of(A.pad, P), P, A.lv[0], ac4, F.dir, F.cell[0], F.cell[1], F.cell[2], F.cell[3]);
    if (A.first) A.cf[q] = A.c_flux * G;
    else A.cf[q] += A.c_flux * G;
}

// One thread per kA4VxRun cells along vx of one (x, y, vy) of a patch
// (lanes along vy, so loads are coalesced): the x and vx face averages of
// the run come from windows of the padded copy held in registers, every
// face flux of the run evaluated once (the x faces on vx rows k0 - 1 ..
// k0 + run, the vx faces k0 - 1/2 .. k0 + run - 1/2); the y and vy faces,
// whose corrections take vy +- 1 and vy +- 2, per cell.  The same formulas
// and operand order as face_flux.  Rows past a ragged last run read the
// last row of the padded copy and are dropped.
template <int KIND>
__global__ __launch_bounds__(256) void k_a4_stage(A4Args A)
{
    constexpr int K = kA4VxRun;
    const int t = blockIdx.x;
    if (KIND != kRhs && t >= A.ntiles) {          // the blocks after the tiles: coarse-fine faces
        a4_face(A, (t - A.ntiles) * 256 + (int)threadIdx.x);
        return;
    }
    const A4Patch P = A.patches[A.tiles[2 * t]];
    const int n0 = P.sz[0], n1 = P.sz[1], n2 = P.sz[2], n3 = P.sz[3];
    const int ng = (n2 + K - 1) / K;
    const int c = A.tiles[2 * t + 1] + (int)threadIdx.x;       // below 2^31: the host checks the patch sizes
    if (c >= n0 * n1 * ng * n3) return;
    int r = c;
    const int l = divmod_rcp(r, n3, P.isz[3]);
    const int kg = divmod_rcp(r, ng, 1.0 / ng);
    const int j = divmod_rcp(r, n1, P.isz[1]);
    const int i = r;
    const int k0 = kg * K;
    const A4Level& L = A.lv[P.lev];
    const A4View U = view_of(A.pad, P);
    const A4Acc ac4 = acc_at(A.a, L, P.lo[0] + i, P.lo[1] + j);
    const bool acc_ff = KIND != kRhs && A.ff_acc && A.c_flux != 0.0 && P.lev == 1;
    const long long S0 = (long long)n1 * n2 * n3, S1 = (long long)n0 * n2 * n3, S2 = (long long)n0 * n1 * n3;
    double* ff = acc_ff ? A.ff_acc + P.foff : nullptr;
    auto row = [&](int k) { return min(k, n2 + 1); };
    double kk[K], f0[K];

    // x faces (transverse correction along vx)
    {
        double fp[K + 2], fm[K + 2];
#pragma unroll
        for (int q = 0; q < K + 2; ++q) {
            const int k = row(k0 - 1 + q);
            const double u0 = U(i - 2, j, k, l), u1 = U(i - 1, j, k, l), u2 = U(i, j, k, l), u3 = U(i + 1, j, k, l),
                         u4 = U(i + 2, j, k, l);
            fp[q] = face4<double>(u1, u2, u3, u4);
            fm[q] = face4<double>(u0, u1, u2, u3);
            if (q >= 1 && q <= K) f0[q - 1] = u2;
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int k = k0 + q;
            const double vb = L.v_lo + ((double)(P.lo[2] + k) + 0.5) * L.h[2];
            const double gx1 = vb * fp[q + 1] + L.h[2] / 24.0 * (fp[q + 2] - fp[q]);
            const double gx0 = vb * fm[q + 1] + L.h[2] / 24.0 * (fm[q + 2] - fm[q]);
            kk[q] = -(gx1 - gx0) * L.hi[0];
            if (acc_ff && k < n2) {
                if (i == 0) flux_store(ff + ((long long)j * n2 + k) * n3 + l, gx0, A);
                if (i == n0 - 1) flux_store(ff + S0 + ((long long)j * n2 + k) * n3 + l, gx1, A);
            }
        }
    }
    // y faces (transverse correction along vy)
    {
        const double vbl = L.v_lo + ((double)(P.lo[3] + l) + 0.5) * L.h[3];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int k = row(k0 + q);
            double fp[3], fm[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double u0 = U(i, j - 2, k, l + b - 1), u1 = U(i, j - 1, k, l + b - 1), u2 = U(i, j, k, l + b - 1),
                             u3 = U(i, j + 1, k, l + b - 1), u4 = U(i, j + 2, k, l + b - 1);
                fp[b] = face4<double>(u1, u2, u3, u4);
                fm[b] = face4<double>(u0, u1, u2, u3);
            }
            const double gy1 = vbl * fp[1] + L.h[3] / 24.0 * (fp[2] - fp[0]);
            const double gy0 = vbl * fm[1] + L.h[3] / 24.0 * (fm[2] - fm[0]);
            kk[q] = kk[q] - (gy1 - gy0) * L.hi[1];
            if (acc_ff && k0 + q < n2) {
                double* fy = ff + 2 * S0;
                if (j == 0) flux_store(fy + ((long long)i * n2 + k) * n3 + l, gy0, A);
                if (j == n1 - 1) flux_store(fy + S1 + ((long long)i * n2 + k) * n3 + l, gy1, A);
            }
        }
    }
    // the five configuration positions of the velocity faces' corrections
    const int pi[5] = {i, i + 1, i - 1, i, i}, pj[5] = {j, j, j, j + 1, j - 1};
    const double acx = ac4.c[0], daxx = ac4.dx[0], dayx = ac4.dy[0];
    const double acy = ac4.c[1], daxy = ac4.dx[1], dayy = ac4.dy[1];
    // vx faces k0 - 1/2 .. k0 + K - 1/2
    {
        double G[K + 1];
        double w[5][K + 4];            // vx rows k0 - 2 .. k0 + K + 1
#pragma unroll
        for (int p = 0; p < 5; ++p)
#pragma unroll
            for (int q = 0; q < K + 4; ++q) w[p][q] = U(pi[p], pj[p], row(k0 - 2 + q), l);
#pragma unroll
        for (int m = 0; m < K + 1; ++m) {
            double fv[5];
#pragma unroll
            for (int p = 0; p < 5; ++p) fv[p] = face4<double>(w[p][m], w[p][m + 1], w[p][m + 2], w[p][m + 3]);
            G[m] = acx * fv[0] + (daxx * (fv[1] - fv[2]) + dayx * (fv[3] - fv[4])) / 48.0;
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int k = k0 + q;
            kk[q] = kk[q] - (G[q + 1] - G[q]) * L.hi[2];
            if (acc_ff && k < n2) {
                double* fk = ff + 2 * S0 + 2 * S1;
                if (k == 0) flux_store(fk + ((long long)i * n1 + j) * n3 + l, G[q], A);
                if (k == n2 - 1) flux_store(fk + S2 + ((long long)i * n1 + j) * n3 + l, G[q + 1], A);
            }
        }
    }
    // vy faces l - 1/2 and l + 1/2, per cell
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const int k = row(k0 + q);
        double fvp[5], fvm[5];
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            const double u0 = U(pi[p], pj[p], k, l - 2), u1 = U(pi[p], pj[p], k, l - 1), u2 = U(pi[p], pj[p], k, l),
                         u3 = U(pi[p], pj[p], k, l + 1), u4 = U(pi[p], pj[p], k, l + 2);
            fvp[p] = face4<double>(u1, u2, u3, u4);
            fvm[p] = face4<double>(u0, u1, u2, u3);
        }
        const double gl1 = acy * fvp[0] + (daxy * (fvp[1] - fvp[2]) + dayy * (fvp[3] - fvp[4])) / 48.0;
        const double gl0 = acy * fvm[0] + (daxy * (fvm[1] - fvm[2]) + dayy * (fvm[3] - fvm[4])) / 48.0;
        kk[q] = kk[q] - (gl1 - gl0) * L.hi[3];
        if (acc_ff && k0 + q < n2) {
            double* fl = ff + 2 * S0 + 2 * S1 + 2 * S2;
            if (l == 0) flux_store(fl + ((long long)i * n1 + j) * n2 + k, gl0, A);
            if (l == n3 - 1) flux_store(fl + (long long)n0 * n1 * n2 + ((long long)i * n1 + j) * n2 + k, gl1, A);
        }
    }
    // the stage combine of the run's cells
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const int k = k0 + q;
        if (k >= n2) break;
        const long long o = P.off + (((long long)i * n1 + j) * n2 + k) * n3 + l;
        if (KIND == kRhs) {
            A.fout[o] = kk[q];
        } else if (KIND == kStage1) {
            A.acc[o] = f0[q] + A.c_acc * kk[q];
            A.fout[o] = f0[q] + A.c_next * kk[q];
        } else if (KIND == kStage23) {
            A.acc[o] = A.acc[o] + A.c_acc * kk[q];
            A.fout[o] = A.fn[o] + A.c_next * kk[q];
        } else {
            A.fout[o] = A.acc[o] + A.c_acc * kk[q];
        }
    }
}

// The sums the Mask reduction combines, in one launch.  Blocks below ncx ncy:
// one per level-0 configuration column c, whose velocity plane sum S the
// block forms once; every masked sum that reads column c (target column
// c - (a, b) for stencil offsets a, b in [-2, 2], masked by the velocity
// rectangles level 1 covers in the target column, rects[rp[t] .. rp[t+1]),
// k0 k1 l0 l1 inclusive) is S less the covered cells, which one wave reads
// back (the block has just read the plane, so from the caches), and goes to
// M[t * 25 + (a+2) * 5 + (b+2)].  Blocks from ncx ncy on: one wave per
// level-1 row segment, M[25 ncx ncy + k] = the sum of len[k] consecutive
// values at off[k].
__global__ __launch_bounds__(256) void k_a4_moment_sums(const double* __restrict__ f, const int* __restrict__ rp,
                                                       const int4* __restrict__ rects, int ncx, int ncy, int nvy,
                                                       int plane, const long long* __restrict__ off,
                                                       const int* __restrict__ len, int ntasks,
                                                       double* __restrict__ M)
{
    __shared__ double red[4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int ncol = ncx * ncy;
    if ((int)blockIdx.x >= ncol) {
        const int task = ((int)blockIdx.x - ncol) * 4 + wv;
        if (task >= ntasks) return;                      // uniform per wave
        const double* p = f + off[task];
        const int n = len[task];
        double s = 0.0;
        for (int j = lane; j < n; j += 64) s += p[j];
        s = wave_sum(s);
        if (lane == 0) M[25 * ncol + task] = s;
        return;
    }
    const int c = (int)blockIdx.x;
    const int ci = c / ncy, cj = c - ci * ncy;
    const double* src = f + (long long)c * plane;
    double acc = 0.0;
#pragma unroll 4
    for (int q = t; q < plane; q += 256) acc += src[q];
    acc = wave_sum(acc);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    const double S = ((red[0] + red[1]) + red[2]) + red[3];
    for (int s = wv; s < 25; s += 4) {
        const int a = s / 5 - 2, b = s - (s / 5) * 5 - 2;
        const int tgt = wrap4(ci - a, ncx) * ncy + wrap4(cj - b, ncy);
        const int e0 = rp[tgt], e1 = rp[tgt + 1];
        double cov = 0.0;
        if (e0 < e1) {                                   // uniform per wave
            for (int e = e0; e < e1; ++e) {
                const int4 r = rects[e];
                const int w = r.w - r.z + 1, cnt = (r.y - r.x + 1) * w;
                for (int q = lane; q < cnt; q += 64) cov += src[(r.x + q / w) * nvy + r.z + q % w];
            }
            cov = wave_sum(cov);
        }
        if (lane == 0) M[tgt * 25 + s] = S - cov;
    }
}

// the coarse acceleration: the mean of the R x R fine values of each component
__global__ __launch_bounds__(256) void k_a4_inject(double* __restrict__ a, int ncx, int ncy, int R)
{
    const int q = (int)blockIdx.x * 256 + threadIdx.x;
    const int nc = ncx * ncy;
    if (q >= 2 * nc) return;
    const int comp = q / nc, cell = q - comp * nc;
    const int i = cell / ncy, j = cell - (cell / ncy) * ncy;
    const int nfy = ncy * R;
    const double* af = a + 2 * nc + (long long)comp * nc * R * R;
    double s = 0.0;
    for (int u = 0; u < R; ++u)
        for (int w = 0; w < R; ++w) s += af[(long long)(i * R + u) * nfy + (j * R + w)];
    a[q] = s / (R * R);
}

__global__ __launch_bounds__(256) void k_a4_reflux(double* __restrict__ f, const long long* __restrict__ cell,
                                                  const int* __restrict__ ptr, const int* __restrict__ code,
                                                  const int* __restrict__ fine, int nfine,
                                                  const double* __restrict__ ff, const double* __restrict__ cf,
                                                  const A4Face* __restrict__ faces, double h0, double h1, double h2,
                                                  double h3, int ncorr)
{
    const int q = (int)blockIdx.x * 256 + threadIdx.x;
    if (q >= ncorr) return;
    double val = f[cell[q]];
    for (int e = ptr[q]; e < ptr[q + 1]; ++e) {
        const int cd = code[e];
        const bool lower = cd < 0;                   // the face is the cell's lower face
        const int fi = lower ? -cd - 1 : cd;
        double s = 0.0;
        for (int u = 0; u < nfine; ++u) s += ff[fine[(long long)fi * nfine + u]];
        const double diff = s / nfine - cf[fi];
        const int d = faces[fi].dir;
        const double h = d == 0 ? h0 : (d == 1 ? h1 : (d == 2 ? h2 : h3));
        val += lower ? h * diff : -h * diff;
    }
    f[cell[q]] = val;
}

__global__ __launch_bounds__(256) void k_a4_average(double* __restrict__ f, const long long* __restrict__ dst,
                                                   const long long* __restrict__ src, const int* __restrict__ strides,
                                                   int R, int n)
{
    const int q = (int)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const long long s0 = strides[3 * q], s1 = strides[3 * q + 1], s2 = strides[3 * q + 2];
    const double* b = f + src[q];
    double s = 0.0;
    for (int u0 = 0; u0 < R; ++u0)
        for (int u1 = 0; u1 < R; ++u1)
            for (int u2 = 0; u2 < R; ++u2)
                for (int u3 = 0; u3 < R; ++u3) s += b[u0 * s0 + u1 * s1 + u2 * s2 + u3];
    f[dst[q]] = s / ((double)R * R * R * R);
}

}  // namespace

hipError_t launch_a4_pad(const double* f, const A4Patch* patches, const int* list, int npatch, long long total,
                         const int* nb, const A4Level* lv_host, const double* B, int R, const double* gxc,
                         const double* gyc, const double* gxf, const double* gyf, const A4Interp* ip,
                         const A4PadTiles& tl, double* scratch, double* pad, hipStream_t stream)
{
    if (total <= 0) return hipSuccess;
    A4PadArgs A{};
    A.f = f;
    A.patches = patches;
    A.list = list;
    A.npatch = npatch;
    A.nb = nb;
    A.lv[0] = lv_host[0];
    A.lv[1] = lv_host[1];
    A.B = B;
    A.R = R;
    A.gxc = gxc;
    A.gyc = gyc;
    A.gxf = gxf;
    A.gyf = gyf;
    A.ip = ip;
    A.nip = npatch - 1;
    A.scratch = scratch;
    A.pad = pad;
    A.tl = tl;
    if (A.nip > 0) {
        if (tl.npass[0] > 0) hipLaunchKernelGGL(k_a4_interp<0>, dim3(tl.npass[0]), dim3(256), 0, stream, A);
        if (tl.npass[1] > 0) hipLaunchKernelGGL(k_a4_interp<1>, dim3(tl.npass[1]), dim3(256), 0, stream, A);
        if (tl.npass[2] > 0) hipLaunchKernelGGL(k_a4_interp<2>, dim3(tl.npass[2]), dim3(256), 0, stream, A);
    }
    if (tl.npad > 0) hipLaunchKernelGGL(k_a4_pad, dim3(tl.npad), dim3(256), 0, stream, A);
    return hipGetLastError();
}

hipError_t launch_a4_stage(int kind, const A4Args& a, hipStream_t stream)
{
    const int fblocks = kind != kRhs && a.cf ? (a.nfaces + 255) / 256 : 0;
    if (a.ntiles + fblocks <= 0) return hipSuccess;
    const dim3 g(a.ntiles + fblocks), b(256);
    switch (kind) {
    case kRhs: hipLaunchKernelGGL(k_a4_stage<kRhs>, g, b, 0, stream, a); break;
    case kStage1: hipLaunchKernelGGL(k_a4_stage<kStage1>, g, b, 0, stream, a); break;
    case kStage23: hipLaunchKernelGGL(k_a4_stage<kStage23>, g, b, 0, stream, a); break;
    default: hipLaunchKernelGGL(k_a4_stage<kStage4>, g, b, 0, stream, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_a4_moment_sums(const double* f, const int* rp, const int4* rects, const int* n,
                                const long long* task_off, const int* task_len, int ntasks, double* M,
                                hipStream_t stream)
{
    const int ncol = n[0] * n[1];
    const int blocks = ncol + (ntasks + 3) / 4;
    hipLaunchKernelGGL(k_a4_moment_sums, dim3(blocks), dim3(256), 0, stream, f, rp, rects, n[0], n[1], n[3],
                       n[2] * n[3], task_off, task_len, ntasks, M);
    return hipGetLastError();
}

hipError_t launch_a4_inject(double* a, int ncx, int ncy, int R, hipStream_t stream)
{
    const int n = 2 * ncx * ncy;
    hipLaunchKernelGGL(k_a4_inject, dim3((n + 255) / 256), dim3(256), 0, stream, a, ncx, ncy, R);
    return hipGetLastError();
}

hipError_t launch_a4_reflux(double* f, const long long* cell, const int* ptr, const int* code, const int* fine,
                            int nfine, const double* ff, const double* cf, const A4Face* faces, const double* hdt,
                            double dt, int ncorr, hipStream_t stream)
{
    if (ncorr <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_a4_reflux, dim3((ncorr + 255) / 256), dim3(256), 0, stream, f, cell, ptr, code, fine, nfine,
                       ff, cf, faces, dt * hdt[0], dt * hdt[1], dt * hdt[2], dt * hdt[3], ncorr);
    return hipGetLastError();
}

hipError_t launch_a4_average(double* f, const long long* dst, const long long* src, const int* strides, int R, int n,
                             hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_a4_average, dim3((n + 255) / 256), dim3(256), 0, stream, f, dst, src, strides, R, n);
    return hipGetLastError();
}

}  // namespace vp
