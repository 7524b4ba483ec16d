// HIP kernels of regridding (section 3) for 1D+1V levels stored [x][v]
// (FP64):
//   k_tag          the refinement criterion delta1 f + delta2 f > tol on a
//                  level (x periodic, velocity ghosts = equilibrium);
//   k_prolong      the conservative limited WENO5 interpolation of the
//                  coarse level into every new level-1 patch, x then v, one
//                  thread per coarse cell of a patch;
//   k_copy_old     new fine cells that an old level-1 patch covers take the
//                  old fine value.
#include <hip/hip_runtime.h>

#include "vp_internal.hpp"

namespace vp {

namespace {

__device__ __forceinline__ int wrapr(int i, int n)
{
    const int r = i % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ double level_at(const double* f, int nx, int nv, const double* vg, int i, int j)
{
    if (j < 0) return vg[j + 2];
    if (j >= nv) return vg[j - nv + 2];
    return f[(size_t)wrapr(i, nx) * nv + j];
}

struct Ghosts {
    double v[4];   // equilibrium cell averages at j = -2, -1, nv, nv + 1
};

// the same criterion from the values of the cell and its four neighbours
__device__ __forceinline__ double tag_from(double c, double xm, double xp, double vm, double vp, double dx, double dv)
{
#pragma clang fp contract(off)
    const double gx = xp - xm, gv = vp - vm;
    const double d1 = __builtin_sqrt(0.5 * (dx * (gx * gx) + dv * (gv * gv)));
    const double sx = (xp - 2.0 * c) + xm, sv = (vp - 2.0 * c) + vm;
    const double d2 = 0.5 * ((dx * dx) * __builtin_fabs(sx) + (dv * dv) * __builtin_fabs(sv));
    return d1 + d2;
}

// delta1 f + delta2 f of one cell.  The operations run in a fixed order
// without fused multiply-adds (per direction the squared central
// difference scaled by h, x term plus v term, halved, square root; the
// second differences as (f(+) - 2 f) + f(-), magnitudes scaled by h^2,
// x plus v, halved; the sum of the two), so that the value is reproducible
// to the last bit.
__device__ double tag_value(const double* f, int nx, int nv, const double* vg, double dx, double dv, int i, int j)
{
    const double c = level_at(f, nx, nv, vg, i, j);
    const double xm = level_at(f, nx, nv, vg, i - 1, j), xp = level_at(f, nx, nv, vg, i + 1, j);
    const double vm = level_at(f, nx, nv, vg, i, j - 1), vp = level_at(f, nx, nv, vg, i, j + 1);
    return tag_from(c, xm, xp, vm, vp, dx, dv);
}

typedef double tag_d2 __attribute__((ext_vector_type(2)));

// DPP wave shifts of a double: lane l reads lane l + 1 (wave_shl:1) or lane
// l - 1 (wave_shr:1); the lane without a source is overridden by the caller
template <int CTRL>
__device__ __forceinline__ double tag_dpp(double x)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

constexpr int kTagRows = 8;     // x rows marched by one thread

// one row of a thread's four cells, and the one value beyond the wave's
// ends that lane 0 (left neighbour) or lane 63 (right neighbour) needs
struct TagRow {
    tag_d2 a, b;
    double e;
};

// four consecutive velocity cells per thread (nv % 4 == 0), marching
// kTagRows x rows with the rows i-1, i, i+1 in registers, so each row is
// read about once (rows past the end of x, in the last block, are read
// wrapped and their tags not stored); velocity neighbours come from the adjacent lanes, the
// tags of the four cells leave in one 4-byte store
__global__ __launch_bounds__(256) void k_tag4(const double* __restrict__ f, int nx, int nv, Ghosts g, double dx,
                                              double dv, double tol, unsigned* __restrict__ tags4,
                                              double* __restrict__ values)
{
    const int lane = (int)(threadIdx.x & 63);
    const int j0 = (int)(blockIdx.x * 256 + threadIdx.x) * 4;
    const bool live = j0 < nv;
    const int jc = live ? j0 : nv - 4;          // idle lanes read a valid group, store nothing
    const bool edge = lane == 0 || lane == 63;
    const int je = lane == 0 ? (jc > 0 ? jc - 1 : 0) : (jc + 4 < nv ? jc + 4 : nv - 1);
    const int i0 = (int)blockIdx.y * kTagRows;
    const int i1 = i0 + kTagRows < nx ? i0 + kTagRows : nx;
    auto load = [&](int i, TagRow& r) {
        const double* row = f + (size_t)wrapr(i, nx) * nv;
        r.a = *reinterpret_cast<const tag_d2*>(row + jc);
        r.b = *reinterpret_cast<const tag_d2*>(row + jc + 2);
        r.e = edge ? row[je] : 0.0;
    };
    // fully unrolled, so that the rows need no register moves and the load
    // of row i + 2 is in flight while row i is evaluated
    TagRow r[kTagRows + 2];
    load(i0 - 1, r[0]);
    load(i0, r[1]);
#pragma unroll
    for (int k = 0; k < kTagRows; ++k) {
        if (k == 0) load(i0 + 1, r[2]);
        if (k + 3 < kTagRows + 2) load(i0 + k + 2, r[k + 3]);
        const TagRow& m = r[k];
        const TagRow& c = r[k + 1];
        const TagRow& p = r[k + 2];
        double vlo = tag_dpp<0x138>(c.b.y), vhi = tag_dpp<0x130>(c.a.x);
        if (lane == 0) vlo = c.e;
        if (lane == 63) vhi = c.e;
        if (jc == 0) vlo = g.v[1];
        if (jc + 4 >= nv) vhi = g.v[2];
        const double cv[6] = {vlo, c.a.x, c.a.y, c.b.x, c.b.y, vhi};
        const double xm[4] = {m.a.x, m.a.y, m.b.x, m.b.y}, xp[4] = {p.a.x, p.a.y, p.b.x, p.b.y};
        unsigned packed = 0;
        double t[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            t[w] = tag_from(cv[w + 1], xm[w], xp[w], cv[w], cv[w + 2], dx, dv);
            packed |= (t[w] > tol ? 1u : 0u) << (8 * w);
        }
        const int i = i0 + k;
        if (live && i < i1) {
            const size_t e = (size_t)i * nv + j0;
            tags4[e / 4] = packed;
            if (values) {
                *reinterpret_cast<tag_d2*>(values + e) = tag_d2{t[0], t[1]};
                *reinterpret_cast<tag_d2*>(values + e + 2) = tag_d2{t[2], t[3]};
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_tag(const double* __restrict__ f, int nx, int nv, Ghosts g, double dx,
                                             double dv, double tol, unsigned char* __restrict__ tags,
                                             double* __restrict__ values)
{
    const int j = (int)(blockIdx.x * 256 + threadIdx.x);
    const int i = (int)blockIdx.y;
    if (j >= nv) return;
    const double t = tag_value(f, nx, nv, g.v, dx, dv, i, j);
    const size_t e = (size_t)i * nv + j;
    tags[e] = t > tol ? 1 : 0;
    if (values) values[e] = t;
}

// The criterion on a 2D+2V mesh [x][y][vx][vy]: the sums over the four
// directions in the order x, y, vx, vy, each term formed as in tag_from
// (no fused multiply-adds, correctly rounded square root).  Block row
// blockIdx.y is a run of kTag4DRows configuration cells along y at one x;
// its threads cover 256 consecutive cells of the velocity plane and march
// along y, so every neighbour load (the same plane position in the x and y
// neighbour planes, vx +- 1 rows, vy +- 1 lanes) is coalesced and the y
// neighbours are reused from registers.  Index arithmetic is 32-bit (the plan limits
// keep every element offset below 2^31).
__device__ __forceinline__ double tag_term(double p, double m, double u, double h, double& s2)
{
#pragma clang fp contract(off)
    const double g = p - m, sd = (p - 2.0 * u) + m;
    s2 = (h * h) * __builtin_fabs(sd);
    return h * (g * g);
}

constexpr int kTag4DRows = 8;     // configuration cells along y per thread

__global__ __launch_bounds__(256) void k_tag4d(Tag4DArgs a)
{
#pragma clang fp contract(off)
    const int plane = a.nvx * a.nvy;
    const int q = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (q >= plane) return;
    const int nyb = (a.ny + kTag4DRows - 1) / kTag4DRows;
    const int by = (int)blockIdx.y;
    const int i = by / nyb, j0 = (by - (by / nyb) * nyb) * kTag4DRows;
    const int j1 = min(j0 + kTag4DRows, a.ny);
    const int k = q / a.nvy, l = q - (q / a.nvy) * a.nvy;
    const int ip = i + 1 == a.nx ? 0 : i + 1, im = i == 0 ? a.nx - 1 : i - 1;
    const double* f = a.f;
    const double gyl = a.gy[l + 2], gxk = a.gx[k + 2];
    const double gvxp = a.gx[k + 3] * gyl, gvxm = a.gx[k + 1] * gyl;
    const double gvyp = gxk * a.gy[l + 3], gvym = gxk * a.gy[l + 1];
    // march along y, the y neighbours rolling through registers
    double ym = f[(i * a.ny + (j0 == 0 ? a.ny - 1 : j0 - 1)) * plane + q];
    double u = f[(i * a.ny + j0) * plane + q];
    for (int j = j0; j < j1; ++j) {
        const int jp = j + 1 == a.ny ? 0 : j + 1;
        const int base = (i * a.ny + j) * plane;
        const double yp = f[(i * a.ny + jp) * plane + q];
        const double xp = f[(ip * a.ny + j) * plane + q], xm = f[(im * a.ny + j) * plane + q];
        const double vxp = k + 1 < a.nvx ? f[base + q + a.nvy] : gvxp;
        const double vxm = k > 0 ? f[base + q - a.nvy] : gvxm;
        const double vyp = l + 1 < a.nvy ? f[base + q + 1] : gvyp;
        const double vym = l > 0 ? f[base + q - 1] : gvym;
        double t2, s1, s2;
        s1 = tag_term(xp, xm, u, a.h[0], t2);
        s2 = t2;
        s1 = s1 + tag_term(yp, ym, u, a.h[1], t2);
        s2 = s2 + t2;
        s1 = s1 + tag_term(vxp, vxm, u, a.h[2], t2);
        s2 = s2 + t2;
        s1 = s1 + tag_term(vyp, vym, u, a.h[3], t2);
        s2 = s2 + t2;
        const double v = __builtin_sqrt(0.5 * s1) + 0.5 * s2;
        a.tags[base + q] = v > a.tol ? 1 : 0;
        if (a.values) a.values[base + q] = v;
        ym = u;
        u = yp;
    }
}

// The same with four consecutive vy cells per thread (nvy % 4 == 0): the
// rows come in as 32-byte vector loads, the inner vy neighbours are the
// thread's own values, and the four tags go out as one 32-bit store.  Per
// cell the arithmetic is that of k_tag4d, term by term.
typedef double tag_d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_tag4d_v4(Tag4DArgs a)
{
#pragma clang fp contract(off)
    const int plane = a.nvx * a.nvy, nq = a.nvy >> 2;
    const int g = (int)blockIdx.x * 256 + (int)threadIdx.x;      // group of four vy cells
    if (g >= plane >> 2) return;
    const int nyb = (a.ny + kTag4DRows - 1) / kTag4DRows;
    const int by = (int)blockIdx.y;
    const int i = by / nyb, j0 = (by - (by / nyb) * nyb) * kTag4DRows;
    const int j1 = min(j0 + kTag4DRows, a.ny);
    const int k = g / nq, l0 = (g - (g / nq) * nq) * 4;
    const int q = k * a.nvy + l0;
    const int ip = i + 1 == a.nx ? 0 : i + 1, im = i == 0 ? a.nx - 1 : i - 1;
    const double* f = a.f;
    auto ld4 = [&](int off) { return *reinterpret_cast<const tag_d4*>(f + off); };
    double gvxp[4], gvxm[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        gvxp[w] = a.gx[k + 3] * a.gy[l0 + w + 2];
        gvxm[w] = a.gx[k + 1] * a.gy[l0 + w + 2];
    }
    const double gxk = a.gx[k + 2];
    const double gvym = gxk * a.gy[l0 + 1], gvyp = gxk * a.gy[l0 + 6];
    tag_d4 ym = ld4((i * a.ny + (j0 == 0 ? a.ny - 1 : j0 - 1)) * plane + q);
    tag_d4 u = ld4((i * a.ny + j0) * plane + q);
    for (int j = j0; j < j1; ++j) {
        const int jp = j + 1 == a.ny ? 0 : j + 1;
        const int base = (i * a.ny + j) * plane;
        const tag_d4 yp = ld4((i * a.ny + jp) * plane + q);
        const tag_d4 xp = ld4((ip * a.ny + j) * plane + q), xm = ld4((im * a.ny + j) * plane + q);
        const tag_d4 vxp = k + 1 < a.nvx ? ld4(base + q + a.nvy) : tag_d4{gvxp[0], gvxp[1], gvxp[2], gvxp[3]};
        const tag_d4 vxm = k > 0 ? ld4(base + q - a.nvy) : tag_d4{gvxm[0], gvxm[1], gvxm[2], gvxm[3]};
        const double left = l0 > 0 ? f[base + q - 1] : gvym;
        const double right = l0 + 4 < a.nvy ? f[base + q + 4] : gvyp;
        const double uu[6] = {left, u.x, u.y, u.z, u.w, right};
        const double xpv[4] = {xp.x, xp.y, xp.z, xp.w}, xmv[4] = {xm.x, xm.y, xm.z, xm.w};
        const double ypv[4] = {yp.x, yp.y, yp.z, yp.w}, ymv[4] = {ym.x, ym.y, ym.z, ym.w};
        const double vxpv[4] = {vxp.x, vxp.y, vxp.z, vxp.w}, vxmv[4] = {vxm.x, vxm.y, vxm.z, vxm.w};
        unsigned packed = 0;
        double vout[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const double c = uu[w + 1];
            double t2, s1, s2;
            s1 = tag_term(xpv[w], xmv[w], c, a.h[0], t2);
            s2 = t2;
            s1 = s1 + tag_term(ypv[w], ymv[w], c, a.h[1], t2);
            s2 = s2 + t2;
            s1 = s1 + tag_term(vxpv[w], vxmv[w], c, a.h[2], t2);
            s2 = s2 + t2;
            s1 = s1 + tag_term(uu[w + 2], uu[w], c, a.h[3], t2);
            s2 = s2 + t2;
            vout[w] = __builtin_sqrt(0.5 * s1) + 0.5 * s2;
            packed |= (vout[w] > a.tol ? 1u : 0u) << (8 * w);
        }
        *reinterpret_cast<unsigned*>(a.tags + base + q) = packed;
        if (a.values) *reinterpret_cast<tag_d4*>(a.values + base + q) = tag_d4{vout[0], vout[1], vout[2], vout[3]};
        ym = u;
        u = yp;
    }
}

// R fine cell averages of the middle of u[0..4] (eqs. aux1, aux2,
// interp_r_avg; B^(0) = 2 D_i - D_{i+1}, the value the definition gives);
// every candidate renormalised to the coarse average, then combined with
// the WENO5 weights (ideal weights 3/10, 3/5, 1/10, epsilon 1e-6)
template <int R>
__device__ __forceinline__ void prolong1d(const double* u, double* out)
{
    const double Dm2 = u[1] - u[0], Dm1 = u[2] - u[1], D0 = u[3] - u[2], Dp1 = u[4] - u[3];
    const double Lm1 = Dm1 - Dm2, L0 = D0 - Dm1, Lp1 = Dp1 - D0;
    const double b0 = 13.0 / 12.0 * Lp1 * Lp1 + 0.25 * (Dp1 - 3.0 * D0) * (Dp1 - 3.0 * D0);
    const double b1 = 13.0 / 12.0 * L0 * L0 + 0.25 * (D0 + Dm1) * (D0 + Dm1);
    const double b2 = 13.0 / 12.0 * Lm1 * Lm1 + 0.25 * (3.0 * Dm1 - Dm2) * (3.0 * Dm1 - Dm2);
    const double a0 = 0.3 / ((1e-6 + b0) * (1e-6 + b0));
    const double a1 = 0.6 / ((1e-6 + b1) * (1e-6 + b1));
    const double a2 = 0.1 / ((1e-6 + b2) * (1e-6 + b2));
    const double as = (a0 + a1) + a2;
    const double w[3] = {a0 / as, a1 / as, a2 / as};
    const double ui = u[2];
    const double A[3] = {ui + (2.0 * Dp1 - 5.0 * D0) / 6.0, ui - (D0 + 2.0 * Dm1) / 6.0, ui - (4.0 * Dm1 - Dm2) / 6.0};
    const double B[3] = {2.0 * D0 - Dp1, Dm1, Dm1};
    const double C[3] = {Lp1, L0, Lm1};
#pragma unroll
    for (int s = 0; s < R; ++s) out[s] = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double fine[R];
        double sum = 0.0;
#pragma unroll
        for (int s = 0; s < R; ++s) {
            fine[s] = A[r] + B[r] * ((2.0 * s + 1.0) / (2.0 * R)) + C[r] * ((3.0 * s * s + 3.0 * s + 1.0) / (6.0 * R * R));
            sum += fine[s];
        }
        fine[R - 1] += ui - sum / R;
#pragma unroll
        for (int s = 0; s < R; ++s) out[s] += w[r] * fine[s];
    }
}

// blockIdx.y: new patch; thread: one coarse cell of its footprint
template <int R>
__global__ __launch_bounds__(128) void k_prolong(const double* __restrict__ fc, int ncx, int ncv, Ghosts g,
                                                 const AmrPatch* __restrict__ patches, double* __restrict__ fnew)
{
    const AmrPatch P = patches[blockIdx.y];
    const int pcx = P.nx / R, pcv = P.nv / R;
    const int q = (int)(blockIdx.x * 128 + threadIdx.x);
    if (q >= pcx * pcv) return;
    const int cxl = q / pcv, cvl = q - (q / pcv) * pcv;
    const int cx = P.gx0 / R + cxl, cv = P.gv0 / R + cvl;
    // x first: the R fine rows of this coarse column at coarse v rows cv-2 .. cv+2
    double T[R][5];
#pragma unroll
    for (int e = 0; e < 5; ++e) {
        double u[5], o[R];
#pragma unroll
        for (int k = 0; k < 5; ++k) u[k] = level_at(fc, ncx, ncv, g.v, cx - 2 + k, cv - 2 + e);
        prolong1d<R>(u, o);
#pragma unroll
        for (int s = 0; s < R; ++s) T[s][e] = o[s];
    }
    // then v
#pragma unroll
    for (int s = 0; s < R; ++s) {
        double o[R];
        prolong1d<R>(T[s], o);
        double* dst = fnew + P.off + (size_t)(cxl * R + s) * P.nv + (size_t)cvl * R;
#pragma unroll
        for (int t = 0; t < R; ++t) dst[t] = o[t];
    }
}

// blockIdx.y: new patch; thread: one fine cell; the old patches are
// disjoint, so at most one covers the cell
__global__ __launch_bounds__(256) void k_copy_old(const double* __restrict__ fold,
                                                  const AmrPatch* __restrict__ old_patches, int nold,
                                                  const AmrPatch* __restrict__ new_patches,
                                                  double* __restrict__ fnew)
{
    const AmrPatch P = new_patches[blockIdx.y];
    const int q = (int)(blockIdx.x * 256 + threadIdx.x);
    if (q >= P.nx * P.nv) return;
    const int lx = q / P.nv, lv = q - (q / P.nv) * P.nv;
    const int gx = P.gx0 + lx, gv = P.gv0 + lv;
    for (int o = 0; o < nold; ++o) {
        const AmrPatch Q = old_patches[o];
        if (gx >= Q.gx0 && gx < Q.gx0 + Q.nx && gv >= Q.gv0 && gv < Q.gv0 + Q.nv) {
            fnew[P.off + q] = fold[Q.off + (size_t)(gx - Q.gx0) * Q.nv + (gv - Q.gv0)];
            return;
        }
    }
}

// ---- multi-level hierarchies

// the criterion on every cell of the listed patches of one level, its
// neighbours outside the patch read from the patch's ghost frame; tags and
// values land in the level's dense [nx_l][nv_l] arrays
__global__ __launch_bounds__(256) void k_hier_tag(const double* __restrict__ f, const double* __restrict__ frame,
                                                 const HPatch* __restrict__ patches, const int* __restrict__ list,
                                                 int nv_l, double dx, double dv, double tol,
                                                 uint8_t* __restrict__ tags, double* __restrict__ values)
{
    const HPatch P = patches[list[blockIdx.y]];
    const int q = (int)(blockIdx.x * 256 + threadIdx.x);
    if (q >= P.nx * P.nv) return;
    const int r = q / P.nv, c = q - (q / P.nv) * P.nv;
    const double* fp = f + P.off;
    const double* fr = frame + P.frame;
    const double* fc = fr + (size_t)4 * (P.nv + 4);
    const double cc = fp[q];
    const double xm = r > 0 ? fp[q - P.nv] : fr[(size_t)1 * (P.nv + 4) + c + 2];
    const double xp = r + 1 < P.nx ? fp[q + P.nv] : fr[(size_t)2 * (P.nv + 4) + c + 2];
    const double vm = c > 0 ? fp[q - 1] : fc[(size_t)r * 4 + 1];
    const double vp = c + 1 < P.nv ? fp[q + 1] : fc[(size_t)r * 4 + 2];
    const double t = tag_from(cc, xm, xp, vm, vp, dx, dv);
    const size_t o = (size_t)(P.gx0 + r) * nv_l + (P.gv0 + c);
    tags[o] = t > tol ? 1 : 0;
    if (values) values[o] = t;
}

// conservative limited WENO5 prolongation of the new parent level into the
// listed new patches of one level (x with RX, then v with RV): a thread per
// parent cell of a patch reads its 5 x 5 parent window from a source table
// (state element, or equilibrium value eqv[-1 - src]) and writes RX x RV
// fine cells

template <int RX, int RV>
__global__ __launch_bounds__(128) void k_hier_prolong(double* __restrict__ f, const int* __restrict__ win,
                                                     const HProlongPatch* __restrict__ pp,
                                                     const double* __restrict__ eqv)
{
    const HProlongPatch P = pp[blockIdx.y];
    const int q = (int)(blockIdx.x * 128 + threadIdx.x);
    if (q >= P.pcx * P.pcv) return;
    const int cxl = q / P.pcv, cvl = q - (q / P.pcv) * P.pcv;
    const int W = P.pcv + 4;
    const int* w0 = win + P.win + (size_t)cxl * W + cvl;   // window cell (cxl - 2 + 2, cvl - 2 + 2)
    auto val = [&](int a, int b) {
        const int s = w0[(size_t)a * W + b];
        return s >= 0 ? f[s] : eqv[-1 - s];
    };
    double T[RX][5];
#pragma unroll
    for (int e = 0; e < 5; ++e) {
        double u[5], o[RX];
#pragma unroll
        for (int k = 0; k < 5; ++k) u[k] = val(k, e);
        prolong1d<RX>(u, o);
#pragma unroll
        for (int s = 0; s < RX; ++s) T[s][e] = o[s];
    }
#pragma unroll
    for (int s = 0; s < RX; ++s) {
        double o[RV];
        prolong1d<RV>(T[s], o);
        double* dst = f + P.off + (size_t)(cxl * RX + s) * P.nv + (size_t)cvl * RV;
#pragma unroll
        for (int t = 0; t < RV; ++t) dst[t] = o[t];
    }
}

// old values into new patches: one block column per (new patch, old patch)
// intersection, copying its rows

__global__ __launch_bounds__(256) void k_hier_copy(double* __restrict__ fnew, const double* __restrict__ fold,
                                                  const HCopyBlock* __restrict__ blocks)
{
    const HCopyBlock B = blocks[blockIdx.y];
    const int q = (int)(blockIdx.x * 256 + threadIdx.x);
    if (q >= B.nx * B.nv) return;
    const int r = q / B.nv, c = q - (q / B.nv) * B.nv;
    fnew[B.dst + (size_t)r * B.dst_stride + c] = fold[B.src + (size_t)r * B.src_stride + c];
}

}  // namespace

hipError_t launch_tag4d(const Tag4DArgs& a, hipStream_t stream)
{
    const long long n = (long long)a.nx * a.ny * a.nvx * a.nvy;
    if (n == 0) return hipSuccess;
    if (n >= (1ll << 31) || a.nx * a.ny > 65535) return hipErrorInvalidValue;
    const int plane = a.nvx * a.nvy;
    const int nyb = (a.ny + kTag4DRows - 1) / kTag4DRows;
    const bool v4 = a.nvy % 4 == 0 && (reinterpret_cast<uintptr_t>(a.f) & 31) == 0 &&
                    (reinterpret_cast<uintptr_t>(a.tags) & 3) == 0 &&
                    (reinterpret_cast<uintptr_t>(a.values) & 31) == 0;
    if (v4)
        hipLaunchKernelGGL(k_tag4d_v4, dim3((unsigned)((plane / 4 + 255) / 256), (unsigned)(a.nx * nyb)), dim3(256),
                           0, stream, a);
    else
        hipLaunchKernelGGL(k_tag4d, dim3((unsigned)((plane + 255) / 256), (unsigned)(a.nx * nyb)), dim3(256), 0,
                           stream, a);
    return hipGetLastError();
}

hipError_t launch_tag(const double* f, int nx, int nv, const double* vg, double dx, double dv, double tol,
                      unsigned char* tags, double* values, hipStream_t stream)
{
    Ghosts g;
    for (int q = 0; q < 4; ++q) g.v[q] = vg[q];
    const bool al = (reinterpret_cast<uintptr_t>(f) % 16 == 0) && (reinterpret_cast<uintptr_t>(tags) % 4 == 0) &&
                    (!values || reinterpret_cast<uintptr_t>(values) % 16 == 0);
    if (nv % 4 == 0 && al) {
        const dim3 grid((unsigned)((nv / 4 + 255) / 256), (unsigned)((nx + kTagRows - 1) / kTagRows));
        hipLaunchKernelGGL(k_tag4, grid, dim3(256), 0, stream, f, nx, nv, g, dx, dv, tol,
                           reinterpret_cast<unsigned*>(tags), values);
    } else {
        const dim3 grid((unsigned)((nv + 255) / 256), (unsigned)nx);
        hipLaunchKernelGGL(k_tag, grid, dim3(256), 0, stream, f, nx, nv, g, dx, dv, tol, tags, values);
    }
    return hipGetLastError();
}

hipError_t launch_prolong(const double* fc, int ncx, int ncv, const double* vgc, int R, const AmrPatch* d_patches,
                          int npatch, int max_coarse_cells, double* fnew, hipStream_t stream)
{
    if (npatch == 0) return hipSuccess;
    Ghosts g;
    for (int q = 0; q < 4; ++q) g.v[q] = vgc[q];
    const dim3 grid((unsigned)((max_coarse_cells + 127) / 128), (unsigned)npatch);
    switch (R) {
    case 2: hipLaunchKernelGGL((k_prolong<2>), grid, dim3(128), 0, stream, fc, ncx, ncv, g, d_patches, fnew); break;
    case 4: hipLaunchKernelGGL((k_prolong<4>), grid, dim3(128), 0, stream, fc, ncx, ncv, g, d_patches, fnew); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_copy_old(const double* fold, const AmrPatch* d_old, int nold, const AmrPatch* d_new, int nnew,
                           int max_fine_cells, double* fnew, hipStream_t stream)
{
    if (nnew == 0 || nold == 0) return hipSuccess;
    const dim3 grid((unsigned)((max_fine_cells + 255) / 256), (unsigned)nnew);
    hipLaunchKernelGGL(k_copy_old, grid, dim3(256), 0, stream, fold, d_old, nold, d_new, fnew);
    return hipGetLastError();
}

hipError_t launch_hier_tag(const double* f, const double* frame, const HPatch* d_patches, const int* d_list, int n,
                           int max_cells, int nv_l, double dx, double dv, double tol, uint8_t* tags, double* values,
                           hipStream_t stream)
{
    if (n <= 0 || max_cells <= 0) return hipSuccess;
    const dim3 grid((unsigned)((max_cells + 255) / 256), (unsigned)n);
    hipLaunchKernelGGL(k_hier_tag, grid, dim3(256), 0, stream, f, frame, d_patches, d_list, nv_l, dx, dv, tol, tags,
                       values);
    return hipGetLastError();
}

hipError_t launch_hier_prolong(double* f, const int* d_win, const HProlongPatch* pp, int n, int max_parent_cells,
                               int rx, int rv, const double* eqv, hipStream_t stream)
{
    if (n <= 0 || max_parent_cells <= 0) return hipSuccess;
    const dim3 grid((unsigned)((max_parent_cells + 127) / 128), (unsigned)n), blk(128);
#define VP_HP(RX, RV)                                                                                   \
    if (rx == RX && rv == RV) {                                                                          \
        hipLaunchKernelGGL((k_hier_prolong<RX, RV>), grid, blk, 0, stream, f, d_win, pp, eqv);           \
        return hipGetLastError();                                                                        \
    }
    VP_HP(1, 2) VP_HP(1, 4) VP_HP(1, 8) VP_HP(2, 1) VP_HP(2, 2) VP_HP(2, 4) VP_HP(2, 8) VP_HP(4, 1) VP_HP(4, 2)
    VP_HP(4, 4) VP_HP(4, 8) VP_HP(8, 1) VP_HP(8, 2) VP_HP(8, 4) VP_HP(8, 8)
#undef VP_HP
    return hipErrorInvalidValue;
}

hipError_t launch_hier_copy(double* fnew, const double* fold, const HCopyBlock* d_blocks, int n, int max_cells,
                            hipStream_t stream)
{
    if (n <= 0 || max_cells <= 0) return hipSuccess;
    const dim3 grid((unsigned)((max_cells + 255) / 256), (unsigned)n);
    hipLaunchKernelGGL(k_hier_copy, grid, dim3(256), 0, stream, fnew, fold, d_blocks);
    return hipGetLastError();
}

}  // namespace vp
