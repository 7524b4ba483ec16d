// HIP kernels of the single-level 2D+2V path (FP64), f stored
// [x][y][vx][vy] with vy contiguous.
//
// Stage kernel: one wavefront per configuration cell (x, y) advances that
// cell's whole velocity plane.  Lane l owns the velocity column vy = l and
// the wave marches along vx.  With more than 64 cells along vy the plane is
// cut into segments of 60 columns, one block row per segment: lane l owns
// vy = 60 s - 2 + l, lanes 2 .. 61 produce the segment, and the two outer
// lanes on each side hold its neighbours or the equilibrium ghosts.  At
// each vx position the wave reads the rows of the nine planes of the stencil (the cell itself and its x +-1, +-2 and
// y +-1, +-2 neighbours), 64 contiguous doubles per row, from rows the
// block stages in LDS for its whole tile of cells.  Face averages along x
// and y are formed from those rows, faces along vx from a rolling window of
// the march, and faces along vy from neighbouring lanes (cross-lane
// permutes); the velocity ghosts are products of the 1D equilibrium cell
// averages.  The wave also sums its output plane, which gives the velocity
// moment of the configuration cell directly.
#include <hip/hip_runtime.h>
#include <type_traits>

#include "vp_internal.hpp"
#include "vp_stage_tile.hpp"

namespace vp {

namespace {

using namespace dev;

__device__ __forceinline__ double f4(double um1, double u0, double u1, double u2)
{
    return (7.0 * (u0 + u1) - (um1 + u2)) * (1.0 / 12.0);
}

// The fluxes enter the update only through differences across a cell, and
// face averages and product-rule corrections are linear in the cell
// values, so the wave combines before it differentiates:
//   x: Gx(x+1/2) - Gx(x-1/2) = vbar_x Dx + (dvx/24) (Dx(vx+1) - Dx(vx-1)),
//      Dx = (8 (f(x+1) - f(x-1)) - (f(x+2) - f(x-2))) / 12, the difference
//      of the two x-face averages;
//   y: the same with Dy and the vy neighbours (lanes);
//   vx: Gvx on a face is the face average along vx of
//      V = ax f + (dax_x (f(x+1) - f(x-1)) + dax_y (f(y+1) - f(y-1))) / 48;
//   vy: Gvy is the face average along vy of the corresponding U with ay.
// Ghost cells hold the equilibrium, which is the same in every plane, so
// V and U there reduce to ax g and ay g.
//
// A block owns a tile of TX x TY configuration cells, one wave per cell.
// At every vx position the block stages in LDS the rows of all planes its
// waves read: the tile and a cross-shaped halo two cells deep in x and in
// y, TX TY + 4 (TX + TY) rows, each loaded once per block (3 rows per cell
// for a 4 x 4 tile, where a wave loading its own nine rows would take 9).
// Each wave loads its share of the rows three positions ahead into
// registers (three register sets), stores the rows of the next position
// into a three-slot LDS ring after computing the current one, and the
// block meets at one barrier per position.  Waves whose cell lies past the
// mesh (partial tiles) load and wait like the others and store nothing.
// a double that is the same in every lane of the wave, in scalar registers
__device__ __forceinline__ double uniform_f64(double x)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// DPP wave shifts: lane l reads lane l + 1 (wave_shl:1) or lane l - 1
// (wave_shr:1); the lane with no source is overridden by the callers
constexpr int kLaneNext = 0x130;
constexpr int kLanePrev = 0x138;

template <int TX, int TY>
struct Tile4D {
    static constexpr int NW = TX * TY;                 // waves
    static constexpr int NP = NW + 4 * (TX + TY);      // plane rows per position
    static constexpr int LPW = (NP + NW - 1) / NW;     // rows loaded per wave per position
    // LDS row of plane (i, j) relative to the tile origin; (i, j) lies in the
    // tile or in its cross halo
    static __device__ __forceinline__ int pid(int i, int j)
    {
        if (i >= 0 && i < TX && j >= 0 && j < TY) return i * TY + j;
        if (j >= 0 && j < TY) return NW + (i < 0 ? i + 2 : i - TX + 2) * TY + j;
        return NW + 4 * TY + (j < 0 ? j + 2 : j - TY + 2) * TX + i;
    }
    // inverse of pid
    static __device__ __forceinline__ void plane_ij(int q, int& i, int& j)
    {
        if (q < NW) { i = q / TY; j = q - i * TY; return; }
        q -= NW;
        if (q < 4 * TY) { const int sd = q / TY; j = q - sd * TY; i = sd < 2 ? sd - 2 : TX + sd - 2; return; }
        q -= 4 * TY;
        const int sd = q / TX;
        i = q - sd * TX;
        j = sd < 2 ? sd - 2 : TY + sd - 2;
    }
};

template <int KIND, int TX, int TY, bool SV>
__global__ __launch_bounds__(64 * TX * TY) void k_stage4d(Stage4DArgs A)
{
    using TL = Tile4D<TX, TY>;
    constexpr int NP = TL::NP, LPW = TL::LPW, NW = TL::NW;
    static_assert(NP % NW == 0, "every wave loads the same number of ring rows");
    // ring slots = register sets = prefetch distance in positions
    constexpr bool NEED_FN = KIND == kStage23 || KIND == kLean2 || KIND == kLean3;
    constexpr bool NEED_AC = KIND == kStage23 || KIND == kStage4 || KIND == kLean4;
    constexpr int S = 3;
    __shared__ double rows[S][NP][64];
    __shared__ double gxs[kMaxVx4D + 4];               // vx equilibrium factors with ghosts
    __shared__ double gys[kMaxVy4D + 4];               // vy equilibrium factors with ghosts

    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int nx = A.nx, ny = A.ny, nvx = A.nvx, nvy = A.nvy;
    const int nty = (ny + TY - 1) / TY;
    const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int x0 = (tile / nty) * TX, y0 = (tile - (tile / nty) * nty) * TY;
    const int tx = wave / TY, ty = wave - (wave / TY) * TY;
    const int x = x0 + tx, y = y0 + ty;
    const bool cell_in = x < nx && y < ny;
    const size_t P = (size_t)nvx * nvy;
    auto cfg = [&](int xx, int yy) { return wrapi(xx, nx) * ny + wrapi(yy, ny); };
    // the lane's vy cell; act: the lane produces an output; vin: the lane
    // holds a mesh cell rather than a velocity ghost (segments only)
    const int seg = SV ? (int)blockIdx.y : 0;
    const int vyr = SV ? seg * kSegVy4D - 2 + lane : lane;
    const bool act = SV ? (lane >= 2 && lane < kSegVy4D + 2 && vyr < nvy) : lane < nvy;
    const bool vin = !SV || (vyr >= 0 && vyr < nvy);
    const int vyl = min(max(vyr, 0), nvy - 1);
    // rows this wave loads each position: planes wave, wave + NW, ...
    // (element offsets below 2^31: the plan limits the state to 2^31 elements)
    unsigned lpo[LPW];
#pragma unroll
    for (int k = 0; k < LPW; ++k) {
        int i = 0, j = 0;
        TL::plane_ij(wave + k * NW, i, j);
        lpo[k] = (unsigned)((size_t)cfg(x0 + i, y0 + j) * P + vyl);
    }
    for (int q = (int)threadIdx.x; q < nvx + 4; q += 64 * NW) gxs[q] = A.gx[q];
    if (!SV)
        for (int q = (int)threadIdx.x; q < nvy + 4; q += 64 * NW) gys[q] = A.gy[q];
    const double gyl = SV ? A.gy[min(max(vyr + 2, 0), nvy + 3)] : 0.0;   // the lane's vy equilibrium factor
    // rows this wave reads: c, x-1, x+1, y-1, y+1, x-2, x+2, y-2, y+2
    const int rp[9] = {TL::pid(tx, ty),     TL::pid(tx - 1, ty), TL::pid(tx + 1, ty),
                       TL::pid(tx, ty - 1), TL::pid(tx, ty + 1), TL::pid(tx - 2, ty),
                       TL::pid(tx + 2, ty), TL::pid(tx, ty - 2), TL::pid(tx, ty + 2)};
    const size_t po_c = (size_t)cfg(x, y) * P;

    const double* ax = A.a;
    const double* ay = A.a + nx * ny;
    // the wave's accelerations are the same in every lane: keep them in scalar registers
    const double axc = uniform_f64(ax[cfg(x, y)]),
                 cax_x = uniform_f64((ax[cfg(x + 1, y)] - ax[cfg(x - 1, y)]) * (1.0 / 48.0)),
                 cax_y = uniform_f64((ax[cfg(x, y + 1)] - ax[cfg(x, y - 1)]) * (1.0 / 48.0));
    const double ayc = uniform_f64(ay[cfg(x, y)]),
                 cay_x = uniform_f64((ay[cfg(x + 1, y)] - ay[cfg(x - 1, y)]) * (1.0 / 48.0)),
                 cay_y = uniform_f64((ay[cfg(x, y + 1)] - ay[cfg(x, y - 1)]) * (1.0 / 48.0));
    // vy equilibrium factor of vy cell j (-2 <= j < nvy + 2), staged in LDS
    auto gy_at = [&](int j) { return gys[min(max(j + 2, 0), nvy + 3)]; };
    const double vby = A.vy_lo + ((double)vyr + 0.5) * A.dvy;
    const double dxi = A.dxi, dyi = A.dyi, dvxi = A.dvxi, dvyi = A.dvyi, dvx24 = A.dvx24, dvy24 = A.dvy24;

    // sv = the value of lane + d of a per-lane quantity whose ghost value at
    // lane + d is gq * gy[lane + d]; lanes past the velocity range take the ghost
    // (segments: every lane holds its cell or ghost value, nothing to replace)
    auto nb = [&](double sv, int d, double gq) {
        if (SV) return sv;
        const int src = lane + d;
        return (src >= 0 && src < nvy) ? sv : gq * gy_at(src);
    };

    // Iteration m takes in position m - 2 (slot m mod S) and, from m = 4 on,
    // produces the output at position t = m - 4.  Loads are clamped to the
    // mesh so that they are unconditional (a load under a branch would be
    // waited for).
    const double* __restrict__ fs = A.fs;
    auto load_rows = [&](int m, double* dst) {
        const size_t o = (size_t)min(max(m - 2, 0), nvx - 1) * nvy;
#pragma unroll
        for (int k = 0; k < LPW; ++k) dst[k] = fs[lpo[k] + o];
    };
    auto store_rows = [&](int slot, const double* src) {
#pragma unroll
        for (int k = 0; k < LPW; ++k) rows[slot][wave + k * NW][lane] = src[k];
    };
    auto load_own = [&](int m, double& fnv, double& acv) {
        const size_t o = po_c + (size_t)min(max(m - 4, 0), nvx - 1) * nvy + vyl;
        if (NEED_FN) fnv = __builtin_nontemporal_load(A.fn + o);
        if (NEED_AC) acv = __builtin_nontemporal_load(A.acc + o);
    };

    // rolling state along vx: V at t-1 .. t+2, U, f and Dx at t-1/t .. t+2, Dy at t .. t+2
    double vw[4] = {0, 0, 0, 0}, uw[3] = {0, 0, 0}, cw[3] = {0, 0, 0}, dxw[4] = {0, 0, 0, 0}, dyw[3] = {0, 0, 0};
    auto shift_in = [&](int slot, int p) {
        double (*rs)[64] = rows[slot];
        const bool in = p >= 0 && p < nvx && vin;
        const double g = gxs[min(max(p + 2, 0), nvx + 3)] * (SV ? gyl : gy_at(lane));
        double v[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) v[q] = in ? rs[rp[q]][lane] : g;
        vw[0] = vw[1]; vw[1] = vw[2]; vw[2] = vw[3];
        vw[3] = axc * v[0] + (cax_x * (v[2] - v[1]) + cax_y * (v[4] - v[3]));
        uw[0] = uw[1]; uw[1] = uw[2];
        uw[2] = ayc * v[0] + (cay_x * (v[2] - v[1]) + cay_y * (v[4] - v[3]));
        cw[0] = cw[1]; cw[1] = cw[2]; cw[2] = v[0];
        dxw[0] = dxw[1]; dxw[1] = dxw[2]; dxw[2] = dxw[3];
        dxw[3] = (8.0 * (v[2] - v[1]) - (v[6] - v[5])) * (1.0 / 12.0);
        dyw[0] = dyw[1]; dyw[1] = dyw[2];
        dyw[2] = (8.0 * (v[4] - v[3]) - (v[8] - v[7])) * (1.0 / 12.0);
    };

    const int M = nvx + 4;
    double pr[S][LPW], fnr[S], acr[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        load_rows(q, pr[q]);
        fnr[q] = 0.0;
        acr[q] = 0.0;
    }
    store_rows(0, pr[0]);
    __syncthreads();

    double gvx_lo = 0.0, msum = 0.0;
    const double cacc = A.c_acc, cnext = A.c_next;
    // iteration m = m0 + SB uses slot and register set SB (m0 is a multiple
    // of S), so every slot and set index is a constant
    int m0 = 0;
    auto iter = [&](auto sbc) {
        constexpr int SB = decltype(sbc)::value;
        constexpr int sb = SB;
        constexpr int SN = (SB + 1) % S;
        const int m = m0 + SB;
        load_rows(m + S, pr[SB]);                        // set SB held the rows of m, stored at m - 1
        shift_in(SB, m - 2);
        if (m == 3) gvx_lo = f4(vw[0], vw[1], vw[2], vw[3]);   // face -1/2
        const int t = m - 4;
        if (t >= 0 && t < nvx) {                     // uniform
            const double gxt = gxs[t + 2];
            // x and y: differences of the face fluxes
            const double vbx = A.vx_lo + ((double)t + 0.5) * A.dvx;
            const double kx = (vbx * dxw[1] + dvx24 * (dxw[2] - dxw[0])) * dxi;
            const double dyn = dpp_f64<kLaneNext>(dyw[0]), dyp = dpp_f64<kLanePrev>(dyw[0]);
            const double ky = (vby * dyw[0] + dvy24 * (nb(dyn, 1, 0.0) - nb(dyp, -1, 0.0))) * dyi;
            // vx
            const double gvx_hi = f4(vw[0], vw[1], vw[2], vw[3]);
            // vy: upper face from lanes -1 .. +2; lower face from lane - 1 (lane 0: the box face)
            const double gu = ayc * gxt;
            const double u0 = uw[0];
            const double r1 = dpp_f64<kLaneNext>(u0), r2 = dpp_f64<kLaneNext>(r1), rm = dpp_f64<kLanePrev>(u0);
            const double um = nb(rm, -1, gu), u1 = nb(r1, 1, gu), u2 = nb(r2, 2, gu);
            const double gvy_hi = f4(um, u0, u1, u2);
            const double gvy_s = dpp_f64<kLanePrev>(gvy_hi);
            double gvy_lo = gvy_s;
            if (!SV) {
                const double gvy_b = f4(gu * gy_at(lane - 2), um, u0, u1);
                gvy_lo = lane == 0 ? gvy_b : gvy_s;
            }

            const double k = -kx - ky - (gvx_hi - gvx_lo) * dvxi - (gvy_hi - gvy_lo) * dvyi;
            gvx_lo = gvx_hi;

            const size_t o = po_c + (size_t)t * nvy + vyl;
            const bool st = act && cell_in;
            const double f0 = cw[0];                 // the stage state at the output position
            double out;
            if (KIND == kRhs) {
                out = k;
            } else if (KIND == kStage1) {
                out = f0 + cnext * k;
                if (st) __builtin_nontemporal_store(f0 + cacc * k, A.acc + o);
            } else if (KIND == kStage23) {
                out = fnr[sb] + cnext * k;
                if (st) __builtin_nontemporal_store(acr[sb] + cacc * k, A.acc + o);
            } else if (KIND == kStage4) {
                out = acr[sb] + cacc * k;
            } else if (KIND == kLean1) {
                out = f0 + cnext * k;
            } else if (KIND == kLean2) {
                out = fnr[sb] + cnext * k;
                if (st) __builtin_nontemporal_store((fnr[sb] + f0) * (1.0 / 3.0) + cacc * k, A.acc + o);
            } else if (KIND == kLean3) {
                out = fnr[sb] + cnext * k;
            } else {                                 // kLean4
                out = acr[sb] + (f0 * (1.0 / 3.0) + cacc * k);
            }
            if (st) __builtin_nontemporal_store(out, A.fout + o);
            if (act) msum += out;
        }
        load_own(m + S, fnr[sb], acr[sb]);           // for iteration m + S
        store_rows(SN, pr[SN]);                          // the rows of m + 1, loaded at m + 1 - S
        __syncthreads();
    };
#pragma unroll 1
    for (; m0 < M; m0 += S) {
        iter(std::integral_constant<int, 0>{});
        iter(std::integral_constant<int, 1>{});
        if constexpr (S == 3) iter(std::integral_constant<int, 2 % S>{});
    }
    if (KIND != kRhs && A.n && cell_in) {
        const double sm = wave_sum(msum);
        if (lane == 0) A.n[(size_t)seg * nx * ny + cfg(x, y)] = sm * A.mscale;   // a segment's share
    }
}

// n[e] = sum over the segments of their shares of the moment
__global__ __launch_bounds__(256) void k_sum_segments(double* __restrict__ n, int nseg, int ncfg)
{
    const int e = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (e >= ncfg) return;
    double s = n[e];
    for (int q = 1; q < nseg; ++q) s += n[(size_t)q * ncfg + e];
    n[e] = s;
}

// n = dvx dvy sum over the velocity plane, one wave per configuration cell
__global__ __launch_bounds__(256) void k_moment4d(const double* __restrict__ f, int ncfg, size_t plane,
                                                 double scale, double* __restrict__ n)
{
    const int cell = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (cell >= ncfg) return;
    const double* p = f + (size_t)cell * plane;
    double s = 0.0;
    for (size_t q = lane; q < plane; q += 64) s += p[q];
    s = wave_sum(s);
    if (lane == 0) n[cell] = s * scale;
}

// ---------------------------------------------------------------- 2D Poisson
//
// Periodic Poisson problem of the summed 1D fourth-order operators, solved
// in the real orthonormal Fourier basis Q (columns = basis vectors) that
// diagonalises every symmetric circulant matrix:
//   g = (Qx^T rho Qy) / lambda (zero mode dropped),  phi = Qx g Qy^T,
// then E = -D phi per direction and a = (q/m) E.  Two launches of one
// block per row (nx, ny <= 64; larger meshes below): the forward transform of one Fourier row,
// then the inverse transform of five x rows and the field of the middle
// one.  Rows computed by several blocks are computed identically.

constexpr int kP2 = kPoisson2DSmall;        // 64: rows and columns per matrix at most
constexpr int kP2Q = 256 / kP2;             // 4 groups of 64 threads split each sum

// block k: g[k][l] = invlam(k, l) sum_j (sum_i Qx[i][k] rho'[i][j]) Qy[j][l],
// rho' = rho - mean(rho) = mean(n) - n
__global__ __launch_bounds__(256) void k_poisson2d_fwd(const double* __restrict__ n, int nx, int ny,
                                                      const double* __restrict__ Qx,
                                                      const double* __restrict__ Qy,
                                                      const double* __restrict__ invlamT, double* __restrict__ g)
{
    constexpr int SEG = kP2 / kP2Q;          // 16 terms of a sum per thread
    __shared__ double part[kP2Q][kP2];
    __shared__ double w[kP2];
    __shared__ double red[256 / 64];
    const int t = threadIdx.x, lane = t & 63, q = t >> 6;
    const int k = blockIdx.x;
    const int N = nx * ny;
    // every load of the block in flight together: the mean's share, the
    // rho column j = lane for rows i in [SEG q, SEG q + SEG), and Qx[i][k]
    double vm[kP2 * kP2 / 256], vn[SEG], vq[SEG], vy[SEG];
#pragma unroll
    for (int r = 0; r < kP2 * kP2 / 256; ++r) {
        const int e = t + r * 256;
        vm[r] = e < N ? n[e] : 0.0;
    }
    const int j = lane;
#pragma unroll
    for (int u = 0; u < SEG; ++u) {
        const int i = q * SEG + u;
        const bool in = i < nx && j < ny;
        vn[u] = in ? n[i * ny + j] : 0.0;
        vq[u] = i < nx ? Qx[i * nx + k] : 0.0;
        const int jj = q * SEG + u;              // step 2: Qy[jj][l = lane]
        vy[u] = (jj < ny && lane < ny) ? Qy[jj * ny + lane] : 0.0;
    }
    double sm = 0.0;
#pragma unroll
    for (int r = 0; r < kP2 * kP2 / 256; ++r) sm += vm[r];
    sm = wave_sum(sm);
    if (lane == 0) red[q] = sm;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int r = 0; r < 256 / 64; ++r) tot += red[r];
    const double mean = tot / N;
    // w[j] = sum_i Qx[i][k] rho'[i][j]
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < SEG; ++u) acc += vq[u] * (mean - vn[u]);
    part[q][lane] = acc;
    __syncthreads();
    if (t < kP2) w[t] = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
    __syncthreads();
    // g[k][l] = invlam * sum_j w[j] Qy[j][l], l = lane
    acc = 0.0;
#pragma unroll
    for (int u = 0; u < SEG; ++u) acc += w[q * SEG + u] * vy[u];
    part[q][lane] = acc;
    __syncthreads();
    if (t < ny) {
        const double s2 = ((part[0][t] + part[1][t]) + part[2][t]) + part[3][t];
        g[k * ny + t] = s2 * invlamT[t * nx + k];
    }
}

// block b: phi at rows R b - 2 .. R b + R + 1 (periodic), phi[i'][j] =
// sum_l h[i'][l] Qy[j][l] with h[i'][l] = sum_k Qx[i'][k] g[k][l]; then E
// and a at rows R b .. R b + R - 1.  R > 1 (the fine configuration mesh of a
// two-level hierarchy of ratio R): also the coarse a of coarse row b, the
// mean of the R x R fine values over each coarse cell.
template <int R>
__global__ __launch_bounds__(256) void k_poisson2d_inv(const double* __restrict__ g, int nx, int ny, double dx,
                                                      double dy, double qm, const double* __restrict__ Qx,
                                                      const double* __restrict__ Qy, double* __restrict__ phi_out,
                                                      double* __restrict__ E_out, double* __restrict__ a_out,
                                                      double* __restrict__ a_coarse)
{
    constexpr int SEG = kP2 / kP2Q;
    constexpr int NR = R + 4;                    // potential rows of the block
    __shared__ double part[kP2Q][NR][kP2];
    __shared__ double h[NR][kP2];
    __shared__ double ph[NR][kP2];
    __shared__ double qx[NR][kP2];
    __shared__ double af[2][R][kP2];
    const int t = threadIdx.x, lane = t & 63, q = t >> 6;
    const int i0 = (int)blockIdx.x * R;
    const int N = nx * ny;
    // Qx rows i0-2 .. i0+R+1 into LDS; g column l = lane for k in [SEG q, SEG q + SEG);
    // Qy[j = lane][l] for l in [SEG q, SEG q + SEG)
    for (int e = t; e < NR * kP2; e += 256) {
        const int r = e / kP2, kk = e - r * kP2;
        qx[r][kk] = kk < nx ? Qx[wrapi(i0 - 2 + r, nx) * nx + kk] : 0.0;
    }
    double vg[SEG], vy[SEG];
#pragma unroll
    for (int u = 0; u < SEG; ++u) {
        const int kk = q * SEG + u;
        vg[u] = (kk < nx && lane < ny) ? g[kk * ny + lane] : 0.0;
        const int l = q * SEG + u;
        vy[u] = (l < ny && lane < ny) ? Qy[lane * ny + l] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < SEG; ++u) acc += qx[r][q * SEG + u] * vg[u];
        part[q][r][lane] = acc;
    }
    __syncthreads();
    for (int e = t; e < NR * kP2; e += 256) {
        const int r = e / kP2, l = e - r * kP2;
        h[r][l] = ((part[0][r][l] + part[1][r][l]) + part[2][r][l]) + part[3][r][l];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < SEG; ++u) acc += h[r][q * SEG + u] * vy[u];
        part[q][r][lane] = acc;
    }
    __syncthreads();
    for (int e = t; e < NR * kP2; e += 256) {
        const int r = e / kP2, jj = e - r * kP2;
        ph[r][jj] = ((part[0][r][jj] + part[1][r][jj]) + part[2][r][jj]) + part[3][r][jj];
    }
    __syncthreads();
    for (int e = t; e < R * ny; e += 256) {
        const int rr = e / ny, jj = e - rr * ny;
        const int c = rr + 2;                    // the row's potential row
        const int jp1 = wrapi(jj + 1, ny), jm1 = wrapi(jj - 1, ny), jp2 = wrapi(jj + 2, ny), jm2 = wrapi(jj - 2, ny);
        const double cx = 1.0 / (12.0 * dx), cy = 1.0 / (12.0 * dy);
        const double ex = -(8.0 * (ph[c + 1][jj] - ph[c - 1][jj]) - (ph[c + 2][jj] - ph[c - 2][jj])) * cx;
        const double ey = -(8.0 * (ph[c][jp1] - ph[c][jm1]) - (ph[c][jp2] - ph[c][jm2])) * cy;
        const int o = (i0 + rr) * ny + jj;
        if (phi_out) phi_out[o] = ph[c][jj];
        if (E_out) { E_out[o] = ex; E_out[N + o] = ey; }
        if (a_out) { a_out[o] = qm * ex; a_out[N + o] = qm * ey; }
        if (R > 1) { af[0][rr][jj] = qm * ex; af[1][rr][jj] = qm * ey; }
    }
    if (R > 1) {
        __syncthreads();
        const int ncy = ny / R, nc = (nx / R) * ncy;
        for (int e = t; e < 2 * ncy; e += 256) {
            const int comp = e / ncy, jc = e - comp * ncy;
            double s = 0.0;
#pragma unroll
            for (int u = 0; u < R; ++u)
#pragma unroll
                for (int w = 0; w < R; ++w) s += af[comp][u][jc * R + w];
            a_coarse[comp * nc + (int)blockIdx.x * ncy + jc] = s / (R * R);
        }
    }
}

// ---------------------------------------------------------------- 2D Poisson, larger meshes
//
// The same solve for meshes of more than 64 cells in x or y (up to 256):
// one block per Fourier row computes g[k][:] = -(Qx^T n Qy)[k][:] / lambda
// (the mean of n lies in the zero mode, which is dropped), one block per x
// row the potential phi[i][:] = (Qx g Qy^T)[i][:], then one thread per cell
// the field.  QyT holds Qy transposed so that every inner loop reads
// consecutive doubles across the threads.
__global__ __launch_bounds__(256) void k_poisson2d_fwd_l(const double* __restrict__ n, int nx, int ny,
                                                        const double* __restrict__ Qx, const double* __restrict__ Qy,
                                                        const double* __restrict__ invlamT, double* __restrict__ g)
{
    __shared__ double w[kMaxPoisson2D];
    const int k = blockIdx.x, t = threadIdx.x;
    if (t < ny) {
        double acc = 0.0;
        for (int i = 0; i < nx; ++i) acc += Qx[i * nx + k] * n[i * ny + t];
        w[t] = acc;
    }
    __syncthreads();
    if (t < ny) {
        double acc = 0.0;
        for (int j = 0; j < ny; ++j) acc += w[j] * Qy[j * ny + t];
        g[k * ny + t] = -acc * invlamT[t * nx + k];
    }
}

__global__ __launch_bounds__(256) void k_poisson2d_inv_l(const double* __restrict__ g, int nx, int ny,
                                                        const double* __restrict__ Qx, const double* __restrict__ QyT,
                                                        double* __restrict__ phi)
{
    __shared__ double h[kMaxPoisson2D];
    const int i = blockIdx.x, t = threadIdx.x;
    if (t < ny) {
        double acc = 0.0;
        for (int k = 0; k < nx; ++k) acc += Qx[i * nx + k] * g[k * ny + t];
        h[t] = acc;
    }
    __syncthreads();
    if (t < ny) {
        double acc = 0.0;
        for (int l = 0; l < ny; ++l) acc += h[l] * QyT[l * ny + t];
        phi[i * ny + t] = acc;
    }
}

__global__ __launch_bounds__(256) void k_field2d_l(const double* __restrict__ ph, int nx, int ny, double dx,
                                                  double dy, double qm, double* __restrict__ phi_out,
                                                  double* __restrict__ E_out, double* __restrict__ a_out)
{
    const int e = (int)blockIdx.x * 256 + (int)threadIdx.x;
    const int N = nx * ny;
    if (e >= N) return;
    const int i = e / ny, j = e - (e / ny) * ny;
    auto at = [&](int ii, int jj) { return ph[wrapi(ii, nx) * ny + wrapi(jj, ny)]; };
    const double ex = -(8.0 * (at(i + 1, j) - at(i - 1, j)) - (at(i + 2, j) - at(i - 2, j))) / (12.0 * dx);
    const double ey = -(8.0 * (at(i, j + 1) - at(i, j - 1)) - (at(i, j + 2) - at(i, j - 2))) / (12.0 * dy);
    if (phi_out) phi_out[e] = ph[e];
    if (E_out) { E_out[e] = ex; E_out[N + e] = ey; }
    if (a_out) { a_out[e] = qm * ex; a_out[N + e] = qm * ey; }
}

template <int KIND, bool SV>
hipError_t launch_stage4d_t(int tx, int ty, const Stage4DArgs& a, hipStream_t stream)
{
    const int nseg = SV ? (a.nvy + kSegVy4D - 1) / kSegVy4D : 1;
    const dim3 g((unsigned)(((a.nx + tx - 1) / tx) * ((a.ny + ty - 1) / ty)), (unsigned)nseg);
    if (tx == 4 && ty == 4) hipLaunchKernelGGL((k_stage4d<KIND, 4, 4, SV>), g, dim3(1024), 0, stream, a);
    else if (tx == 2 && ty == 4) hipLaunchKernelGGL((k_stage4d<KIND, 2, 4, SV>), g, dim3(512), 0, stream, a);
    else if (tx == 4 && ty == 2) hipLaunchKernelGGL((k_stage4d<KIND, 4, 2, SV>), g, dim3(512), 0, stream, a);
    else if (tx == 2 && ty == 2) hipLaunchKernelGGL((k_stage4d<KIND, 2, 2, SV>), g, dim3(256), 0, stream, a);
    else return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && SV && KIND != kRhs && a.n) {
        const int ncfg = a.nx * a.ny;
        hipLaunchKernelGGL(k_sum_segments, dim3((ncfg + 255) / 256), dim3(256), 0, stream, a.n, nseg, ncfg);
        e = hipGetLastError();
    }
    return e;
}

template <int KIND>
hipError_t launch_stage4d_k(int tx, int ty, const Stage4DArgs& a, hipStream_t stream)
{
    return a.nvy > kMaxVy4D ? launch_stage4d_t<KIND, true>(tx, ty, a, stream)
                            : launch_stage4d_t<KIND, false>(tx, ty, a, stream);
}

}  // namespace

hipError_t launch_stage4d(int tx, int ty, int kind, const Stage4DArgs& a, hipStream_t stream)
{
    switch (kind) {
    case kRhs: return launch_stage4d_k<kRhs>(tx, ty, a, stream);
    case kLean1: return launch_stage4d_k<kLean1>(tx, ty, a, stream);
    case kLean2: return launch_stage4d_k<kLean2>(tx, ty, a, stream);
    case kLean3: return launch_stage4d_k<kLean3>(tx, ty, a, stream);
    case kLean4: return launch_stage4d_k<kLean4>(tx, ty, a, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_moment4d(const double* f, int ncfg, size_t plane, double scale, double* n, hipStream_t stream)
{
    hipLaunchKernelGGL(k_moment4d, dim3((ncfg + 3) / 4), dim3(256), 0, stream, f, ncfg, plane, scale, n);
    return hipGetLastError();
}

hipError_t launch_poisson2d(const double* n, int nx, int ny, double dx, double dy, double qm, const double* Qx,
                            const double* Qy, const double* invlamT, double* g, double* phi, double* E, double* a,
                            hipStream_t stream)
{
    return launch_poisson2d_coarse(n, nx, ny, dx, dy, qm, Qx, Qy, invlamT, g, phi, E, a, 1, nullptr, stream);
}

hipError_t launch_poisson2d_coarse(const double* n, int nx, int ny, double dx, double dy, double qm,
                                   const double* Qx, const double* Qy, const double* invlamT, double* g, double* phi,
                                   double* E, double* a, int R, double* a_coarse, hipStream_t stream)
{
    if (nx > kMaxPoisson2D || ny > kMaxPoisson2D || nx < 1 || ny < 1 || !g) return hipErrorInvalidValue;
    if (a_coarse && ((R != 2 && R != 4) || nx % R || ny % R || nx > kPoisson2DSmall || ny > kPoisson2DSmall))
        return hipErrorInvalidValue;
    if (nx <= kPoisson2DSmall && ny <= kPoisson2DSmall) {
        hipLaunchKernelGGL(k_poisson2d_fwd, dim3(nx), dim3(256), 0, stream, n, nx, ny, Qx, Qy, invlamT, g);
        if (!a_coarse)
            hipLaunchKernelGGL(k_poisson2d_inv<1>, dim3(nx), dim3(256), 0, stream, g, nx, ny, dx, dy, qm, Qx, Qy, phi,
                               E, a, nullptr);
        else if (R == 2)
            hipLaunchKernelGGL(k_poisson2d_inv<2>, dim3(nx / 2), dim3(256), 0, stream, g, nx, ny, dx, dy, qm, Qx, Qy,
                               phi, E, a, a_coarse);
        else
            hipLaunchKernelGGL(k_poisson2d_inv<4>, dim3(nx / 4), dim3(256), 0, stream, g, nx, ny, dx, dy, qm, Qx, Qy,
                               phi, E, a, a_coarse);
        return hipGetLastError();
    }
    // g holds the coefficients, then the potential; Qy is followed by its transpose
    const int N = nx * ny;
    double* ph = g + N;
    hipLaunchKernelGGL(k_poisson2d_fwd_l, dim3(nx), dim3(256), 0, stream, n, nx, ny, Qx, Qy, invlamT, g);
    hipLaunchKernelGGL(k_poisson2d_inv_l, dim3(nx), dim3(256), 0, stream, g, nx, ny, Qx, Qy + (size_t)ny * ny, ph);
    hipLaunchKernelGGL(k_field2d_l, dim3((N + 255) / 256), dim3(256), 0, stream, ph, nx, ny, dx, dy, qm, phi, E, a);
    return hipGetLastError();
}

}  // namespace vp
