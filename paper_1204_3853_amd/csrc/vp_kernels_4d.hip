// HIP kernels of the single-level 2D+2V path (FP64), f stored
// [x][y][vx][vy] with vy contiguous.
//
// Stage kernel: one wavefront per configuration cell (x, y) advances that
// cell's whole velocity plane.  Lane l owns the velocity column vy = l and
// the wave marches along vx; at each vx position it loads the rows of the
// nine planes of the stencil (the cell itself and its x +-1, +-2 and
// y +-1, +-2 neighbours), 64 contiguous doubles per row.  Face averages
// along x and y are formed from those rows, faces along vx from a rolling
// window of the march, and faces along vy from neighbouring lanes
// (cross-lane permutes); the velocity ghosts are products of the 1D
// equilibrium cell averages.  The wave also sums its output plane, which
// gives the velocity moment of the configuration cell directly.
#include <hip/hip_runtime.h>

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
// The march is software-pipelined: the rows of NB - 1 positions ahead of
// the one being consumed are in flight while a position is computed.
template <int KIND, int NB>
__global__ __launch_bounds__(256) void k_stage4d(Stage4DArgs A)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int cell = xcd_remap((int)blockIdx.x, (int)gridDim.x) * 4 + wave;
    const int nx = A.nx, ny = A.ny, nvx = A.nvx, nvy = A.nvy;
    if (cell >= nx * ny) return;                        // uniform per wave; the kernel has no block barrier
    const int x = cell / ny, y = cell - (cell / ny) * ny;
    const size_t P = (size_t)nvx * nvy;
    auto cfg = [&](int xx, int yy) { return wrapi(xx, nx) * ny + wrapi(yy, ny); };
    // the nine planes: c, x-1, x+1, y-1, y+1, x-2, x+2, y-2, y+2
    const size_t po[9] = {(size_t)cfg(x, y) * P,     (size_t)cfg(x - 1, y) * P, (size_t)cfg(x + 1, y) * P,
                          (size_t)cfg(x, y - 1) * P, (size_t)cfg(x, y + 1) * P, (size_t)cfg(x - 2, y) * P,
                          (size_t)cfg(x + 2, y) * P, (size_t)cfg(x, y - 2) * P, (size_t)cfg(x, y + 2) * P};
    const double* __restrict__ fs = A.fs;
    const double* ax = A.a;
    const double* ay = A.a + nx * ny;
    const double axc = ax[cfg(x, y)], cax_x = (ax[cfg(x + 1, y)] - ax[cfg(x - 1, y)]) * (1.0 / 48.0),
                 cax_y = (ax[cfg(x, y + 1)] - ax[cfg(x, y - 1)]) * (1.0 / 48.0);
    const double ayc = ay[cfg(x, y)], cay_x = (ay[cfg(x + 1, y)] - ay[cfg(x - 1, y)]) * (1.0 / 48.0),
                 cay_y = (ay[cfg(x, y + 1)] - ay[cfg(x, y - 1)]) * (1.0 / 48.0);

    const bool act = lane < nvy;
    const int vyl = act ? lane : nvy - 1;
    double gyd[5];                                      // vy equilibrium factors at lane - 2 .. lane + 2
#pragma unroll
    for (int d = 0; d < 5; ++d) gyd[d] = A.gy[min(max(lane + d, 0), nvy + 3)];
    const double gyl = gyd[2];
    const double vby = A.vy_lo + ((double)lane + 0.5) * A.dvy;
    const double dxi = A.dxi, dyi = A.dyi, dvxi = A.dvxi, dvyi = A.dvyi, dvx24 = A.dvx24, dvy24 = A.dvy24;

    // lane + d of a per-lane quantity whose ghost value at lane + d is gq * gy[lane + d]
    auto nb = [&](double u, int d, double gq) {
        const double s = __shfl(u, lane + d, 64);
        const int src = lane + d;
        return (src >= 0 && src < nvy) ? s : gq * gyd[d + 2];
    };

    double Lb[NB][9], FNb[NB], ACb[NB];
    // loads of lead position p (and of f^n / acc at the output position p - 2) into slot s
    auto issue = [&](int p, int s) {
        const int pc = min(max(p, 0), nvx - 1);
        const size_t o = (size_t)pc * nvy + vyl;
#pragma unroll
        for (int q = 0; q < 9; ++q) Lb[s][q] = fs[po[q] + o];
        const size_t oo = po[0] + (size_t)min(max(p - 2, 0), nvx - 1) * nvy + vyl;
        if (KIND == kStage23) FNb[s] = __builtin_nontemporal_load(A.fn + oo);
        if (KIND == kStage23 || KIND == kStage4) ACb[s] = __builtin_nontemporal_load(A.acc + oo);
    };

    // rolling state along vx: V at t-1 .. t+2, U, f and Dx at t-1/t .. t+2, Dy at t .. t+2
    double vw[4] = {0, 0, 0, 0}, uw[3] = {0, 0, 0}, cw[3] = {0, 0, 0}, dxw[4] = {0, 0, 0, 0}, dyw[3] = {0, 0, 0};
    auto shift_in = [&](const double* r, int p) {
        const bool in = p >= 0 && p < nvx;
        const double g = A.gx[min(max(p + 2, 0), nvx + 3)] * gyl;
        double v[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) v[q] = in ? r[q] : g;
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

#pragma unroll
    for (int p = -2; p <= 1; ++p) {
        issue(p, 0);
        shift_in(Lb[0], p);
    }
    double gvx_lo = f4(vw[0], vw[1], vw[2], vw[3]);      // face -1/2
    double msum = 0.0;
    const double cacc = A.c_acc, cnext = A.c_next;
#pragma unroll
    for (int s = 0; s < NB - 1; ++s) issue(2 + s, s);

#pragma unroll 1
    for (int tb = 0; tb < nvx; tb += NB) {
#pragma unroll
        for (int s = 0; s < NB; ++s) {
            const int t = tb + s;
            issue(t + 2 + NB - 1, (s + NB - 1) % NB);
            shift_in(Lb[s], t + 2);
            if (t >= nvx) continue;                      // uniform
            const double gxt = A.gx[t + 2];
            // x and y: differences of the face fluxes
            const double vbx = A.vx_lo + ((double)t + 0.5) * A.dvx;
            const double kx = (vbx * dxw[1] + dvx24 * (dxw[2] - dxw[0])) * dxi;
            const double ky = (vby * dyw[0] + dvy24 * (nb(dyw[0], 1, 0.0) - nb(dyw[0], -1, 0.0))) * dyi;
            // vx
            const double gvx_hi = f4(vw[0], vw[1], vw[2], vw[3]);
            // vy: upper face from lanes -1 .. +2; lower face from lane - 1 (lane 0: the box face)
            const double gu = ayc * gxt;
            const double u0 = uw[0];
            const double um = nb(u0, -1, gu), u1 = nb(u0, 1, gu), u2 = nb(u0, 2, gu);
            const double gvy_hi = f4(um, u0, u1, u2);
            const double gvy_b = f4(gu * gyd[0], um, u0, u1);
            const double gvy_s = __shfl(gvy_hi, lane - 1, 64);
            const double gvy_lo = lane == 0 ? gvy_b : gvy_s;

            const double k = -kx - ky - (gvx_hi - gvx_lo) * dvxi - (gvy_hi - gvy_lo) * dvyi;
            gvx_lo = gvx_hi;

            const size_t o = po[0] + (size_t)t * nvy + lane;
            double out;
            if (KIND == kRhs) {
                out = k;
                if (act) __builtin_nontemporal_store(out, A.fout + o);
            } else if (KIND == kStage1) {
                const double f0 = cw[0];
                out = f0 + cnext * k;
                if (act) {
                    __builtin_nontemporal_store(f0 + cacc * k, A.acc + o);
                    __builtin_nontemporal_store(out, A.fout + o);
                }
            } else if (KIND == kStage23) {
                out = FNb[s] + cnext * k;
                if (act) {
                    __builtin_nontemporal_store(ACb[s] + cacc * k, A.acc + o);
                    __builtin_nontemporal_store(out, A.fout + o);
                }
            } else {
                out = ACb[s] + cacc * k;
                if (act) __builtin_nontemporal_store(out, A.fout + o);
            }
            if (act) msum += out;
        }
    }
    if (KIND != kRhs && A.n) {
        const double s = wave_sum(msum);
        if (lane == 0) A.n[cell] = s * A.mscale;
    }
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
// block per row (nx, ny <= 64): the forward transform of one Fourier row,
// then the inverse transform of five x rows and the field of the middle
// one.  Rows computed by several blocks are computed identically.

constexpr int kP2 = kMaxPoisson2D;          // 64: rows and columns per matrix at most
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

// block i: phi at rows i-2 .. i+2 (periodic), phi[i'][j] = sum_l h[i'][l] Qy[j][l]
// with h[i'][l] = sum_k Qx[i'][k] g[k][l]; then E and a at row i
__global__ __launch_bounds__(256) void k_poisson2d_inv(const double* __restrict__ g, int nx, int ny, double dx,
                                                      double dy, double qm, const double* __restrict__ Qx,
                                                      const double* __restrict__ Qy, double* __restrict__ phi_out,
                                                      double* __restrict__ E_out, double* __restrict__ a_out)
{
    constexpr int SEG = kP2 / kP2Q;
    __shared__ double part[kP2Q][5][kP2];
    __shared__ double h[5][kP2];
    __shared__ double ph[5][kP2];
    __shared__ double qx[5][kP2];
    const int t = threadIdx.x, lane = t & 63, q = t >> 6;
    const int i = blockIdx.x;
    const int N = nx * ny;
    // Qx rows i-2 .. i+2 into LDS; g column l = lane for k in [SEG q, SEG q + SEG);
    // Qy[j = lane][l] for l in [SEG q, SEG q + SEG)
    for (int e = t; e < 5 * kP2; e += 256) {
        const int r = e / kP2, kk = e - r * kP2;
        qx[r][kk] = kk < nx ? Qx[wrapi(i - 2 + r, nx) * nx + kk] : 0.0;
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
    for (int r = 0; r < 5; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < SEG; ++u) acc += qx[r][q * SEG + u] * vg[u];
        part[q][r][lane] = acc;
    }
    __syncthreads();
    for (int e = t; e < 5 * kP2; e += 256) {
        const int r = e / kP2, l = e - r * kP2;
        h[r][l] = ((part[0][r][l] + part[1][r][l]) + part[2][r][l]) + part[3][r][l];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < SEG; ++u) acc += h[r][q * SEG + u] * vy[u];
        part[q][r][lane] = acc;
    }
    __syncthreads();
    for (int e = t; e < 5 * kP2; e += 256) {
        const int r = e / kP2, jj = e - r * kP2;
        ph[r][jj] = ((part[0][r][jj] + part[1][r][jj]) + part[2][r][jj]) + part[3][r][jj];
    }
    __syncthreads();
    if (t < ny) {
        const int jj = t;
        const int jp1 = wrapi(jj + 1, ny), jm1 = wrapi(jj - 1, ny), jp2 = wrapi(jj + 2, ny), jm2 = wrapi(jj - 2, ny);
        const double cx = 1.0 / (12.0 * dx), cy = 1.0 / (12.0 * dy);
        const double ex = -(8.0 * (ph[3][jj] - ph[1][jj]) - (ph[4][jj] - ph[0][jj])) * cx;
        const double ey = -(8.0 * (ph[2][jp1] - ph[2][jm1]) - (ph[2][jp2] - ph[2][jm2])) * cy;
        const int e = i * ny + jj;
        if (phi_out) phi_out[e] = ph[2][jj];
        if (E_out) { E_out[e] = ex; E_out[N + e] = ey; }
        if (a_out) { a_out[e] = qm * ex; a_out[N + e] = qm * ey; }
    }
}

template <int KIND>
hipError_t launch_stage4d_k(int rb, const Stage4DArgs& a, hipStream_t stream)
{
    const int ncfg = a.nx * a.ny;
    const dim3 g((ncfg + 3) / 4), b(256);
    switch (rb) {
    case 1: hipLaunchKernelGGL((k_stage4d<KIND, 2>), g, b, 0, stream, a); break;
    case 2: hipLaunchKernelGGL((k_stage4d<KIND, 3>), g, b, 0, stream, a); break;
    case 4: hipLaunchKernelGGL((k_stage4d<KIND, 4>), g, b, 0, stream, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stage4d(int rb, int kind, const Stage4DArgs& a, hipStream_t stream)
{
    switch (kind) {
    case kRhs: return launch_stage4d_k<kRhs>(rb, a, stream);
    case kStage1: return launch_stage4d_k<kStage1>(rb, a, stream);
    case kStage23: return launch_stage4d_k<kStage23>(rb, a, stream);
    default: return launch_stage4d_k<kStage4>(rb, a, stream);
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
    if (nx > kMaxPoisson2D || ny > kMaxPoisson2D || !g) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_poisson2d_fwd, dim3(nx), dim3(256), 0, stream, n, nx, ny, Qx, Qy, invlamT, g);
    hipLaunchKernelGGL(k_poisson2d_inv, dim3(nx), dim3(256), 0, stream, g, nx, ny, dx, dy, qm, Qx, Qy, phi, E, a);
    return hipGetLastError();
}

}  // namespace vp
