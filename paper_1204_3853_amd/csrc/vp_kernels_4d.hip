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

template <int KIND, int RB>
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
    const double axc = ax[cfg(x, y)], dax_x = ax[cfg(x + 1, y)] - ax[cfg(x - 1, y)],
                 dax_y = ax[cfg(x, y + 1)] - ax[cfg(x, y - 1)];
    const double ayc = ay[cfg(x, y)], day_x = ay[cfg(x + 1, y)] - ay[cfg(x - 1, y)],
                 day_y = ay[cfg(x, y + 1)] - ay[cfg(x, y - 1)];

    const bool act = lane < nvy;
    const int vyl = act ? lane : nvy - 1;
    // 1D equilibrium factors along vy at lane + d, d = -2..2 (used where lane + d is a ghost)
    double gyd[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) gyd[d] = A.gy[min(max(lane + d, 0), nvy + 3)];
    const double gyl = gyd[2];
    const double vby = A.vy_lo + ((double)lane + 0.5) * A.dvy;
    const double dxi = A.dxi, dyi = A.dyi, dvxi = A.dvxi, dvyi = A.dvyi, dvx24 = A.dvx24, dvy24 = A.dvy24;

    // value of lane + d of a row at a vx position whose equilibrium factor is gq
    auto nb = [&](double u, int d, double gq) {
        const double s = __shfl(u, lane + d, 64);
        const int src = lane + d;
        return (src >= 0 && src < nvy) ? s : gq * gyd[d + 2];
    };
    // rows of the nine planes at vx position p (equilibrium products outside the velocity box)
    auto ld9 = [&](int p, double* v) {
        const int pc = min(max(p, 0), nvx - 1);
        const size_t o = (size_t)pc * nvy + vyl;
        double r[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) r[q] = fs[po[q] + o];
        const bool in = p >= 0 && p < nvx;
        const double g = A.gx[min(p + 2, nvx + 3)] * gyl;
#pragma unroll
        for (int q = 0; q < 9; ++q) v[q] = in ? r[q] : g;
    };

    // rolling state: rows at t-1 .. t+2 of the five planes used along vx and vy,
    // x-face averages at t-1 .. t+2, y-face averages at t .. t+2
    double w[5][4], fxl[4], fxh[4], fyl[3], fyh[3];
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int m = 0; m < 4; ++m) w[q][m] = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) { fxl[m] = 0.0; fxh[m] = 0.0; }
#pragma unroll
    for (int m = 0; m < 3; ++m) { fyl[m] = 0.0; fyh[m] = 0.0; }
    auto shift_in = [&](const double* v) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            w[q][0] = w[q][1]; w[q][1] = w[q][2]; w[q][2] = w[q][3]; w[q][3] = v[q];
        }
        fxl[0] = fxl[1]; fxl[1] = fxl[2]; fxl[2] = fxl[3];
        fxh[0] = fxh[1]; fxh[1] = fxh[2]; fxh[2] = fxh[3];
        fxl[3] = f4(v[5], v[1], v[0], v[2]);             // face x - 1/2
        fxh[3] = f4(v[1], v[0], v[2], v[6]);             // face x + 1/2
        fyl[0] = fyl[1]; fyl[1] = fyl[2];
        fyh[0] = fyh[1]; fyh[1] = fyh[2];
        fyl[2] = f4(v[7], v[3], v[0], v[4]);             // face y - 1/2
        fyh[2] = f4(v[3], v[0], v[4], v[8]);             // face y + 1/2
    };
    // flux through the vx face between window positions 0..3 (face between 1 and 2)
    auto gvx = [&]() {
        const double fc = f4(w[0][0], w[0][1], w[0][2], w[0][3]);
        const double fxm = f4(w[1][0], w[1][1], w[1][2], w[1][3]);
        const double fxp = f4(w[2][0], w[2][1], w[2][2], w[2][3]);
        const double fym = f4(w[3][0], w[3][1], w[3][2], w[3][3]);
        const double fyp = f4(w[4][0], w[4][1], w[4][2], w[4][3]);
        return axc * fc + (dax_x * (fxp - fxm) + dax_y * (fyp - fym)) * (1.0 / 48.0);
    };

    {
        double v[9];
#pragma unroll 1
        for (int p = -2; p <= 1; ++p) {
            ld9(p, v);
            shift_in(v);
        }
    }
    double gvx_lo = gvx();                               // face -1/2
    double msum = 0.0;
    const double cacc = A.c_acc, cnext = A.c_next;

#pragma unroll 1
    for (int tb = 0; tb < nvx; tb += RB) {
        double L[RB][9], FN[RB], AC[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            ld9(tb + q + 2, L[q]);
            const size_t o = po[0] + (size_t)min(tb + q, nvx - 1) * nvy + vyl;
            if (KIND == kStage23) FN[q] = A.fn[o];
            if (KIND == kStage23 || KIND == kStage4) AC[q] = A.acc[o];
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int t = tb + q;
            shift_in(L[q]);
            if (t >= nvx) continue;                      // uniform
            const double gxt = A.gx[t + 2];
            // x
            const double vbx = A.vx_lo + ((double)t + 0.5) * A.dvx;
            const double gxh = vbx * fxh[1] + dvx24 * (fxh[2] - fxh[0]);
            const double gxl = vbx * fxl[1] + dvx24 * (fxl[2] - fxl[0]);
            // y (product-rule term along vy from the neighbouring lanes)
            const double gyh = vby * fyh[0] + dvy24 * (nb(fyh[0], 1, gxt) - nb(fyh[0], -1, gxt));
            const double gyl2 = vby * fyl[0] + dvy24 * (nb(fyl[0], 1, gxt) - nb(fyl[0], -1, gxt));
            // vx
            const double gvx_hi = gvx();
            // vy: upper face from lanes -1 .. +2 of the five planes; lower face from lane - 1
            double fh[5], flb[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const double u0 = w[q][1];
                const double um = nb(u0, -1, gxt), u1 = nb(u0, 1, gxt), u2 = nb(u0, 2, gxt);
                fh[q] = f4(um, u0, u1, u2);
                flb[q] = f4(gxt * gyd[0], um, u0, u1);   // lower face of lane 0 (velocity-box face)
            }
            const double gvy_hi = ayc * fh[0] + (day_x * (fh[2] - fh[1]) + day_y * (fh[4] - fh[3])) * (1.0 / 48.0);
            const double gvy_b = ayc * flb[0] + (day_x * (flb[2] - flb[1]) + day_y * (flb[4] - flb[3])) * (1.0 / 48.0);
            const double gvy_s = __shfl(gvy_hi, lane - 1, 64);
            const double gvy_lo = lane == 0 ? gvy_b : gvy_s;

            const double k = -(gxh - gxl) * dxi - (gyh - gyl2) * dyi - (gvx_hi - gvx_lo) * dvxi -
                             (gvy_hi - gvy_lo) * dvyi;
            gvx_lo = gvx_hi;

            const size_t o = po[0] + (size_t)t * nvy + lane;
            double out;
            if (KIND == kRhs) {
                out = k;
                if (act) A.fout[o] = out;
            } else if (KIND == kStage1) {
                const double f0 = w[0][1];
                out = f0 + cnext * k;
                if (act) { A.acc[o] = f0 + cacc * k; A.fout[o] = out; }
            } else if (KIND == kStage23) {
                out = FN[q] + cnext * k;
                if (act) { A.acc[o] = AC[q] + cacc * k; A.fout[o] = out; }
            } else {
                out = AC[q] + cacc * k;
                if (act) A.fout[o] = out;
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

constexpr int kLd = kMaxPoisson2D + 1;

// C = A B for A (M x K) and B (K x N) in LDS with row stride kLd; each
// thread computes a 4 x 4 block; C is stored transposed when `tr`.
// Rows and columns past the sizes are zero in A and B, so the padded
// entries of C come out zero.
__device__ __forceinline__ void mm_lds(const double* A, const double* B, int M, int K, int N, double* C, bool tr)
{
    const int t = threadIdx.x;
    const int r0 = (t >> 4) * 4, c0 = (t & 15) * 4;
    if (r0 >= M || c0 >= N) return;
    double acc[4][4] = {};
#pragma unroll 4
    for (int k = 0; k < K; ++k) {
        double a[4], b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = A[(r0 + r) * kLd + k];
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = B[k * kLd + c0 + c];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (tr) C[(c0 + c) * kLd + r0 + r] = acc[r][c];
            else C[(r0 + r) * kLd + c0 + c] = acc[r][c];
        }
}

__device__ __forceinline__ void load_mat(const double* __restrict__ g, int rows, int cols, double* S)
{
    for (int q = threadIdx.x; q < rows * cols; q += 256) {
        const int r = q / cols, c = q - (q / cols) * cols;
        S[r * kLd + c] = g[q];
    }
}

// Periodic Poisson problem of the summed 1D fourth-order operators,
// solved in the real orthonormal Fourier basis that diagonalises every
// symmetric circulant matrix: phi = Qx [ (Qx^T rho Qy) / lambda ] Qy^T,
// the zero mode dropped.  Then E = -D phi per direction and a = (q/m) E.
__global__ __launch_bounds__(256) void k_poisson2d(const double* __restrict__ n, int nx, int ny, double dx,
                                                  double dy, double qm, const double* __restrict__ Qx,
                                                  const double* __restrict__ QxT, const double* __restrict__ Qy,
                                                  const double* __restrict__ QyT,
                                                  const double* __restrict__ invlamT, double* __restrict__ phi_out,
                                                  double* __restrict__ E_out, double* __restrict__ a_out)
{
    extern __shared__ double sm[];
    constexpr int S = kMaxPoisson2D * kLd;
    double* A = sm;
    double* B = sm + S;
    double* Q1 = sm + 2 * S;
    double* Q2 = sm + 3 * S;
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int N = nx * ny;
    for (int q = t; q < 4 * S; q += 256) sm[q] = 0.0;
    double s = 0.0;
    for (int q = t; q < N; q += 256) s += n[q];
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    const double mean = red[0] / N;
    // rho - mean(rho) = mean(n) - n
    for (int q = t; q < N; q += 256) {
        const int i = q / ny, j = q - (q / ny) * ny;
        A[i * kLd + j] = mean - n[q];
    }
    load_mat(Qy, ny, ny, Q1);
    load_mat(Qx, nx, nx, Q2);
    __syncthreads();
    mm_lds(A, Q1, nx, ny, ny, B, true);        // B[l][i] = (rho Qy)[i][l]
    __syncthreads();
    mm_lds(B, Q2, ny, nx, nx, A, false);       // A[l][k] = (Qx^T rho Qy)[k][l]
    __syncthreads();
    for (int q = t; q < N; q += 256) {
        const int l = q / nx, k = q - (q / nx) * nx;
        A[l * kLd + k] *= invlamT[q];
    }
    load_mat(QxT, nx, nx, Q2);
    load_mat(QyT, ny, ny, Q1);
    __syncthreads();
    mm_lds(A, Q2, ny, nx, nx, B, true);        // B[i][l] = (Qx hat)[i][l]
    __syncthreads();
    mm_lds(B, Q1, nx, ny, ny, A, false);       // A[i][j] = phi
    __syncthreads();
    const double cx = 1.0 / (12.0 * dx), cy = 1.0 / (12.0 * dy);
    for (int q = t; q < N; q += 256) {
        const int i = q / ny, j = q - (q / ny) * ny;
        const int ip1 = wrapi(i + 1, nx), im1 = wrapi(i - 1, nx), ip2 = wrapi(i + 2, nx), im2 = wrapi(i - 2, nx);
        const int jp1 = wrapi(j + 1, ny), jm1 = wrapi(j - 1, ny), jp2 = wrapi(j + 2, ny), jm2 = wrapi(j - 2, ny);
        const double ex = -(8.0 * (A[ip1 * kLd + j] - A[im1 * kLd + j]) - (A[ip2 * kLd + j] - A[im2 * kLd + j])) * cx;
        const double ey = -(8.0 * (A[i * kLd + jp1] - A[i * kLd + jm1]) - (A[i * kLd + jp2] - A[i * kLd + jm2])) * cy;
        if (phi_out) phi_out[q] = A[i * kLd + j];
        if (E_out) { E_out[q] = ex; E_out[N + q] = ey; }
        if (a_out) { a_out[q] = qm * ex; a_out[N + q] = qm * ey; }
    }
}

template <int KIND>
hipError_t launch_stage4d_k(int rb, const Stage4DArgs& a, hipStream_t stream)
{
    const int ncfg = a.nx * a.ny;
    const dim3 g((ncfg + 3) / 4), b(256);
    switch (rb) {
    case 1: hipLaunchKernelGGL((k_stage4d<KIND, 1>), g, b, 0, stream, a); break;
    case 2: hipLaunchKernelGGL((k_stage4d<KIND, 2>), g, b, 0, stream, a); break;
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

size_t poisson2d_lds_bytes() { return (size_t)4 * kMaxPoisson2D * kLd * sizeof(double); }

hipError_t poisson2d_prepare()
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_poisson2d),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)poisson2d_lds_bytes());
}

hipError_t launch_poisson2d(const double* n, int nx, int ny, double dx, double dy, double qm, const double* Qx,
                            const double* QxT, const double* Qy, const double* QyT, const double* invlamT,
                            double* phi, double* E, double* a, hipStream_t stream)
{
    if (nx > kMaxPoisson2D || ny > kMaxPoisson2D) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_poisson2d, dim3(1), dim3(256), poisson2d_lds_bytes(), stream, n, nx, ny, dx, dy, qm, Qx,
                       QxT, Qy, QyT, invlamT, phi, E, a);
    return hipGetLastError();
}

}  // namespace vp
