// HIP kernels of the 1D+1V single-level path (gfx950, wave64).
//
// Stage kernel: one block owns a velocity strip of TV = NT*W cells and
// marches along a segment of configuration rows.  Each step of the march
// stages one new row of the stage state into a five-row LDS ring (with a
// two-cell halo on each side of the strip, synthesised for the velocity
// ghosts), forms the fourth-order face averages and product-rule fluxes of
// the row (section 2 of the paper), takes the flux divergence, applies the
// RK4 stage combination and writes the row's velocity-moment partial sum.
// Every state element is read from HBM once per stage (halo rows and
// columns are re-read from cache), and v is the contiguous, coalesced axis.
#include <hip/hip_runtime.h>

#include "vp_internal.hpp"

namespace vp {

namespace {

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so that tiles sharing halo rows and columns
// run under the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, l = b >> 3;
    return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

__device__ __forceinline__ int wrapi(int i, int n)
{
    if (i >= 0 && i < n) return i;
    int r = i % n;
    return r < 0 ? r + n : r;
}

template <typename T>
__device__ __forceinline__ T ghost_val(const T* __restrict__ row, int j, int nv, const double* vg)
{
    if (j >= 0 && j < nv) return row[j];
    if (j == -2) return (T)vg[0];
    if (j == -1) return (T)vg[1];
    if (j == nv) return (T)vg[2];
    if (j == nv + 1) return (T)vg[3];
    return (T)0;
}

template <typename T, int W> struct VecIO;
template <> struct VecIO<double, 1> {
    static __device__ __forceinline__ void ld(const double* p, double* o) { o[0] = p[0]; }
    static __device__ __forceinline__ void st(double* p, const double* o) { p[0] = o[0]; }
};
template <> struct VecIO<double, 2> {
    static __device__ __forceinline__ void ld(const double* p, double* o)
    {
        double2 v = *reinterpret_cast<const double2*>(p);
        o[0] = v.x; o[1] = v.y;
    }
    static __device__ __forceinline__ void st(double* p, const double* o)
    {
        *reinterpret_cast<double2*>(p) = make_double2(o[0], o[1]);
    }
};
template <> struct VecIO<float, 1> {
    static __device__ __forceinline__ void ld(const float* p, float* o) { o[0] = p[0]; }
    static __device__ __forceinline__ void st(float* p, const float* o) { p[0] = o[0]; }
};
template <> struct VecIO<float, 4> {
    static __device__ __forceinline__ void ld(const float* p, float* o)
    {
        float4 v = *reinterpret_cast<const float4*>(p);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
    static __device__ __forceinline__ void st(float* p, const float* o)
    {
        *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
    }
};

__device__ __forceinline__ double wave_sum(double s)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
    return s;
}

template <typename T>
__device__ __forceinline__ T face4(T um1, T u0, T u1, T u2)
{
    // ideal-weight (unlimited) face average of cell averages
    return (T(7) * (u0 + u1) - (um1 + u2)) * T(1.0 / 12.0);
}

template <typename T, int W, int NT, int KIND>
__global__ __launch_bounds__(NT) void k_stage1d(Stage1DArgs A)
{
    constexpr int TV = NT * W;
    constexpr int LPAD = (W > 2) ? W : 2;                    // keeps own data W-aligned in LDS
    constexpr int RW = ((LPAD + TV + 2 + 3) / 4) * 4;
    constexpr int NWAVE = NT / 64;
    __shared__ __attribute__((aligned(16))) T ring[5][RW];
    __shared__ double mom[NWAVE][kMaxTx];

    const T* __restrict__ fs = static_cast<const T*>(A.fs);
    const T* __restrict__ fn = static_cast<const T*>(A.fn);
    T* __restrict__ acc = static_cast<T*>(A.acc);
    T* __restrict__ fout = static_cast<T*>(A.fout);
    const double* __restrict__ av = A.a;

    const int nx = A.nx, nv = A.nv;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    const int strip = tile % A.nstrip;
    const int seg = tile / A.nstrip;
    const int j0 = strip * TV;
    const int i0 = seg * A.tx;
    const int i1 = min(i0 + A.tx, nx);
    const int t = threadIdx.x;
    const int jt = j0 + t * W;
    const bool own_in = jt < nv;          // nv % W == 0 for W > 1, so the whole vector is in range
    const int lane = t & 63, wave = t >> 6;

    // register copy of one row of the stage state: own cells + halo cells
    T cur[W];
    T curh[2] = {T(0), T(0)};
    auto load_row = [&](int r) {
        const T* row = fs + (size_t)r * nv;
        if (own_in) {
            VecIO<T, W>::ld(row + jt, cur);
        } else {
#pragma unroll
            for (int w = 0; w < W; ++w) cur[w] = ghost_val(row, jt + w, nv, A.vg);
        }
        if (t == 0) {
            curh[0] = ghost_val(row, j0 - 2, nv, A.vg);
            curh[1] = ghost_val(row, j0 - 1, nv, A.vg);
        } else if (t == NT - 1) {
            curh[0] = ghost_val(row, j0 + TV, nv, A.vg);
            curh[1] = ghost_val(row, j0 + TV + 1, nv, A.vg);
        }
    };
    auto store_row = [&](int slot) {
        T* dst = &ring[slot][0];
#pragma unroll
        for (int w = 0; w < W; ++w) dst[LPAD + t * W + w] = cur[w];
        if (t == 0) {
            dst[LPAD - 2] = curh[0];
            dst[LPAD - 1] = curh[1];
        } else if (t == NT - 1) {
            dst[LPAD + TV] = curh[0];
            dst[LPAD + TV + 1] = curh[1];
        }
    };
    // LDS column index of global velocity cell j
    const int c0 = LPAD + t * W;   // own first cell

    // face average along x at columns jt-1 .. jt+W of face (row r1 - 1/2 .. ) from 4 ring rows
    auto fx_cols = [&](int sm1, int s0, int s1, int s2, T* Fx) {
#pragma unroll
        for (int q = 0; q < W + 2; ++q) {
            const int c = c0 - 1 + q;
            Fx[q] = face4<T>(ring[sm1][c], ring[s0][c], ring[s1][c], ring[s2][c]);
        }
    };
    // face average along v at faces jt-1/2 .. jt+W-1/2 of one ring row
    auto fv_faces = [&](int s, T* Fv) {
        T u[W + 4];
#pragma unroll
        for (int q = 0; q < W + 4; ++q) u[q] = ring[s][c0 - 2 + q];
#pragma unroll
        for (int m = 0; m <= W; ++m) Fv[m] = face4<T>(u[m], u[m + 1], u[m + 2], u[m + 3]);
    };

    T vb[W];
#pragma unroll
    for (int w = 0; w < W; ++w) vb[w] = (T)(A.v_lo + ((double)(jt + w) + 0.5) * A.dv);
    const T dxi = (T)A.dxi, dvi = (T)A.dvi, dv24 = (T)A.dv24;

    // ---- prologue: rows i0-2 .. i0+1 into slots 0..3
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        load_row(wrapi(i0 - 2 + q, nx));
        store_row(q);
    }
    if (i0 < i1) load_row(wrapi(i0 + 2, nx));
    __syncthreads();

    T gx_old[W];
    {
        T Fx[W + 2];
        fx_cols(0, 1, 2, 3, Fx);
#pragma unroll
        for (int w = 0; w < W; ++w) gx_old[w] = vb[w] * Fx[w + 1] + dv24 * (Fx[w + 2] - Fx[w]);
    }
    T fvA[W + 1], fvB[W + 1];
    fv_faces(1, fvA);
    fv_faces(2, fvB);
    T a_m1 = (T)av[wrapi(i0 - 1, nx)];
    T a_0 = (T)av[i0 < nx ? i0 : 0];

#pragma unroll 1
    for (int i = i0; i < i1; ++i) {
        const int q = i - i0;
        const int s_m1 = (q + 1) % 5, s_0 = (q + 2) % 5, s_p1 = (q + 3) % 5, s_p2 = (q + 4) % 5;
        store_row(s_p2);
        if (i + 1 < i1) load_row(wrapi(i + 3, nx));

        T fnv[W], accv[W];
        const size_t rowoff = (size_t)i * nv + jt;
        if (KIND == kStage23 && own_in) VecIO<T, W>::ld(fn + rowoff, fnv);
        if ((KIND == kStage23 || KIND == kStage4) && own_in) VecIO<T, W>::ld(acc + rowoff, accv);
        const T a_p1 = (T)av[wrapi(i + 1, nx)];

        __syncthreads();

        T Fx[W + 2];
        fx_cols(s_m1, s_0, s_p1, s_p2, Fx);
        T fvC[W + 1];
        fv_faces(s_p1, fvC);
        const T da48 = (a_p1 - a_m1) * T(1.0 / 48.0);
        T gv[W + 1];
#pragma unroll
        for (int m = 0; m <= W; ++m) gv[m] = a_0 * fvB[m] + da48 * (fvC[m] - fvA[m]);
        T kk[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const T gx_new = vb[w] * Fx[w + 1] + dv24 * (Fx[w + 2] - Fx[w]);
            kk[w] = -(gx_new - gx_old[w]) * dxi - (gv[w + 1] - gv[w]) * dvi;
            gx_old[w] = gx_new;
        }

        if (KIND == kRhs) {
            if (own_in) VecIO<T, W>::st(fout + rowoff, kk);
        } else {
            T nxt[W];
            if (KIND == kStage1) {
                // f^n is the stage state itself: take it from the ring
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const T f0 = ring[s_0][c0 + w];
                    accv[w] = f0 + (T)A.c_acc * kk[w];
                    nxt[w] = f0 + (T)A.c_next * kk[w];
                }
                if (own_in) {
                    VecIO<T, W>::st(acc + rowoff, accv);
                    VecIO<T, W>::st(fout + rowoff, nxt);
                }
            } else if (KIND == kStage23) {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    accv[w] = accv[w] + (T)A.c_acc * kk[w];
                    nxt[w] = fnv[w] + (T)A.c_next * kk[w];
                }
                if (own_in) {
                    VecIO<T, W>::st(acc + rowoff, accv);
                    VecIO<T, W>::st(fout + rowoff, nxt);
                }
            } else {  // kStage4: f^{n+1} = acc + dt/6 k4
#pragma unroll
                for (int w = 0; w < W; ++w) nxt[w] = accv[w] + (T)A.c_acc * kk[w];
                if (own_in) VecIO<T, W>::st(fout + rowoff, nxt);
            }
            if (A.part) {
                double s = 0.0;
                if (own_in) {
#pragma unroll
                    for (int w = 0; w < W; ++w) s += (double)nxt[w];
                }
                s = wave_sum(s);
                if (lane == 0) mom[wave][q] = s;
            }
        }
#pragma unroll
        for (int m = 0; m <= W; ++m) { fvA[m] = fvB[m]; fvB[m] = fvC[m]; }
        a_m1 = a_0;
        a_0 = a_p1;
    }

    if (KIND != kRhs && A.part) {
        __syncthreads();
        for (int q = t; q < i1 - i0; q += NT) {
            double s = 0.0;
#pragma unroll
            for (int wv = 0; wv < NWAVE; ++wv) s += mom[wv][q];
            A.part[(size_t)strip * nx + i0 + q] = s;
        }
    }
}

// n_i = dv * sum_j f_ij, one block per row, fixed summation order.
template <typename T>
__global__ __launch_bounds__(256) void k_moment_rows(const T* __restrict__ f, int nv, double dv,
                                                    double* __restrict__ n)
{
    __shared__ double red[4];
    const int i = blockIdx.x;
    const T* row = f + (size_t)i * nv;
    double s = 0.0;
    for (int j = threadIdx.x; j < nv; j += 256) s += (double)row[j];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) n[i] = dv * (((red[0] + red[1]) + red[2]) + red[3]);
}

// ------------------------------------------------------------------ Poisson
//
// The periodic operator of the discrete potential equation factors as
//   A = (S + S^-1 - 2)(S + S^-1 - 14),  S the periodic shift,
// since 30 - 16 (z + 1/z) + (z^2 + 1/z^2) = (w - 2)(w - 14) with w = z + 1/z.
// So A phi = r is solved as y = (S + S^-1 - 14)^-1 r (a short convolution
// with the exact periodic Green's function, which decays by 7 - sqrt(48)
// per cell) followed by the periodic second difference
// d_i - d_{i-1} = y_i with d_i = phi_{i+1} - phi_i (two prefix sums).  The
// field only needs d:  E_i = -(7 (d_i + d_{i-1}) - d_{i+1} - d_{i-2}) / (12 dx).

__device__ double block_sum_1024(double s, double* red)
{
    s = wave_sum(s);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = s;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int wv = 0; wv < kPoissonThreads / 64; ++wv) tot += red[wv];
    return tot;
}

// exclusive prefix of per-thread values over the block, fixed order
__device__ double block_exclusive_scan_1024(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        double y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) red[wave] = x;
    __syncthreads();
    double off = 0.0;
    for (int wv = 0; wv < wave; ++wv) off += red[wv];
    return off + x - v;
}

__global__ __launch_bounds__(kPoissonThreads) void k_poisson1d(
    const double* __restrict__ part, int nstrip, const double* __restrict__ n_in, double dv, int nx,
    double dx, double qm, const double* __restrict__ green, int gk, double* __restrict__ n_out,
    double* __restrict__ phi_out, double* __restrict__ E_out, double* __restrict__ a_out)
{
    extern __shared__ double sm[];
    double* r = sm;            // nx: rho, then r, then y
    double* d = sm + nx;       // nx: d = phi_{i+1} - phi_i
    __shared__ double red[kPoissonThreads / 64];
    const int t = threadIdx.x;
    const int c = (nx + kPoissonThreads - 1) / kPoissonThreads;
    const int lo = min(t * c, nx), hi = min(lo + c, nx);

    // moment and charge density
    double s = 0.0;
    for (int i = t; i < nx; i += kPoissonThreads) {
        double n;
        if (part) {
            double acc = 0.0;
            for (int q = 0; q < nstrip; ++q) acc += part[(size_t)q * nx + i];
            n = dv * acc;
        } else {
            n = n_in[i];
        }
        if (n_out) n_out[i] = n;
        r[i] = 1.0 - n;
    }
    __syncthreads();
    for (int i = lo; i < hi; ++i) s += r[i];
    const double mean_rho = block_sum_1024(s, red) / nx;
    const double scale = 12.0 * dx * dx;
    for (int i = lo; i < hi; ++i) r[i] = scale * (r[i] - mean_rho);
    __syncthreads();

    // y = (S + S^-1 - 14)^-1 r ; each thread keeps its contiguous chunk in registers
    constexpr int CM = kMaxPoisson1D / kPoissonThreads;
    double yv[CM];
    const bool full = nx <= 2 * gk + 1;
#pragma unroll
    for (int m = 0; m < CM; ++m) {
        const int i = lo + m;
        double acc = 0.0;
        if (i < hi) {
            if (full) {
                for (int q = 0; q < nx; ++q) acc += green[wrapi(i - q, nx)] * r[q];
            } else {
                acc = green[0] * r[i];
                for (int o = 1; o <= gk; ++o) acc += green[o] * (r[wrapi(i + o, nx)] + r[wrapi(i - o, nx)]);
            }
        }
        yv[m] = acc;
    }
    s = 0.0;
#pragma unroll
    for (int m = 0; m < CM; ++m) s += yv[m];
    const double mean_y = block_sum_1024(s, red) / nx;

    // d = prefix(y) - mean(prefix(y))
    double run = 0.0;
#pragma unroll
    for (int m = 0; m < CM; ++m) {
        if (lo + m < hi) run += yv[m] - mean_y;
        yv[m] = run;
    }
    const double off = block_exclusive_scan_1024(run, red);
    s = 0.0;
#pragma unroll
    for (int m = 0; m < CM; ++m) {
        yv[m] += off;
        if (lo + m < hi) s += yv[m];
    }
    const double mean_d = block_sum_1024(s, red) / nx;
#pragma unroll
    for (int m = 0; m < CM; ++m)
        if (lo + m < hi) d[lo + m] = yv[m] - mean_d;
    __syncthreads();

    for (int i = t; i < nx; i += kPoissonThreads) {
        const double E = -(7.0 * (d[i] + d[wrapi(i - 1, nx)]) - d[wrapi(i + 1, nx)] - d[wrapi(i - 2, nx)]) /
                         (12.0 * dx);
        if (E_out) E_out[i] = E;
        if (a_out) a_out[i] = qm * E;
    }
    if (phi_out) {
        // phi_i = sum_{m < i} d_m + const, zero mean
        double run2 = 0.0;
#pragma unroll
        for (int m = 0; m < CM; ++m) {
            yv[m] = run2;
            if (lo + m < hi) run2 += d[lo + m];
        }
        const double off2 = block_exclusive_scan_1024(run2, red);
        s = 0.0;
#pragma unroll
        for (int m = 0; m < CM; ++m) {
            yv[m] += off2;
            if (lo + m < hi) s += yv[m];
        }
        const double mean_phi = block_sum_1024(s, red) / nx;
#pragma unroll
        for (int m = 0; m < CM; ++m)
            if (lo + m < hi) phi_out[lo + m] = yv[m] - mean_phi;
    }
}

__global__ void k_scale(const double* __restrict__ x, double s, double* __restrict__ y, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = s * x[i];
}

template <typename T, int W, int NT>
hipError_t launch_stage_t(int kind, const Stage1DArgs& a, hipStream_t stream)
{
    const int nstrip = a.nstrip;
    const int nseg = (a.nx + a.tx - 1) / a.tx;
    const dim3 grid(nstrip * nseg), block(NT);
    switch (kind) {
    case kRhs: hipLaunchKernelGGL((k_stage1d<T, W, NT, kRhs>), grid, block, 0, stream, a); break;
    case kStage1: hipLaunchKernelGGL((k_stage1d<T, W, NT, kStage1>), grid, block, 0, stream, a); break;
    case kStage23: hipLaunchKernelGGL((k_stage1d<T, W, NT, kStage23>), grid, block, 0, stream, a); break;
    default: hipLaunchKernelGGL((k_stage1d<T, W, NT, kStage4>), grid, block, 0, stream, a); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stage1d(int dtype, const StageShape& sh, int kind, const Stage1DArgs& a,
                          hipStream_t stream)
{
    if (dtype == VP_F64) {
        if (sh.w == 2 && sh.nt == 128) return launch_stage_t<double, 2, 128>(kind, a, stream);
        if (sh.w == 2 && sh.nt == 256) return launch_stage_t<double, 2, 256>(kind, a, stream);
        if (sh.w == 2 && sh.nt == 64) return launch_stage_t<double, 2, 64>(kind, a, stream);
        if (sh.w == 1 && sh.nt == 128) return launch_stage_t<double, 1, 128>(kind, a, stream);
        if (sh.w == 1 && sh.nt == 64) return launch_stage_t<double, 1, 64>(kind, a, stream);
    } else {
        if (sh.w == 4 && sh.nt == 64) return launch_stage_t<float, 4, 64>(kind, a, stream);
        if (sh.w == 4 && sh.nt == 128) return launch_stage_t<float, 4, 128>(kind, a, stream);
        if (sh.w == 1 && sh.nt == 128) return launch_stage_t<float, 1, 128>(kind, a, stream);
        if (sh.w == 1 && sh.nt == 64) return launch_stage_t<float, 1, 64>(kind, a, stream);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_moment_rows(int dtype, const void* f, int nx, int nv, double dv, double* n,
                              hipStream_t stream)
{
    if (dtype == VP_F64)
        hipLaunchKernelGGL(k_moment_rows<double>, dim3(nx), dim3(256), 0, stream,
                           static_cast<const double*>(f), nv, dv, n);
    else
        hipLaunchKernelGGL(k_moment_rows<float>, dim3(nx), dim3(256), 0, stream,
                           static_cast<const float*>(f), nv, dv, n);
    return hipGetLastError();
}

hipError_t poisson1d_prepare()
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(k_poisson1d),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(2 * kMaxPoisson1D * sizeof(double)));
}

hipError_t launch_poisson1d(const double* part, int nstrip, const double* n_in, double dv, int nx,
                            double dx, double qm, const double* green, int gk, double* n_out,
                            double* phi, double* E, double* a, hipStream_t stream)
{
    const size_t lds = 2 * (size_t)nx * sizeof(double);
    hipLaunchKernelGGL(k_poisson1d, dim3(1), dim3(kPoissonThreads), lds, stream, part, nstrip, n_in,
                       dv, nx, dx, qm, green, gk, n_out, phi, E, a);
    return hipGetLastError();
}

hipError_t launch_scale(const double* x, double s, double* y, int n, hipStream_t stream)
{
    hipLaunchKernelGGL(k_scale, dim3((n + 255) / 256), dim3(256), 0, stream, x, s, y, n);
    return hipGetLastError();
}

}  // namespace vp
