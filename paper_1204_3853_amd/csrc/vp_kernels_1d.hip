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
#include <type_traits>

#include "vp_internal.hpp"
#include "vp_stage_tile.hpp"

namespace vp {

namespace {

using namespace dev;

// The FP64 centred-face kernels are held to 128 VGPRs (four waves per SIMD).
template <typename T, int W, int NT, int KIND>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 4 : 1))) void k_stage1d(Stage1DArgs A)
{
    stage_tile_uniform<T, W, NT, KIND, false>(A, xcd_remap(blockIdx.x, gridDim.x));
}

// limited face averages (section 2, eq. limitedFace)
template <typename T, int W, int NT, int KIND>
__global__ __launch_bounds__(NT) void k_stage1d_lim(Stage1DArgs A)
{
    stage_tile_uniform<T, W, NT, KIND, true>(A, xcd_remap(blockIdx.x, gridDim.x));
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
//
// The null space: (S + S^-1 - 14) maps constants to -12 times themselves,
// so removing the mean of y after the convolution is the same as projecting
// rho onto zero mean first.  d is the prefix sum of y minus its mean; the
// mean of the prefix sums follows from the same block reduction as the mean
// of y:  sum_i D_i = sum_m y~_m (N - m).
//
// One block of kPoissonThreads threads; thread t owns the contiguous cells
// [t c, t c + c), c = ceil(nx / kPoissonThreads).

__device__ __forceinline__ void block_sum2(double& a, double& b, double* red)
{
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = kPoissonThreads / 64;
    __syncthreads();
    if (lane == 0) { red[wave] = a; red[NW + wave] = b; }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int wv = 0; wv < NW; ++wv) { ta += red[wv]; tb += red[NW + wv]; }
    a = ta;
    b = tb;
}

// exclusive prefix of per-thread values over the block, fixed order
__device__ double block_exclusive_scan(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) red[wave] = x;
    __syncthreads();
    double off = 0.0;
    for (int wv = 0; wv < wave; ++wv) off += red[wv];
    return off + x - v;
}

// ---------------------------------------------------------------- split field solve
//
// Double-double arithmetic (an unevaluated sum hi + lo, the error-free
// transformations of Knuth's two-sum and of an fma product) for the sums
// that reach across the whole mesh: the prefix of y up to a chunk is a
// difference of two sums of size |mean y| times the chunk offset, so in
// plain FP64 its rounding grows with the mesh size.
struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD dd_two_sum(double a, double b)
{
    const double s = a + b;
    const double bb = s - a;
    return DD{s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ DD dd_add(DD a, DD b)
{
    const DD s = dd_two_sum(a.hi, b.hi);
    const double lo = s.lo + (a.lo + b.lo);
    const double hi = s.hi + lo;
    return DD{hi, lo - (hi - s.hi)};
}

__device__ __forceinline__ DD dd_neg(DD a) { return DD{-a.hi, -a.lo}; }

// a times a double
__device__ __forceinline__ DD dd_mul(DD a, double b)
{
    const double p = a.hi * b;
    const double e = fma(a.hi, b, -p) + a.lo * b;
    const double hi = p + e;
    return DD{hi, e - (hi - p)};
}

// a divided by a double
__device__ __forceinline__ DD dd_div(DD a, double b)
{
    const double q = a.hi / b;
    const double r = (fma(-q, b, a.hi) + a.lo) / b;
    const double hi = q + r;
    return DD{hi, r - (hi - q)};
}

// the product of two doubles, exactly
__device__ __forceinline__ DD dd_prod(double a, double b)
{
    const double p = a * b;
    return DD{p, fma(a, b, -p)};
}

__device__ __forceinline__ DD dd_wave_sum(DD v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const DD u{__shfl_xor(v.hi, o, 64), __shfl_xor(v.lo, o, 64)};
        v = dd_add(v, u);
    }
    return v;
}
//
// The same solve as k_poisson1d, spread over chunks of kFieldChunk
// configuration cells so that many CUs share it (for meshes of at least
// kFieldSplitMin cells):
//   k_field_chunks: per chunk, the moment from the stage kernel's strip
//     partials (with a 16-cell periodic halo), r = 12 dx^2 (1 - n), the
//     tridiagonal-factor inverse y = g * r over the chunk, and the chunk's
//     sums of y and of y_m (N - m) in double-double;
//   k_field_finish: per chunk, the global mean of y and of D from the
//     chunk sums, the chunk's prefix offset (all in double-double), an
//     in-chunk scan for d = D - mean(D) (D_i = sum_{m <= i} (y_m - mean y)),
//     and the field E_i = -(7 (d_i + d_{i-1}) - d_{i+1} - d_{i-2}) / (12 dx),
//     a = (q/m) E.
// All sums run in a fixed order.

__global__ __launch_bounds__(kFieldChunk) void k_field_chunks(SpeciesMoments m, int nx, double dx,
                                                              const double* __restrict__ green,
                                                              double* __restrict__ y, double* __restrict__ csum)
{
    constexpr int K = kGreenTaps;
    __shared__ double r[kFieldChunk + 2 * K];
    __shared__ double gs[K + 1];
    __shared__ double red[4 * (kFieldChunk / 64)];
    const int t = threadIdx.x;
    const int c0 = blockIdx.x * kFieldChunk;
    if (t <= K) gs[t] = green[t];
    const double scale = 12.0 * dx * dx;
    // the charge density of rows c0 - K .. c0 + kFieldChunk + K - 1
    // (periodic): per species the sum of its strip partials (the loads of
    // both rows a thread owns in flight together), weighted, added to the
    // background
    constexpr int NQ = (kFieldChunk + 2 * K + kFieldChunk - 1) / kFieldChunk;
    double rho[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) rho[u] = m.background;
    for (int sp = 0; sp < m.ns; ++sp) {
        const double* part = m.part[sp];
        const int nstrip = m.nstrip[sp];
        double acc[NQ];
#pragma unroll
        for (int u = 0; u < NQ; ++u) acc[u] = 0.0;
        for (int s0 = 0; s0 < nstrip; s0 += 8) {
            double v[NQ][8];
#pragma unroll
            for (int u = 0; u < NQ; ++u) {
                const int i = wrapi(c0 - K + min(t + u * kFieldChunk, kFieldChunk + 2 * K - 1), nx);
#pragma unroll
                for (int q = 0; q < 8; ++q) v[u][q] = (s0 + q < nstrip) ? part[(size_t)(s0 + q) * nx + i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < NQ; ++u)
#pragma unroll
                for (int q = 0; q < 8; ++q) acc[u] += v[u][q];
        }
#pragma unroll
        for (int u = 0; u < NQ; ++u) rho[u] += m.w[sp] * acc[u];
    }
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int q = t + u * kFieldChunk;
        if (q < kFieldChunk + 2 * K) r[q] = scale * rho[u];
    }
    __syncthreads();
    const int i = c0 + t;
    double yi = gs[0] * r[t + K];
#pragma unroll
    for (int o = 1; o <= K; ++o) yi += gs[o] * (r[t + K + o] + r[t + K - o]);
    DD sy{0.0, 0.0}, sw{0.0, 0.0};
    if (i < nx) {
        y[i] = yi;
        sy.hi = yi;
        sw = dd_prod(yi, (double)(nx - i));
    }
    sy = dd_wave_sum(sy);
    sw = dd_wave_sum(sw);
    const int lane = t & 63, wave = t >> 6;
    constexpr int NW = kFieldChunk / 64;
    if (lane == 0) {
        red[wave] = sy.hi;
        red[NW + wave] = sy.lo;
        red[2 * NW + wave] = sw.hi;
        red[3 * NW + wave] = sw.lo;
    }
    __syncthreads();
    if (t == 0) {
        DD a{0.0, 0.0}, b{0.0, 0.0};
        for (int w = 0; w < NW; ++w) {
            a = dd_add(a, DD{red[w], red[NW + w]});
            b = dd_add(b, DD{red[2 * NW + w], red[3 * NW + w]});
        }
        csum[4 * blockIdx.x] = a.hi;
        csum[4 * blockIdx.x + 1] = a.lo;
        csum[4 * blockIdx.x + 2] = b.hi;
        csum[4 * blockIdx.x + 3] = b.lo;
    }
}

__global__ __launch_bounds__(kFieldChunk) void k_field_finish(const double* __restrict__ y,
                                                              const double* __restrict__ csum, int nchunk, int nx,
                                                              double dx, FieldOutputs out)
{
    __shared__ double d[kFieldChunk + 4];     // d_i for i = c0 - 2 .. c0 + kFieldChunk + 1
    __shared__ double red[kFieldChunk / 64];
    __shared__ double cs[4 * (kMaxPoisson1D / kFieldChunk)];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int c = blockIdx.x, c0 = c * kFieldChunk;
    // the rows of y this block reads, loaded while the chunk sums are summed
    const double yt = y[wrapi(c0 + t, nx)];
    const double ye0 = y[wrapi(c0 + kFieldChunk, nx)], ye1 = y[wrapi(c0 + kFieldChunk + 1, nx)];
    const double ym1 = y[wrapi(c0 - 1, nx)];
    if (t < 4 * nchunk) cs[t] = csum[t];
    __syncthreads();
    // global sums and the prefix of y - mean(y) up to the chunk start, in
    // chunk order, in double-double
    DD sy{0.0, 0.0}, sw{0.0, 0.0}, pre{0.0, 0.0};
    for (int q = 0; q < nchunk; ++q) {
        if (q == c) pre = sy;
        sy = dd_add(sy, DD{cs[4 * q], cs[4 * q + 1]});
        sw = dd_add(sw, DD{cs[4 * q + 2], cs[4 * q + 3]});
    }
    const DD ybar_dd = dd_div(sy, (double)nx);
    // sum_i i for i = 1 .. nx is an integer below 2^53
    const DD mean_D = dd_div(dd_add(sw, dd_neg(dd_mul(ybar_dd, 0.5 * (double)nx * (double)(nx + 1)))), (double)nx);
    const DD off_dd = dd_add(dd_add(pre, dd_neg(dd_mul(ybar_dd, (double)c0))), dd_neg(mean_D));   // d_{c0 - 1}
    const double ybar = ybar_dd.hi, ybar_lo = ybar_dd.lo;
    const double off = off_dd.hi + off_dd.lo;
    // inclusive scan of y - mean(y) over rows c0 .. c0 + kFieldChunk + 1 (periodic)
    const double yv = (yt - ybar) - ybar_lo;
    double x = yv;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double u = __shfl_up(x, o, 64);
        if (lane >= o) x += u;
    }
    if (lane == 63) red[wave] = x;
    __syncthreads();
    double wo = 0.0;
    for (int w = 0; w < wave; ++w) wo += red[w];
    d[t + 2] = off + wo + x;
    if (t < 2) {
        // rows past the chunk: d continues with y of rows c0 + 256, c0 + 257
        double tail = 0.0;
        for (int w = 0; w < kFieldChunk / 64; ++w) tail += red[w];
        double e = off + tail + ((ye0 - ybar) - ybar_lo);
        if (t == 1) e += (ye1 - ybar) - ybar_lo;
        d[kFieldChunk + 2 + t] = e;
    }
    if (t == 0) {
        // rows before the chunk: d_{c0 - 1} = off, d_{c0 - 2} = off - (y_{c0 - 1} - mean y)
        d[1] = off;
        d[0] = off - ((ym1 - ybar) - ybar_lo);
    }
    __syncthreads();
    const int i = c0 + t;
    double E = 0.0;
    if (i < nx) {
        E = -(7.0 * (d[t + 2] + d[t + 1]) - d[t + 3] - d[t]) / (12.0 * dx);
        for (int k = 0; k < out.n; ++k) out.a[k][i] = out.qm[k] * E;
    }
    if (out.inject_R > 0) {
        // two levels: the coarse acceleration is (q/m) times the mean of the
        // R fine values (R divides the chunk size and nx)
        __syncthreads();
        d[t] = E;
        __syncthreads();
        const int R = out.inject_R;
        if (t < kFieldChunk / R && c0 + t * R < nx) {
            double se = 0.0;
            for (int q = 0; q < R; ++q) se += d[t * R + q];
            out.inject_a[c0 / R + t] = out.inject_qm * (se / R);
        }
    }
}

// adjoint = 0: r = 12 dx^2 (1 - n) from the moment n_in; outputs phi, E, a.
// adjoint = 1: n_in holds abar; r = 12 dx^2 D (q/m) abar (D the field
// stencil without its sign); phi_out receives phi_scale * S r / (12 dx^2)-
// solution, i.e. z = -dv S D (q/m) abar with phi_scale = -dv.
__global__ __launch_bounds__(kPoissonThreads) void k_poisson1d(
    const double* __restrict__ n_in, int nx, double dx, double qm, const double* __restrict__ green, int gk,
    double* __restrict__ phi_out, double* __restrict__ E_out, double* __restrict__ a_out, int adjoint,
    double phi_scale, PoissonExtra X)
{
    constexpr int K = kGreenTaps;
    constexpr int SUB = 8;               // outputs per register window of the convolution
    extern __shared__ double sm[];
    __shared__ double red[2 * (kPoissonThreads / 64)];
    __shared__ double gs[K + 1];
    const int t = threadIdx.x;
    const bool full = nx <= 2 * gk + 1;   // the table then holds all nx periodic values
    if (!full && t <= K) gs[t] = green[t];

    // Thread t owns the contiguous chunk [t c, t c + c) (c a power of two)
    // for the convolution and the prefix sums.  LDS arrays carry one pad
    // cell per chunk, so a wave's chunk-wise accesses fall on different
    // banks; elementwise loops use strided ownership.
    int lc = 0;
    while ((kPoissonThreads << lc) < nx) ++lc;
    const int c = 1 << lc;
    const int lo = min(t * c, nx), hi = min(lo + c, nx);
    auto pad = [&](int j) { return j + (j >> lc); };
    double* rext = sm;                                   // r_i at pad(i + K), i in [-K, nx + K + SUB)
    double* ybuf = sm + pad(nx + 2 * K + SUB) + 1;       // y_i at pad(i); later d_i at pad(i + 2)
    auto rp = [&](int i) { return pad(i + K); };

    // r = 12 dx^2 (1 - n); every load of the block is issued before any is used
    const double scale = 12.0 * dx * dx;
    {
        constexpr int RM = kMaxPoisson1D / kPoissonThreads;
        double nv[RM];
        if (X.slots) {
            // n_i = sum_k w_k slots[idx_k] over the fixed-order list of cell i
#pragma unroll
            for (int m = 0; m < RM; ++m) {
                const int i = t + m * kPoissonThreads;
                double sacc = 0.0;
                if (i < nx) {
                    const int k0 = X.rowptr[i], k1 = X.rowptr[i + 1];
#pragma unroll 4
                    for (int k = k0; k < k1; ++k) sacc += X.w[k] * X.slots[X.idx[k]];
                }
                nv[m] = sacc;
            }
        } else if (X.part) {
            // the moment from the stage kernel's strip partials, in strip order
#pragma unroll
            for (int m = 0; m < RM; ++m) {
                const int i = t + m * kPoissonThreads;
                double sacc = 0.0;
                if (i < nx)
                    for (int q = 0; q < X.nstrip; ++q) sacc += X.part[(size_t)q * nx + i];
                nv[m] = X.dv * sacc;
                if (X.n_out && i < nx) X.n_out[i] = nv[m];
            }
        } else {
#pragma unroll
            for (int m = 0; m < RM; ++m) {
                const int i = t + m * kPoissonThreads;
                nv[m] = i < nx ? n_in[i] : 0.0;
            }
        }
        if (!adjoint) {
#pragma unroll
            for (int m = 0; m < RM; ++m) {
                const int i = t + m * kPoissonThreads;
                if (i < nx) rext[rp(i)] = scale * (1.0 - nv[m]);
            }
        } else {
            // u = D (q/m) abar through a temporary copy of (q/m) abar in ybuf
#pragma unroll
            for (int m = 0; m < RM; ++m) {
                const int i = t + m * kPoissonThreads;
                if (i < nx) ybuf[i] = qm * nv[m];
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < RM; ++m) {
                const int i = t + m * kPoissonThreads;
                if (i < nx) {
                    const double d1 = ybuf[wrapi(i + 1, nx)] - ybuf[wrapi(i - 1, nx)];
                    const double d2 = ybuf[wrapi(i + 2, nx)] - ybuf[wrapi(i - 2, nx)];
                    rext[rp(i)] = scale * (8.0 * d1 - d2) / (12.0 * dx);
                }
            }
        }
    }
    __syncthreads();
    for (int e = t; e < 2 * K + SUB; e += kPoissonThreads) {   // periodic halo
        const int i = e < K ? e - K : nx + (e - K);
        rext[rp(i)] = rext[rp(wrapi(i, nx))];
    }
    __syncthreads();

    // y = (S + S^-1 - 14)^-1 r over the own chunk, plus the sums for mean(y)
    // and mean(D)
    double sy = 0.0, syw = 0.0;
    if (full) {
        for (int i = lo; i < hi; ++i) {
            double acc = 0.0;
            for (int q = 0; q < nx; ++q) acc += green[wrapi(i - q, nx)] * rext[rp(q)];
            ybuf[pad(i)] = acc;
            sy += acc;
            syw += acc * (double)(nx - i);
        }
    } else {
        for (int j0 = lo; j0 < hi; j0 += SUB) {
            double w[SUB + 2 * K];
#pragma unroll
            for (int q = 0; q < SUB + 2 * K; ++q) w[q] = rext[rp(j0 - K + q)];
#pragma unroll
            for (int u = 0; u < SUB; ++u) {
                double acc = gs[0] * w[u + K];
#pragma unroll
                for (int o = 1; o <= K; ++o) acc += gs[o] * (w[u + K + o] + w[u + K - o]);
                const int i = j0 + u;
                if (i < hi) {
                    ybuf[pad(i)] = acc;
                    sy += acc;
                    syw += acc * (double)(nx - i);
                }
            }
        }
    }
    block_sum2(sy, syw, red);
    const double mean_y = sy / nx;
    // mean of D_i = sum_{m<=i} (y_m - mean_y):  (sum_m y_m (N - m) - mean_y N (N + 1) / 2) / N
    const double mean_D = (syw - mean_y * 0.5 * (double)nx * (double)(nx + 1)) / nx;

    // d = D - mean(D); d_i is written over rext at dp(i), with a 2-cell periodic halo
    double run = 0.0;
    for (int i = lo; i < hi; ++i) run += ybuf[pad(i)] - mean_y;
    const double off = block_exclusive_scan(run, red);   // ends with a barrier: rext is free
    double* dext = rext;
    auto dp = [&](int i) { return pad(i + 2); };
    double pre = off - mean_D;
    for (int i = lo; i < hi; ++i) {
        pre += ybuf[pad(i)] - mean_y;
        dext[dp(i)] = pre;
        // the owners of the first and last two cells also write the halo
        if (i < 2) dext[dp(nx + i)] = pre;
        if (i >= nx - 2) dext[dp(i - nx)] = pre;
    }
    __syncthreads();
    if (nx < 2) {      // one cell: every halo cell is d_0
        if (t == 0) dext[dp(-2)] = dext[dp(-1)] = dext[dp(1)] = dext[dp(2)] = dext[dp(0)];
        __syncthreads();
    }

    for (int i = t; i < nx; i += kPoissonThreads) {
        const double E = -(7.0 * (dext[dp(i)] + dext[dp(i - 1)]) - dext[dp(i + 1)] - dext[dp(i - 2)]) /
                         (12.0 * dx);
        if (E_out) E_out[i] = E;
        if (X.inject_R > 0) {
            ybuf[pad(i)] = E;
            a_out[nx / X.inject_R + i] = qm * E;
        } else if (X.inject_L > 0) {
            ybuf[pad(i)] = E;
        } else if (a_out) {
            a_out[i] = qm * E;
        }
    }
    if (X.inject_L > 0) {
        // every level of a hierarchy: (q/m) times the mean of the rt fine
        // values over each of its cells (rt = 1 on the finest level)
        __syncthreads();
        for (int l = 0; l < X.inject_L; ++l) {
            const int rt = X.inject_rt[l];
            for (int k = t; k < nx / rt; k += kPoissonThreads) {
                double se = 0.0;
                for (int q = 0; q < rt; ++q) se += ybuf[pad(k * rt + q)];
                a_out[X.inject_off[l] + k] = qm * (se / rt);
            }
        }
        return;      // phi is not requested with injection
    }
    if (X.inject_R > 0) {
        // two levels: the coarse acceleration is (q/m) times the mean of the R fine values
        __syncthreads();
        const int R = X.inject_R;
        for (int k = t; k < nx / R; k += kPoissonThreads) {
            double se = 0.0;
            for (int q = 0; q < R; ++q) se += ybuf[pad(k * R + q)];
            a_out[k] = qm * (se / R);
        }
        return;      // phi is not requested with injection
    }
    if (phi_out) {
        // phi_i = sum_{m < i} d_m + const, zero mean
        double run2 = 0.0, sw = 0.0;
        for (int i = lo; i < hi; ++i) run2 += dext[dp(i)];
        const double off2 = block_exclusive_scan(run2, red);
        double p2 = off2;
        for (int i = lo; i < hi; ++i) {
            ybuf[pad(i)] = p2;
            sw += p2;
            p2 += dext[dp(i)];
        }
        double dummy = 0.0;
        block_sum2(sw, dummy, red);
        const double mean_phi = sw / nx;
        for (int i = t; i < nx; i += kPoissonThreads) phi_out[i] = phi_scale * (ybuf[pad(i)] - mean_phi);
    }
}

__global__ void k_scale(const double* __restrict__ x, double s, double* __restrict__ y, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = s * x[i];
}

// one row per thread: every species' strip sums in a fixed order, then
// rho = background + sum_s w_s (sum of its strips), n_eff = 1 - rho
__global__ __launch_bounds__(256) void k_species_neff(SpeciesMoments m, int nx, double* __restrict__ n_eff)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nx) return;
    double rho = m.background;
    for (int s = 0; s < m.ns; ++s) {
        const double* part = m.part[s];
        const int nstrip = m.nstrip[s];
        double acc = 0.0;
        for (int q0 = 0; q0 < nstrip; q0 += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = (q0 + u < nstrip) ? part[(size_t)(q0 + u) * nx + i] : 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u) acc += v[u];
        }
        rho += m.w[s] * acc;
    }
    n_eff[i] = 1.0 - rho;
}

template <typename T, int W, int NT>
hipError_t launch_stage_t(int kind, const Stage1DArgs& a, hipStream_t stream)
{
    const int nstrip = a.nstrip;
    const int nseg = (a.nx + a.tx - 1) / a.tx;
    const dim3 grid(nstrip * nseg), block(NT);
    auto go = [&](auto kind_c) {
        constexpr int K = decltype(kind_c)::value;
        if (a.lim) hipLaunchKernelGGL((k_stage1d_lim<T, W, NT, K>), grid, block, 0, stream, a);
        else hipLaunchKernelGGL((k_stage1d<T, W, NT, K>), grid, block, 0, stream, a);
        return true;
    };
    bool ok = false;
    switch (kind) {
    case kRhs: ok = go(std::integral_constant<int, kRhs>{}); break;
    case kLean1: ok = go(std::integral_constant<int, kLean1>{}); break;
    case kLean2: ok = go(std::integral_constant<int, kLean2>{}); break;
    case kLean3: ok = go(std::integral_constant<int, kLean3>{}); break;
    case kLean4: ok = go(std::integral_constant<int, kLean4>{}); break;
    default: break;
    }
    if (!ok) return hipErrorInvalidValue;
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

// LDS doubles of k_poisson1d for nx cells: the padded r (and later d)
// array over [-K, nx + K + 8) and the padded y array over [0, nx)
size_t poisson1d_lds_doubles(int nx)
{
    int lc = 0;
    while ((kPoissonThreads << lc) < nx) ++lc;
    auto pad = [&](size_t j) { return j + (j >> lc); };
    return pad((size_t)nx + 2 * kGreenTaps + 8) + 1 + pad((size_t)nx) + 1;
}

hipError_t poisson1d_prepare()
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(k_poisson1d),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(poisson1d_lds_doubles(kMaxPoisson1D) * sizeof(double)));
}

hipError_t launch_poisson1d(const double* part, int nstrip, const double* n_in, double dv, int nx,
                            double dx, double qm, const double* green, int gk, double* n_out,
                            double* phi, double* E, double* a, hipStream_t stream)
{
    // with partial sums the kernel forms the moment itself (n_out unused)
    (void)n_out;
    PoissonExtra X{};
    if (part) {
        X.part = part;
        X.nstrip = nstrip;
        X.dv = dv;
    }
    const size_t lds = poisson1d_lds_doubles(nx) * sizeof(double);
    hipLaunchKernelGGL(k_poisson1d, dim3(1), dim3(kPoissonThreads), lds, stream, n_in, nx, dx, qm, green, gk,
                       phi, E, a, 0, 1.0, X);
    return hipGetLastError();
}

hipError_t launch_poisson1d_levels(const double* n_in, int nx, double dx, double qm, const double* green, int gk,
                                   double* E, double* a, int L, const int* off, const int* rt, hipStream_t stream)
{
    if (!n_in || !a || L < 1 || L > kHierLevels) return hipErrorInvalidValue;
    PoissonExtra X{};
    X.inject_L = L;
    for (int l = 0; l < L; ++l) {
        if (rt[l] < 1 || nx % rt[l]) return hipErrorInvalidValue;
        X.inject_off[l] = off[l];
        X.inject_rt[l] = rt[l];
    }
    const size_t lds = poisson1d_lds_doubles(nx) * sizeof(double);
    hipLaunchKernelGGL(k_poisson1d, dim3(1), dim3(kPoissonThreads), lds, stream, n_in, nx, dx, qm, green, gk,
                       nullptr, E, a, 0, 1.0, X);
    return hipGetLastError();
}

hipError_t launch_poisson1d_inject(const double* n_in, const PoissonExtra& x, int nx, double dx, double qm,
                                   const double* green, int gk, double* E, double* a, hipStream_t stream)
{
    if ((!x.slots && !n_in) || !a || x.inject_R < 1 || nx % x.inject_R) return hipErrorInvalidValue;
    const size_t lds = poisson1d_lds_doubles(nx) * sizeof(double);
    hipLaunchKernelGGL(k_poisson1d, dim3(1), dim3(kPoissonThreads), lds, stream, n_in, nx, dx, qm, green, gk,
                       nullptr, E, a, 0, 1.0, x);
    return hipGetLastError();
}

hipError_t launch_field_split(const double* part, int nstrip, int nx, double dv, double dx, double qm,
                              const double* green, double* work, double* a, hipStream_t stream)
{
    if (nx < kFieldSplitMin || nx > kMaxPoisson1D) return hipErrorInvalidValue;
    const int nchunk = (nx + kFieldChunk - 1) / kFieldChunk;
    double* y = work;
    double* csum = work + nx;
    SpeciesMoments m{};
    m.part[0] = part;
    m.nstrip[0] = nstrip;
    m.w[0] = -dv;
    m.ns = 1;
    m.background = 1.0;
    FieldOutputs out{};
    out.a[0] = a;
    out.qm[0] = qm;
    out.n = 1;
    hipLaunchKernelGGL(k_field_chunks, dim3(nchunk), dim3(kFieldChunk), 0, stream, m, nx, dx, green, y, csum);
    hipLaunchKernelGGL(k_field_finish, dim3(nchunk), dim3(kFieldChunk), 0, stream, y, csum, nchunk, nx, dx, out);
    return hipGetLastError();
}

hipError_t launch_field_split_species(const SpeciesMoments& m, int nx, double dx, const double* green, double* work,
                                      const FieldOutputs& out, hipStream_t stream)
{
    if (nx < kFieldSplitMin || nx > kMaxPoisson1D || m.ns < 1 || m.ns > kMaxSpecies || out.n < 0 ||
        out.n > kMaxSpecies + 1)
        return hipErrorInvalidValue;
    if (out.inject_R > 0 && (!out.inject_a || kFieldChunk % out.inject_R || nx % out.inject_R))
        return hipErrorInvalidValue;
    const int nchunk = (nx + kFieldChunk - 1) / kFieldChunk;
    double* y = work;
    double* csum = work + nx;
    hipLaunchKernelGGL(k_field_chunks, dim3(nchunk), dim3(kFieldChunk), 0, stream, m, nx, dx, green, y, csum);
    hipLaunchKernelGGL(k_field_finish, dim3(nchunk), dim3(kFieldChunk), 0, stream, y, csum, nchunk, nx, dx, out);
    return hipGetLastError();
}

hipError_t launch_poisson1d_adjoint(const double* part, int nstrip, int nx, double dx, double dv, double qm,
                                    const double* green, int gk, double* abar_out, double* z, hipStream_t stream)
{
    // with partial sums the kernel sums them (and keeps abar in abar_out)
    PoissonExtra X{};
    if (part) {
        X.part = part;
        X.nstrip = nstrip;
        X.dv = 1.0;
        X.n_out = abar_out;
    }
    const size_t lds = poisson1d_lds_doubles(nx) * sizeof(double);
    hipLaunchKernelGGL(k_poisson1d, dim3(1), dim3(kPoissonThreads), lds, stream, abar_out, nx, dx, qm, green,
                       gk, z, nullptr, nullptr, 1, -dv, X);
    return hipGetLastError();
}

__global__ void k_row_broadcast(const double* __restrict__ z, int nv, size_t total, double* __restrict__ out)
{
    const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (p < total) out[p] = z[p / nv];
}

hipError_t launch_row_broadcast(const double* z, int nx, int nv, double* out, hipStream_t stream)
{
    const size_t total = (size_t)nx * nv;
    hipLaunchKernelGGL(k_row_broadcast, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, z, nv, total,
                       out);
    return hipGetLastError();
}

hipError_t launch_scale(const double* x, double s, double* y, int n, hipStream_t stream)
{
    hipLaunchKernelGGL(k_scale, dim3((n + 255) / 256), dim3(256), 0, stream, x, s, y, n);
    return hipGetLastError();
}

hipError_t launch_species_neff(const SpeciesMoments& m, int nx, double* n_eff, hipStream_t stream)
{
    if (m.ns < 1 || m.ns > kMaxSpecies) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_species_neff, dim3((nx + 255) / 256), dim3(256), 0, stream, m, nx, n_eff);
    return hipGetLastError();
}

}  // namespace vp
