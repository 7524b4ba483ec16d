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

// Stage kernel.  A block owns a strip of TV = NT*W velocity cells and a
// segment of configuration rows [i0, i1).  The march proceeds in batches
// of RB rows: all loads of a batch (RB new rows of the stage state plus the
// f^n / accumulator rows being updated) are issued together, so each wave
// keeps RB rows of traffic in flight; the rows go through an 8-slot LDS
// ring that holds the stencil's x-neighbourhood rows i-2 .. i+RB+1.
template <typename T, int W, int NT, int KIND>
__global__ __launch_bounds__(NT) void k_stage1d(Stage1DArgs A)
{
    constexpr int RB = 4;                                    // rows per batch
    constexpr int NSLOT = 8;                                 // ring rows (>= RB + 4)
    constexpr int TV = NT * W;
    constexpr int LPAD = (W > 2) ? W : 2;                    // keeps own data W-aligned in LDS
    constexpr int RW = ((LPAD + TV + 2 + 3) / 4) * 4;
    constexpr int NWAVE = NT / 64;
    __shared__ __attribute__((aligned(16))) T ring[NSLOT][RW];
    __shared__ double mom[NWAVE][kMaxTx];
    __shared__ double aseg[kMaxTx + RB + 2];   // a_{i0-1} .. a_{i1}, then padding

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
    const int jld = own_in ? jt : 0;      // out-of-range threads load a valid cell and discard it
    const int lane = t & 63, wave = t >> 6;
    const int c0 = LPAD + t * W;          // LDS column of the first own cell

    // values of own cells that lie outside [0, nv): velocity ghosts or unused
    T oconst[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int j = jt + w;
        oconst[w] = (j == nv) ? (T)A.vg[2] : (j == nv + 1) ? (T)A.vg[3] : T(0);
    }
    // threads 0..3 also stage one strip-halo cell: j0-2, j0-1, j0+TV, j0+TV+1
    const bool has_halo = t < 4;
    const int hj = t < 2 ? j0 - 2 + t : j0 + TV + (t - 2);
    const int hcol = t < 2 ? LPAD - 2 + t : LPAD + TV + (t - 2);
    const bool halo_in = has_halo && hj >= 0 && hj < nv;
    const int hld = halo_in ? hj : jld;
    const T hconst = (hj == -2) ? (T)A.vg[0] : (hj == -1) ? (T)A.vg[1] : (hj == nv) ? (T)A.vg[2]
                   : (hj == nv + 1) ? (T)A.vg[3] : T(0);

    auto slot_of = [&](int r) { return (r - i0 + 2) & (NSLOT - 1); };   // r >= i0 - 2
    auto load_row = [&](int r, T* v, T& h) {
        const T* row = fs + (size_t)wrapi(r, nx) * nv;
        VecIO<T, W>::ld(row + jld, v);
        h = row[hld];
    };
    auto store_row = [&](int r, const T* v, T h) {
        T* dst = &ring[slot_of(r)][0];
#pragma unroll
        for (int w = 0; w < W; ++w) dst[c0 + w] = own_in ? v[w] : oconst[w];
        if (has_halo) dst[hcol] = halo_in ? h : hconst;
    };
    auto fx_cols = [&](int r, T* Fx) {      // x-face r + 1/2 at columns jt-1 .. jt+W
        const int sm1 = slot_of(r - 1), s0 = slot_of(r), s1 = slot_of(r + 1), s2 = slot_of(r + 2);
#pragma unroll
        for (int q = 0; q < W + 2; ++q) {
            const int c = c0 - 1 + q;
            Fx[q] = face4<T>(ring[sm1][c], ring[s0][c], ring[s1][c], ring[s2][c]);
        }
    };
    auto fv_faces = [&](int r, T* Fv) {     // v-faces jt-1/2 .. jt+W-1/2 of row r
        const int sl = slot_of(r);
        T u[W + 4];
#pragma unroll
        for (int q = 0; q < W + 4; ++q) u[q] = ring[sl][c0 - 2 + q];
#pragma unroll
        for (int m = 0; m <= W; ++m) Fv[m] = face4<T>(u[m], u[m + 1], u[m + 2], u[m + 3]);
    };

    T vb[W];
#pragma unroll
    for (int w = 0; w < W; ++w) vb[w] = (T)(A.v_lo + ((double)(jt + w) + 0.5) * A.dv);
    const T dxi = (T)A.dxi, dvi = (T)A.dvi, dv24 = (T)A.dv24;
    const T cacc = (T)A.c_acc, cnext = (T)A.c_next;

    // ---- prologue: rows i0-2 .. i0+1
    {
        T v[4][W], h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) load_row(i0 - 2 + q, v[q], h[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q) store_row(i0 - 2 + q, v[q], h[q]);
    }
    for (int q = t; q < i1 - i0 + 2; q += NT) aseg[q] = av[wrapi(i0 - 1 + q, nx)];
    for (int q = i1 - i0 + 2 + t; q < kMaxTx + RB + 2; q += NT) aseg[q] = 0.0;
    __syncthreads();

    T gx_old[W];
    {
        T Fx[W + 2];
        fx_cols(i0 - 1, Fx);
#pragma unroll
        for (int w = 0; w < W; ++w) gx_old[w] = vb[w] * Fx[w + 1] + dv24 * (Fx[w + 2] - Fx[w]);
    }
    T fvA[W + 1], fvB[W + 1];
    fv_faces(i0 - 1, fvA);
    fv_faces(i0, fvB);

#pragma unroll 1
    for (int ib = i0; ib < i1; ib += RB) {
        // issue every load of the batch; indices past the segment are clamped
        // so that all loads and their uses are unconditional
        T v[RB][W], h[RB], fnv[RB][W], accv[RB][W];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            load_row(min(ib + 2 + q, i1 + 1), v[q], h[q]);      // new stage-state row
            const size_t off = (size_t)min(ib + q, i1 - 1) * nv + jld;
            if (KIND == kStage23) VecIO<T, W>::ld(fn + off, fnv[q]);
            if (KIND == kStage23 || KIND == kStage4) VecIO<T, W>::ld(acc + off, accv[q]);
        }
        __syncthreads();                              // previous batch done reading its ring rows
#pragma unroll
        for (int q = 0; q < RB; ++q) store_row(ib + 2 + q, v[q], h[q]);
        __syncthreads();

        // compute the batch (rows past the segment are computed and dropped);
        // results stay in registers and are stored together
        T o1[RB][W], o2[RB][W];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int i = ib + q;
            const int qa = i - i0;
            const T a_m1 = (T)aseg[qa], a_0 = (T)aseg[qa + 1], a_p1 = (T)aseg[qa + 2];
            T Fx[W + 2];
            fx_cols(i, Fx);
            T fvC[W + 1];
            fv_faces(i + 1, fvC);
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
#pragma unroll
            for (int m = 0; m <= W; ++m) { fvA[m] = fvB[m]; fvB[m] = fvC[m]; }

            if (KIND == kRhs) {
#pragma unroll
                for (int w = 0; w < W; ++w) o1[q][w] = kk[w];
            } else if (KIND == kStage1) {
                // f^n is the stage state itself: take it from the ring
                const int sl = slot_of(i);
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const T f0 = ring[sl][c0 + w];
                    o1[q][w] = f0 + cacc * kk[w];      // accumulator
                    o2[q][w] = f0 + cnext * kk[w];     // next predictor
                }
            } else if (KIND == kStage23) {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    o1[q][w] = accv[q][w] + cacc * kk[w];
                    o2[q][w] = fnv[q][w] + cnext * kk[w];
                }
            } else {  // kStage4: f^{n+1} = acc + dt/6 k4
#pragma unroll
                for (int w = 0; w < W; ++w) o2[q][w] = accv[q][w] + cacc * kk[w];
            }
            if (KIND != kRhs && A.part) {
                double sm = 0.0;
                if (own_in) {
#pragma unroll
                    for (int w = 0; w < W; ++w) sm += (double)o2[q][w];
                }
                sm = wave_sum(sm);
                if (lane == 0 && i < i1) mom[wave][qa] = sm;
            }
        }
        if (own_in) {
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int i = ib + q;
                if (i < i1) {
                    const size_t rowoff = (size_t)i * nv + jt;
                    if (KIND == kRhs) {
                        VecIO<T, W>::st(fout + rowoff, o1[q]);
                    } else if (KIND == kStage4) {
                        VecIO<T, W>::st(fout + rowoff, o2[q]);
                    } else {
                        VecIO<T, W>::st(acc + rowoff, o1[q]);
                        VecIO<T, W>::st(fout + rowoff, o2[q]);
                    }
                }
            }
        }
    }

    if (KIND != kRhs && A.part) {
        __syncthreads();
        for (int q = t; q < i1 - i0; q += NT) {
            double sm = 0.0;
#pragma unroll
            for (int wv = 0; wv < NWAVE; ++wv) sm += mom[wv][q];
            A.part[(size_t)strip * nx + i0 + q] = sm;
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

// n_i = dv * sum over strips of the stage kernel's per-strip partial sums,
// one row per thread with all strip loads in flight, fixed summation order.
__global__ __launch_bounds__(256) void k_moment_finalize(const double* __restrict__ part, int nstrip, int nx,
                                                        double dv, double* __restrict__ n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= nx) return;
    double acc = 0.0;
    for (int q0 = 0; q0 < nstrip; q0 += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = (q0 + u < nstrip) ? part[(size_t)(q0 + u) * nx + i] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) acc += v[u];
    }
    n[i] = dv * acc;
}

// adjoint = 0: r = 12 dx^2 (1 - n) from the moment n_in; outputs phi, E, a.
// adjoint = 1: n_in holds abar; r = 12 dx^2 D (q/m) abar (D the field
// stencil without its sign); phi_out receives phi_scale * S r / (12 dx^2)-
// solution, i.e. z = -dv S D (q/m) abar with phi_scale = -dv.
__global__ __launch_bounds__(kPoissonThreads) void k_poisson1d(
    const double* __restrict__ n_in, int nx, double dx, double qm, const double* __restrict__ green, int gk,
    double* __restrict__ phi_out, double* __restrict__ E_out, double* __restrict__ a_out, int adjoint,
    double phi_scale)
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
#pragma unroll
        for (int m = 0; m < RM; ++m) {
            const int i = t + m * kPoissonThreads;
            nv[m] = i < nx ? n_in[i] : 0.0;
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
        if (a_out) a_out[i] = qm * E;
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
    // with partial sums: finalise the moment into n_out first (n_out is required)
    if (part) {
        if (!n_out) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_moment_finalize, dim3((nx + 255) / 256), dim3(256), 0, stream, part, nstrip, nx,
                           dv, n_out);
        n_in = n_out;
    }
    const size_t lds = poisson1d_lds_doubles(nx) * sizeof(double);
    hipLaunchKernelGGL(k_poisson1d, dim3(1), dim3(kPoissonThreads), lds, stream, n_in, nx, dx, qm, green, gk,
                       phi, E, a, 0, 1.0);
    return hipGetLastError();
}

hipError_t launch_poisson1d_adjoint(const double* part, int nstrip, int nx, double dx, double dv, double qm,
                                    const double* green, int gk, double* abar_out, double* z, hipStream_t stream)
{
    if (part)
        hipLaunchKernelGGL(k_moment_finalize, dim3((nx + 255) / 256), dim3(256), 0, stream, part, nstrip, nx, 1.0,
                           abar_out);
    const size_t lds = poisson1d_lds_doubles(nx) * sizeof(double);
    hipLaunchKernelGGL(k_poisson1d, dim3(1), dim3(kPoissonThreads), lds, stream, abar_out, nx, dx, qm, green,
                       gk, z, nullptr, nullptr, 1, -dv);
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

}  // namespace vp
