// Device-side building blocks of the 1D+1V stage kernels, shared by the
// single-level kernels and the two-level persistent kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>

#include "vp_internal.hpp"

namespace vp {
namespace dev {

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

// W consecutive elements per thread.  ld/st are ordinary accesses; ldn/stn
// are non-temporal (streamed data read or written once per launch).
typedef double vd2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));
template <typename T, int W> struct VecIO;
template <> struct VecIO<double, 1> {
    static __device__ __forceinline__ void ld(const double* p, double* o) { o[0] = p[0]; }
    static __device__ __forceinline__ void st(double* p, const double* o) { p[0] = o[0]; }
    static __device__ __forceinline__ void ldn(const double* p, double* o) { o[0] = __builtin_nontemporal_load(p); }
    static __device__ __forceinline__ void stn(double* p, const double* o) { __builtin_nontemporal_store(o[0], p); }
};
template <> struct VecIO<double, 2> {
    static __device__ __forceinline__ void ld(const double* p, double* o)
    {
        const vd2 v = *reinterpret_cast<const vd2*>(p);
        o[0] = v.x; o[1] = v.y;
    }
    static __device__ __forceinline__ void st(double* p, const double* o)
    {
        *reinterpret_cast<vd2*>(p) = vd2{o[0], o[1]};
    }
    static __device__ __forceinline__ void ldn(const double* p, double* o)
    {
        const vd2 v = __builtin_nontemporal_load(reinterpret_cast<const vd2*>(p));
        o[0] = v.x; o[1] = v.y;
    }
    static __device__ __forceinline__ void stn(double* p, const double* o)
    {
        __builtin_nontemporal_store(vd2{o[0], o[1]}, reinterpret_cast<vd2*>(p));
    }
};
template <> struct VecIO<float, 1> {
    static __device__ __forceinline__ void ld(const float* p, float* o) { o[0] = p[0]; }
    static __device__ __forceinline__ void st(float* p, const float* o) { p[0] = o[0]; }
    static __device__ __forceinline__ void ldn(const float* p, float* o) { o[0] = __builtin_nontemporal_load(p); }
    static __device__ __forceinline__ void stn(float* p, const float* o) { __builtin_nontemporal_store(o[0], p); }
};
template <> struct VecIO<float, 4> {
    static __device__ __forceinline__ void ld(const float* p, float* o)
    {
        const vf4 v = *reinterpret_cast<const vf4*>(p);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
    static __device__ __forceinline__ void st(float* p, const float* o)
    {
        *reinterpret_cast<vf4*>(p) = vf4{o[0], o[1], o[2], o[3]};
    }
    static __device__ __forceinline__ void ldn(const float* p, float* o)
    {
        const vf4 v = __builtin_nontemporal_load(reinterpret_cast<const vf4*>(p));
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
    static __device__ __forceinline__ void stn(float* p, const float* o)
    {
        __builtin_nontemporal_store(vf4{o[0], o[1], o[2], o[3]}, reinterpret_cast<vf4*>(p));
    }
};

// x moved across lanes by the DPP pattern CTRL (a permutation within each
// row of 16 lanes), as two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over each row of 16 lanes, the same value in every lane of the row:
// neighbours within quads (quad_perm 1,0,3,2), the other pair of the quad
// (quad_perm 2,3,0,1), the other quad of the half row (row_half_mirror),
// the other half row (row_mirror).
__device__ __forceinline__ double row16_sum(double s)
{
    s += dpp_f64<0xB1>(s);
    s += dpp_f64<0x4E>(s);
    s += dpp_f64<0x141>(s);
    s += dpp_f64<0x140>(s);
    return s;
}

// Wave sums of four values per lane: returns, in every lane of lane group
// g = lane / 16, the sum of s[g] over the 64 lanes.  Lanes l and l ^ 32
// trade the two rows the other half keeps (rows 0, 1 stay in the lower
// half, rows 2, 3 in the upper one), then lanes l and l ^ 16 trade one of
// those, and a reduction within the 16 lanes finishes the sum.
__device__ __forceinline__ double wave_sum4(const double (&s)[4], int lane)
{
    const bool hi = (lane & 32) != 0, mid = (lane & 16) != 0;
    const double t0 = (hi ? s[2] : s[0]) + __shfl_xor(hi ? s[0] : s[2], 32, 64);
    const double t1 = (hi ? s[3] : s[1]) + __shfl_xor(hi ? s[1] : s[3], 32, 64);
    const double u = (mid ? t1 : t0) + __shfl_xor(mid ? t0 : t1, 16, 64);
    return row16_sum(u);
}

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

// lo + x h rounded after the product and after the sum (never fused)
__device__ __forceinline__ double centre_unfused(double lo, double x, double h)
{
#pragma clang fp contract(off)
    const double p = x * h;
    return lo + p;
}

// 1 / d for d > 0: the hardware estimate refined by Newton-Raphson steps
// r <- r + r (1 - d r), each of which squares the relative error
__device__ __forceinline__ double recip_nr(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return fma(r, fma(-d, r, 1.0), r);
}
__device__ __forceinline__ float recip_nr(float d)
{
    const float r = __builtin_amdgcn_rcpf(d);
    return fmaf(r, fmaf(-d, r, 1.0f), r);
}

// Limited face average between u0 and u1 (section 2, eq. limitedFace): the
// left- and right-biased third-order candidates (eqs. thirdLeft,
// thirdRight) weighted by provisional WENO weights from the Jiang-Shu
// smoothness of their stencils (ideal weights 1/2, epsilon 1e-6, power 2),
// the larger weight given to the upwind candidate (upl: flow towards +).
// With s = (beta + eps)^2 the provisional left weight is s_r / (s_l + s_r),
// the larger weight max(s_l, s_r) / (s_l + s_r), and the face
// w_l f_l + w_r f_r = f_r + w_l (f_l - f_r).
template <typename T>
__device__ __forceinline__ T face_lim(T um1, T u0, T u1, T u2, bool upl)
{
    const T fr = (T(2) * u0 + T(5) * u1 - u2) * T(1.0 / 6.0);
    const T dlr = (T(3) * (u0 - u1) + (u2 - um1)) * T(1.0 / 6.0);     // f_l - f_r
    const T d1 = um1 - T(2) * u0 + u1, e1 = um1 - u1;
    const T d2 = u0 - T(2) * u1 + u2, e2 = T(3) * u0 - T(4) * u1 + u2;
    const T bl = T(13.0 / 12.0) * d1 * d1 + T(0.25) * e1 * e1 + T(1e-6);
    const T br = T(13.0 / 12.0) * d2 * d2 + T(0.25) * e2 * e2 + T(1e-6);
    const T sl = bl * bl, sr = br * br;
    const T wmax = (sl > sr ? sl : sr) * recip_nr(sl + sr);
    return fr + (upl ? wmax : T(1) - wmax) * dlr;
}

// x moved by the wave-wide DPP shift CTRL (wave_shl:1 = 0x130: lane l reads
// lane l + 1; wave_shr:1 = 0x138: lane l reads lane l - 1); the lane with no
// source receives an unspecified value, which the callers replace
constexpr int kWaveShl1 = 0x130;
constexpr int kWaveShr1 = 0x138;
template <int CTRL>
__device__ __forceinline__ double wave_shift(double x) { return dpp_f64<CTRL>(x); }
template <int CTRL>
__device__ __forceinline__ float wave_shift(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

// Stage kernel.  A block owns a strip of TV = NT*W velocity cells and a
// segment of configuration rows [i0, i1).  The march proceeds in batches
// of RB rows: all loads of a batch (RB new rows of the stage state plus the
// f^n / accumulator rows being updated) are issued together, so each wave
// keeps RB rows of traffic in flight; the rows go through an 8-slot LDS
// ring that holds the stencil's x-neighbourhood rows i-2 .. i+RB+1.
// Even segments march towards increasing x and odd segments towards
// decreasing x, so two neighbouring segments reach the rows they share
// (each other's two halo rows) at about the same time, while those rows
// are still in L2.  Every face flux is formed from the same four rows in
// either direction, so the results do not depend on the direction.
template <typename T, int W, int NT, int KIND, bool LIM = false>
__device__ __forceinline__ void stage_tile_uniform(const Stage1DArgs& A, int tile)
{
    constexpr int RB = 4;                                    // rows per batch
    constexpr int NSLOT = 8;                                 // ring rows (>= RB + 4)
    constexpr int TV = NT * W;
    constexpr int PW = NT + 4;                               // plane width: lane slots -2 .. NT+1
    constexpr int NWAVE = NT / 64;
    // A ring row is stored as W planes: column j0 + W*u + w (w < W) sits in
    // plane w at index u + 2.  Lanes then read and write consecutive 8-byte
    // words of one plane, which is free of LDS bank conflicts, where a
    // row-major row would put a W*8-byte stride between lanes.
    __shared__ __attribute__((aligned(16))) T ring[NSLOT][W][PW];
    __shared__ double mom[NWAVE][kMaxTx];
    __shared__ double aseg[kMaxTx + RB + 2];   // a_{i0-1} .. a_{i1}, then padding

    const T* __restrict__ fs = static_cast<const T*>(A.fs);
    const T* __restrict__ fn = static_cast<const T*>(A.fn);
    T* __restrict__ acc = static_cast<T*>(A.acc);
    T* __restrict__ fout = static_cast<T*>(A.fout);
    const double* __restrict__ av = A.a;

    const int nx = A.nx, nv = A.nv;
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
    const int hu = (hj - j0 + 2 * W);                 // >= 0
    const int hplane = hu % W, hidx = hu / W;         // plane index (u + 2) of the halo cell
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
    // column jt + m of this thread, m in [-2, W + 1] (a compile-time constant)
    auto cell = [&](int sl, int m) -> T& {
        return ring[sl][(m + 2 * W) % W][t + (m + 2 * W) / W];
    };
    auto store_row = [&](int r, const T* v, T h) {
        const int sl = slot_of(r);
#pragma unroll
        for (int w = 0; w < W; ++w) cell(sl, w) = own_in ? v[w] : oconst[w];
        if (has_halo) ring[sl][hplane][hidx] = halo_in ? h : hconst;
    };
    // limited faces: x faces are upwinded by the sign of the column velocity,
    // v faces by the sign of the row's acceleration.  The cell-centre
    // velocity is rounded after the product and after the sum (no fused
    // multiply-add), so that a centre velocity that is zero in exact
    // arithmetic gets the same sign as in an unfused evaluation of
    // v_lo + (j + 1/2) dv.
    bool upx[W + 2];
#pragma unroll
    for (int q = 0; q < W + 2; ++q) upx[q] = centre_unfused(A.v_lo, (double)(jt - 1 + q) + 0.5, A.dv) > 0.0;
    T vb[W];
#pragma unroll
    for (int w = 0; w < W; ++w) vb[w] = (T)(A.v_lo + ((double)(jt + w) + 0.5) * A.dv);
    const T dxi = (T)A.dxi, dvi = (T)A.dvi, dv24 = (T)A.dv24;
    const T cacc = (T)A.c_acc, cnext = (T)A.c_next;

    const int len = i1 - i0;
    static_assert(RB == 4, "the batch reduction of the velocity moments folds four rows");

    // The march runs towards increasing x on even segments and towards
    // decreasing x on odd ones; each direction is compiled separately so
    // that the direction costs no selects in the loop.
    auto march = [&](auto dn_c) {
        constexpr bool DN = decltype(dn_c)::value;
        constexpr int D = DN ? -1 : 1;
        const int ifirst = DN ? i1 - 1 : i0;          // first output row of the march

        // ---- prologue: the four rows around the first output row
        {
            T v[4][W], h[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) load_row(ifirst + D * (q - 2), v[q], h[q]);
#pragma unroll
            for (int q = 0; q < 4; ++q) store_row(ifirst + D * (q - 2), v[q], h[q]);
        }
        for (int q = t; q < i1 - i0 + 2; q += NT) aseg[q] = av[wrapi(i0 - 1 + q, nx)];
        for (int q = i1 - i0 + 2 + t; q < kMaxTx + RB + 2; q += NT) aseg[q] = 0.0;
        __syncthreads();

        // The march window: rows i - D, i, i + D, i + 2D around the current row
        // i, columns jt - 2 .. jt + W + 1, held in registers, so that every ring
        // row is read from LDS once on its way through the window.
        T win[4][W + 4];
        auto load_win = [&](int r, T* u) {
            const int sl = slot_of(r);
#pragma unroll
            for (int q = 0; q < W + 4; ++q) u[q] = cell(sl, q - 2);
        };
        // x faces at columns jt-1 .. jt+W between the middle two of four rows
        // given in march order (taken in increasing x for the face average)
        auto fx_rows = [&](const T* r0, const T* r1, const T* r2, const T* r3, T* Fx) {
            const T* um1 = DN ? r3 : r0;
            const T* u0 = DN ? r2 : r1;
            const T* u1 = DN ? r1 : r2;
            const T* u2 = DN ? r0 : r3;
            if (LIM) {
                // limited faces are costly: each thread evaluates those of its
                // own W columns and takes the two next to them from the
                // neighbouring lanes; lanes at the ends of the wave evaluate
                // theirs (one face per thread: column jt - 1 in lane 0, jt + W
                // in lane 63)
#pragma unroll
                for (int q = 1; q <= W; ++q) Fx[q] = face_lim<T>(um1[q + 1], u0[q + 1], u1[q + 1], u2[q + 1], upx[q]);
                const bool rt = lane == 63;
                const T fe = face_lim<T>(rt ? um1[W + 2] : um1[1], rt ? u0[W + 2] : u0[1], rt ? u1[W + 2] : u1[1],
                                         rt ? u2[W + 2] : u2[1], rt ? upx[W + 1] : upx[0]);
                const T fprev = wave_shift<kWaveShr1>(Fx[W]), fnext = wave_shift<kWaveShl1>(Fx[1]);
                Fx[0] = lane == 0 ? fe : fprev;
                Fx[W + 1] = rt ? fe : fnext;
            } else {
#pragma unroll
                for (int q = 0; q < W + 2; ++q) Fx[q] = face4<T>(um1[q + 1], u0[q + 1], u1[q + 1], u2[q + 1]);
            }
        };
        // v faces jt-1/2 .. jt+W-1/2 of window row u (row r)
        auto fv_row = [&](const T* u, int r, T* Fv) {
            const bool upv = LIM && aseg[max(r - i0 + 1, 0)] > 0.0;
#pragma unroll
            for (int m = 0; m <= W; ++m) {
                if (LIM) Fv[m] = face_lim<T>(u[m], u[m + 1], u[m + 2], u[m + 3], upv);
                else Fv[m] = face4<T>(u[m], u[m + 1], u[m + 2], u[m + 3]);
            }
        };

        // x-flux on the face behind the first row, v-face averages of the row
        // behind and of the first row
        T gx_old[W];
        T fvP[W + 1], fvB[W + 1];
        {
            T pre[W + 4];
            load_win(ifirst - 2 * D, pre);
            load_win(ifirst - D, win[0]);
            load_win(ifirst, win[1]);
            load_win(ifirst + D, win[2]);
            T Fx[W + 2];
            fx_rows(pre, win[0], win[1], win[2], Fx);
#pragma unroll
            for (int w = 0; w < W; ++w) gx_old[w] = vb[w] * Fx[w + 1] + dv24 * (Fx[w + 2] - Fx[w]);
            fv_row(win[0], ifirst - D, fvP);
            fv_row(win[1], ifirst, fvB);
        }

        // The new stage-state rows of batch mb are rows mb + 2 .. mb + RB + 1 of
        // the march (the rows ahead of the batch's output rows); rows past the
        // segment are clamped so that all loads and their uses are unconditional.
        auto load_batch = [&](int mb, T (*v)[W], T* h) {
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int rn = ifirst + D * (mb + q + 2);
                load_row(DN ? max(rn, i0 - 2) : min(rn, i1 + 1), v[q], h[q]);
            }
        };
        auto store_batch = [&](int mb, T (*v)[W], T* h) {
#pragma unroll
            for (int q = 0; q < RB; ++q) store_row(ifirst + D * (mb + q + 2), v[q], h[q]);
        };
        // Stages that stream few words per cell load the rows of the next batch
        // while the current one is computed (the rows stay in registers until
        // the ring slots they replace are free); the others load a batch just
        // before computing it.
        constexpr bool PF = KIND == kLean1;
        if (PF) {
            T v[RB][W], h[RB];
            load_batch(0, v, h);
            store_batch(0, v, h);
            __syncthreads();
        }

#pragma unroll 1
        for (int mb = 0; mb < len; mb += RB) {
            T v[RB][W], h[RB], fnv[RB][W], accv[RB][W];
            const bool more = mb + RB < len;
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                if (!PF) {
                    const int rn = ifirst + D * (mb + q + 2);
                    load_row(DN ? max(rn, i0 - 2) : min(rn, i1 + 1), v[q], h[q]);
                }
                const int ro = ifirst + D * min(mb + q, len - 1);              // row being updated
                const size_t off = (size_t)ro * nv + jld;
                if (KIND == kStage23 || KIND == kLean2 || KIND == kLean3) VecIO<T, W>::ldn(fn + off, fnv[q]);
                if (KIND == kStage23 || KIND == kStage4 || KIND == kLean4) VecIO<T, W>::ldn(acc + off, accv[q]);
            }
            // The prefetch is issued after the loads this batch consumes (loads
            // complete in order, so this batch does not wait for the prefetch)
            // and unconditionally, clamped past the segment (a load under a
            // branch makes the compiler wait for it before the compute).
            if (PF) load_batch(mb + RB, v, h);
            if (!PF) {
                __syncthreads();                          // previous batch done reading its ring rows
                store_batch(mb, v, h);
                __syncthreads();
            }

            // compute the batch (rows past the segment are computed and dropped);
            // results stay in registers and are stored together
            T o1[RB][W], o2[RB][W];
            double sm4[RB];                           // velocity sums of the batch's new rows
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int i = ifirst + D * (mb + q);
                const int qa = i - i0;
                const int qc = max(qa, 0);                // rows past a downward segment are dropped
                const T a_m1 = (T)aseg[qc], a_0 = (T)aseg[qc + 1], a_p1 = (T)aseg[qc + 2];
                load_win(i + 2 * D, win[3]);
                T Fx[W + 2];
                fx_rows(win[0], win[1], win[2], win[3], Fx);   // the face ahead of row i
                T fvN[W + 1];
                fv_row(win[2], i + D, fvN);               // the row ahead
                const T da48 = (a_p1 - a_m1) * T(1.0 / 48.0);
                T gv[W + 1];
#pragma unroll
                for (int m = 0; m <= W; ++m) {
                    const T fa = DN ? fvN[m] : fvP[m];    // row i - 1
                    const T fc = DN ? fvP[m] : fvN[m];    // row i + 1
                    gv[m] = a_0 * fvB[m] + da48 * (fc - fa);
                }
                T kk[W];
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const T gx_new = vb[w] * Fx[w + 1] + dv24 * (Fx[w + 2] - Fx[w]);
                    const T ghi = DN ? gx_old[w] : gx_new;   // face i + 1/2
                    const T glo = DN ? gx_new : gx_old[w];   // face i - 1/2
                    kk[w] = -(ghi - glo) * dxi - (gv[w + 1] - gv[w]) * dvi;
                    gx_old[w] = gx_new;
                }
#pragma unroll
                for (int m = 0; m <= W; ++m) { fvP[m] = fvB[m]; fvB[m] = fvN[m]; }

                if (KIND == kRhs) {
#pragma unroll
                    for (int w = 0; w < W; ++w) o1[q][w] = kk[w];
                } else if (KIND == kStage1) {
                    // f^n is the stage state itself: take it from the window
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const T f0 = win[1][w + 2];
                        o1[q][w] = f0 + cacc * kk[w];      // accumulator
                        o2[q][w] = f0 + cnext * kk[w];     // next predictor
                    }
                } else if (KIND == kStage23) {
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        o1[q][w] = accv[q][w] + cacc * kk[w];
                        o2[q][w] = fnv[q][w] + cnext * kk[w];
                    }
                } else if (KIND == kStage4) {  // f^{n+1} = acc + dt/6 k4
#pragma unroll
                    for (int w = 0; w < W; ++w) o2[q][w] = accv[q][w] + cacc * kk[w];
                } else if (KIND == kLean1) {   // f(2) = f^n + dt/2 k1, f^n from the window
#pragma unroll
                    for (int w = 0; w < W; ++w) o2[q][w] = win[1][w + 2] + cnext * kk[w];
                } else if (KIND == kLean2) {   // f(3), and acc from f(2) = the stage state
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const T f2 = win[1][w + 2];
                        o1[q][w] = (fnv[q][w] + f2) * T(1.0 / 3.0) + cacc * kk[w];
                        o2[q][w] = fnv[q][w] + cnext * kk[w];
                    }
                } else if (KIND == kLean3) {   // f(4) = f^n + dt k3
#pragma unroll
                    for (int w = 0; w < W; ++w) o2[q][w] = fnv[q][w] + cnext * kk[w];
                } else {                       // kLean4: f^{n+1} from acc and f(4) = the stage state
#pragma unroll
                    for (int w = 0; w < W; ++w) {
                        const T f4 = win[1][w + 2];
                        o2[q][w] = accv[q][w] + (f4 * T(1.0 / 3.0) + cacc * kk[w]);
                    }
                }
                sm4[q] = 0.0;
                if (own_in) {
#pragma unroll
                    for (int w = 0; w < W; ++w) sm4[q] += (double)o2[q][w];
                }
                if (own_in && mb + q < len) {
                    const size_t rowoff = (size_t)i * nv + jt;
                    if (KIND == kRhs) {
                        VecIO<T, W>::stn(fout + rowoff, o1[q]);
                    } else if (KIND == kStage4 || KIND == kLean1 || KIND == kLean3 || KIND == kLean4) {
                        VecIO<T, W>::stn(fout + rowoff, o2[q]);
                    } else {
                        VecIO<T, W>::stn(acc + rowoff, o1[q]);
                        VecIO<T, W>::stn(fout + rowoff, o2[q]);
                    }
                }
                // slide the window one row along the march
#pragma unroll
                for (int u = 0; u < W + 4; ++u) {
                    win[0][u] = win[1][u];
                    win[1][u] = win[2][u];
                    win[2][u] = win[3][u];
                }
            }
            if (KIND != kRhs && A.part) {
                const double tot = wave_sum4(sm4, lane);  // row q = lane / 16 of the batch
                const int g = lane >> 4;
                if ((lane & 15) == 0 && mb + g < len) mom[wave][ifirst + D * (mb + g) - i0] = tot;
            }
            if (PF && more) {
                __syncthreads();                          // this batch done reading its ring rows
                store_batch(mb + RB, v, h);
                __syncthreads();
            }
        }
    };
    if (seg & 1) march(std::true_type{});
    else march(std::false_type{});

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


}  // namespace dev
}  // namespace vp
