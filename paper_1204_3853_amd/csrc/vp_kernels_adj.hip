// HIP kernels of the discrete adjoint of the 1D+1V RK4 step (FP64).
//
// Reverse pass of one RK4 step (stages s = 4 .. 1) with lam the cotangent
// of f^{n+1}:
//   kbar_s  = dt b_s lam + dt alpha_{s+1} (g_{s+1} + z_{s+1})     (s < 4)
//   g_s     = (dL/df)^T kbar_s          transposed flux-divergence stencil at a(s)
//   abar_s  = (dL/da)^T kbar_s          a velocity reduction at the state f(s)
//   z_s     = -dv S D (q/m) abar_s      adjoint of moment -> Poisson -> field
//   lam_n   = lam + sum_s (g_s + z_s)
// (S the periodic Poisson solution operator, symmetric; D the fourth-order
// difference of the field, antisymmetric.)  The transposed stencil is
// written in gather form: each cell collects the cotangents of the face
// averages it enters, so the kernel has the forward kernel's structure: an
// x-march over a velocity strip with LDS rings of kbar rows and f(s) rows.
#include <hip/hip_runtime.h>

#include "vp_internal.hpp"

namespace vp {

namespace {

__device__ __forceinline__ int xcd_remap_a(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, l = b >> 3;
    return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

__device__ __forceinline__ int wrapa(int i, int n)
{
    if (i >= 0 && i < n) return i;
    int r = i % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ double wave_sum_a(double s)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
    return s;
}

__device__ __forceinline__ double face4a(double um1, double u0, double u1, double u2)
{
    return (7.0 * (u0 + u1) - (um1 + u2)) * (1.0 / 12.0);
}

template <int W> struct Vd;
template <> struct Vd<1> {
    static __device__ __forceinline__ void ld(const double* p, double* o) { o[0] = p[0]; }
    static __device__ __forceinline__ void st(double* p, const double* o) { p[0] = o[0]; }
};
template <> struct Vd<2> {
    static __device__ __forceinline__ void ld(const double* p, double* o)
    {
        const double2 v = *reinterpret_cast<const double2*>(p);
        o[0] = v.x; o[1] = v.y;
    }
    static __device__ __forceinline__ void st(double* p, const double* o)
    {
        *reinterpret_cast<double2*>(p) = make_double2(o[0], o[1]);
    }
};

// FIRST: s = 4 (kbar = c1 lam, no previous stage, no accumulator update)
template <int W, int NT, bool FIRST>
__global__ __launch_bounds__(NT) void k_adjoint_stage1d(Adjoint1DArgs A)
{
    constexpr int RB = 2;                       // rows per batch
    constexpr int NSLOT = 8;                    // ring rows (>= RB + 4)
    constexpr int TV = NT * W;
    constexpr int LPAD = 2;
    constexpr int RW = ((LPAD + TV + 2 + 1) / 2) * 2;
    constexpr int NWAVE = NT / 64;
    __shared__ __attribute__((aligned(16))) double KB[NSLOT][RW];   // kbar rows, 0 outside [0, nv)
    __shared__ __attribute__((aligned(16))) double FS[NSLOT][RW];   // f(s) rows, velocity ghosts filled
    __shared__ double mom[NWAVE][kMaxTx];
    __shared__ double aseg[kMaxTx + RB + 4];                         // a_{i0-2} .. a_{i1+1}, padding
    __shared__ double zseg[kMaxTx + RB + 4];                         // z_{s+1} at rows i0-2 .. i1+1

    const int nx = A.nx, nv = A.nv;
    const int tile = xcd_remap_a(blockIdx.x, gridDim.x);
    const int strip = tile % A.nstrip;
    const int seg = tile / A.nstrip;
    const int j0 = strip * TV;
    const int i0 = seg * A.tx;
    const int i1 = min(i0 + A.tx, nx);
    const int t = threadIdx.x;
    const int jt = j0 + t * W;
    const bool own_in = jt < nv;
    const int jld = own_in ? jt : 0;
    const int lane = t & 63, wave = t >> 6;
    const int c0 = LPAD + t * W;
    const bool last_cell = own_in && (jt + W == nv);   // owns the top velocity face nv - 1/2

    double gconst[W];   // f(s) values of own cells outside [0, nv)
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int j = jt + w;
        gconst[w] = (j == nv) ? A.vg[2] : (j == nv + 1) ? A.vg[3] : 0.0;
    }
    const bool has_halo = t < 4;
    const int hj = t < 2 ? j0 - 2 + t : j0 + TV + (t - 2);
    const int hcol = t < 2 ? LPAD - 2 + t : LPAD + TV + (t - 2);
    const bool halo_in = has_halo && hj >= 0 && hj < nv;
    const int hld = halo_in ? hj : jld;
    const double hconst = (hj == -2) ? A.vg[0] : (hj == -1) ? A.vg[1] : (hj == nv) ? A.vg[2]
                        : (hj == nv + 1) ? A.vg[3] : 0.0;

    const double* __restrict__ lam = A.lam;
    const double* __restrict__ gp = A.g_prev;
    const double* __restrict__ fs = A.fs;

    auto slot_of = [&](int r) { return (r - i0 + 2) & (NSLOT - 1); };
    struct RowIn { double lk[W], gk[W], f[W], lh, gh, fh; };
    auto load_rows = [&](int r, RowIn& R) {
        const size_t ro = (size_t)wrapa(r, nx) * nv;
        Vd<W>::ld(lam + ro + jld, R.lk);
        Vd<W>::ld(fs + ro + jld, R.f);
        R.lh = lam[ro + hld];
        R.fh = fs[ro + hld];
        if (!FIRST) {
            Vd<W>::ld(gp + ro + jld, R.gk);
            R.gh = gp[ro + hld];
        }
    };
    auto store_rows = [&](int r, const RowIn& R) {
        const int sl = slot_of(r);
        const double zr = FIRST ? 0.0 : zseg[r - i0 + 2];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const double kb = FIRST ? A.c1 * R.lk[w] : A.c1 * R.lk[w] + A.c2 * (R.gk[w] + zr);
            KB[sl][c0 + w] = own_in ? kb : 0.0;
            FS[sl][c0 + w] = own_in ? R.f[w] : gconst[w];
        }
        if (has_halo) {
            const double kb = FIRST ? A.c1 * R.lh : A.c1 * R.lh + A.c2 * (R.gh + zr);
            KB[sl][hcol] = halo_in ? kb : 0.0;
            FS[sl][hcol] = halo_in ? R.fh : hconst;
        }
    };

    double vb[W];
#pragma unroll
    for (int w = 0; w < W; ++w) vb[w] = A.v_lo + ((double)(jt + w) + 0.5) * A.dv;
    const double dxi = A.dxi, dvi = A.dvi, dv24 = A.dv24;

    // x-face cotangent Fbar_x(r + 1/2) at own cells from kbar rows r, r+1
    auto fbx_face = [&](int r, double* out) {
        const int s0 = slot_of(r), s1 = slot_of(r + 1);
        double gx[W + 2];
#pragma unroll
        for (int q = 0; q < W + 2; ++q) gx[q] = (KB[s1][c0 - 1 + q] - KB[s0][c0 - 1 + q]) * dxi;
#pragma unroll
        for (int w = 0; w < W; ++w) out[w] = vb[w] * gx[w + 1] + dv24 * (gx[w] - gx[w + 2]);
    };
    // Gbar_v(r, face) for faces m = 0..W+2, face m between cells jt-2+m and jt-1+m
    auto gv_row = [&](int r, double* out) {
        const int sl = slot_of(r);
#pragma unroll
        for (int m = 0; m <= W + 2; ++m) out[m] = (KB[sl][c0 - 1 + m] - KB[sl][c0 - 2 + m]) * dvi;
    };
    // forward v-face averages Fv(r, face) of f(s) for faces m = 1..W+1 (index m-1)
    auto fv_row = [&](int r, double* out) {
        const int sl = slot_of(r);
        double u[W + 4];
#pragma unroll
        for (int q = 0; q < W + 4; ++q) u[q] = FS[sl][c0 - 2 + q];
#pragma unroll
        for (int m = 1; m <= W + 1; ++m) out[m - 1] = face4a(u[m - 1], u[m], u[m + 1], u[m + 2]);
    };

    // ---- prologue
    for (int q = t; q < i1 - i0 + 4; q += NT) {
        aseg[q] = A.a[wrapa(i0 - 2 + q, nx)];
        zseg[q] = FIRST ? 0.0 : A.z_prev[wrapa(i0 - 2 + q, nx)];
    }
    for (int q = i1 - i0 + 4 + t; q < kMaxTx + RB + 4; q += NT) { aseg[q] = 0.0; zseg[q] = 0.0; }
    __syncthreads();
    {
        RowIn R[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) load_rows(i0 - 2 + q, R[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q) store_rows(i0 - 2 + q, R[q]);
    }
    __syncthreads();
    double fbx[4][W];      // faces i-3/2, i-1/2, i+1/2, i+3/2
    fbx_face(i0 - 2, fbx[0]);
    fbx_face(i0 - 1, fbx[1]);
    fbx_face(i0, fbx[2]);
    double gvm[W + 3], gv0[W + 3];   // rows i-1, i
    gv_row(i0 - 1, gvm);
    gv_row(i0, gv0);
    double fv[4][W + 1];   // Fv rows i-2 .. i+1
#pragma unroll
    for (int q = 0; q < 4; ++q) fv_row(i0 - 2 + q, fv[q]);

#pragma unroll 1
    for (int ib = i0; ib < i1; ib += RB) {
        RowIn R[RB];
        double mold[RB][W], gown[RB][W];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            load_rows(min(ib + 2 + q, i1 + 1), R[q]);
            if (!FIRST) {
                const size_t off = (size_t)min(ib + q, i1 - 1) * nv + jld;
                Vd<W>::ld((A.mu_in ? A.mu_in : lam) + off, mold[q]);
                Vd<W>::ld(gp + off, gown[q]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RB; ++q) store_rows(ib + 2 + q, R[q]);
        __syncthreads();

        double gout[RB][W], mout[RB][W];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int i = ib + q;
            const int qa = i - i0;
            const double am2 = aseg[qa], a0 = aseg[qa + 2], ap2 = aseg[qa + 4];
            fbx_face(i + 1, fbx[3]);
            double gvp[W + 3];
            gv_row(i + 1, gvp);
            double fvn[W + 1];
            fv_row(i + 2, fvn);

            double fbv[W + 3];
#pragma unroll
            for (int m = 0; m <= W + 2; ++m)
                fbv[m] = a0 * gv0[m] + (a0 - am2) * (1.0 / 48.0) * gvm[m] - (ap2 - a0) * (1.0 / 48.0) * gvp[m];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const double gx = (-fbx[3][w] + 7.0 * fbx[2][w] + 7.0 * fbx[1][w] - fbx[0][w]) * (1.0 / 12.0);
                const double gvv = (-fbv[w + 3] + 7.0 * fbv[w + 2] + 7.0 * fbv[w + 1] - fbv[w]) * (1.0 / 12.0);
                gout[q][w] = gx + gvv;
            }
            // acceleration cotangent over the own faces m = 1..W (+ the top face)
            double sa = 0.0;
#pragma unroll
            for (int m = 1; m <= W + 1; ++m) {
                if (m == W + 1 && !last_cell) continue;
                const double Fc = fv[2][m - 1], Fm2 = fv[0][m - 1], Fp2 = fvn[m - 1];
                sa += Fc * gv0[m] + (Fc - Fm2) * (1.0 / 48.0) * gvm[m] - (Fp2 - Fc) * (1.0 / 48.0) * gvp[m];
            }
            if (!own_in) sa = 0.0;
            sa = wave_sum_a(sa);
            if (lane == 0 && i < i1) mom[wave][qa] = sa;
            if (!FIRST) {
                const double zr = zseg[qa + 2];
#pragma unroll
                for (int w = 0; w < W; ++w) mout[q][w] = mold[q][w] + gown[q][w] + zr;
            }
            // roll the windows
#pragma unroll
            for (int w = 0; w < W; ++w) {
                fbx[0][w] = fbx[1][w]; fbx[1][w] = fbx[2][w]; fbx[2][w] = fbx[3][w];
            }
#pragma unroll
            for (int m = 0; m <= W + 2; ++m) { gvm[m] = gv0[m]; gv0[m] = gvp[m]; }
#pragma unroll
            for (int m = 0; m <= W; ++m) {
                fv[0][m] = fv[1][m]; fv[1][m] = fv[2][m]; fv[2][m] = fv[3][m]; fv[3][m] = fvn[m];
            }
        }
        if (own_in) {
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int i = ib + q;
                if (i < i1) {
                    const size_t off = (size_t)i * nv + jt;
                    Vd<W>::st(A.g_out + off, gout[q]);
                    if (!FIRST) Vd<W>::st(A.mu_out + off, mout[q]);
                }
            }
        }
    }
    __syncthreads();
    for (int q = t; q < i1 - i0; q += NT) {
        double sm = 0.0;
#pragma unroll
        for (int wv = 0; wv < NWAVE; ++wv) sm += mom[wv][q];
        A.part[(size_t)strip * nx + i0 + q] = sm;
    }
}

// lam_n = mu + g_1 + z_1 (row-broadcast z)
__global__ __launch_bounds__(256) void k_adjoint_final(const double* __restrict__ mu, const double* __restrict__ g,
                                                      const double* __restrict__ z, int nv, size_t total,
                                                      double* __restrict__ out)
{
    const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (p < total) out[p] = mu[p] + g[p] + z[p / nv];
}

template <int W, int NT>
hipError_t launch_adj_t(bool first, const Adjoint1DArgs& a, hipStream_t stream)
{
    const int nseg = (a.nx + a.tx - 1) / a.tx;
    const dim3 grid(a.nstrip * nseg), block(NT);
    if (first)
        hipLaunchKernelGGL((k_adjoint_stage1d<W, NT, true>), grid, block, 0, stream, a);
    else
        hipLaunchKernelGGL((k_adjoint_stage1d<W, NT, false>), grid, block, 0, stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint_stage1d(int w, bool first, const Adjoint1DArgs& a, hipStream_t stream)
{
    if (w == 2) return launch_adj_t<2, 128>(first, a, stream);
    return launch_adj_t<1, 128>(first, a, stream);
}

hipError_t launch_adjoint_final(const double* mu, const double* g, const double* z, int nx, int nv, double* out,
                                hipStream_t stream)
{
    const size_t total = (size_t)nx * nv;
    hipLaunchKernelGGL(k_adjoint_final, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, mu, g, z,
                       nv, total, out);
    return hipGetLastError();
}

}  // namespace vp
