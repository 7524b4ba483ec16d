// HIP kernels of the multi-level (L <= 4 levels, a ratio per level and
// direction) 1D+1V path.
//
// Every patch of every level, level 0 included, carries a ghost frame two
// cells deep that one launch per stage fills from the stage input: a cell
// that a patch of the same level holds is copied (the exchange of ghost
// cells on a level, x periodic), one outside the velocity box takes the
// level's equilibrium, and the others are the conservative fifth-order
// sub-cell interpolation of the parent level (x then v, section 3).  The
// stage launch then walks a tile table over all patches of all levels with
// the same x-march as the single-level tile, its halo read from the frame,
// plus chunks of coarse faces on coarse-fine interfaces whose fluxes are
// accumulated for the end-of-step correction.
#include <hip/hip_runtime.h>

#include "vp_internal.hpp"
#include "vp_stage_tile.hpp"

namespace vp {

namespace {

using namespace dev;

__device__ __forceinline__ double src_val(const double* __restrict__ f, const double* __restrict__ eqv, int src)
{
    return src >= 0 ? f[src] : eqv[-1 - src];
}

// one thread per frame cell: copy, equilibrium or parent interpolation
__global__ __launch_bounds__(256) void k_hier_fill(const double* __restrict__ f, const int2* __restrict__ desc,
                                                  const HInterp* __restrict__ rec, const double* __restrict__ wts,
                                                  const int* __restrict__ wofs, const double* __restrict__ eqv,
                                                  double* __restrict__ frame, int n)
{
    const int k = (int)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const int2 d = desc[k];
    double v;
    if (d.x >= 0) {
        v = f[d.x];
    } else if (d.x == -1) {
        v = eqv[d.y];
    } else {
        const HInterp& R = rec[d.y];
        const double* bx = wts + wofs[2 * R.lev] + R.s * 5;
        const double* bv = wts + wofs[2 * R.lev + 1] + R.t * 5;
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            double gx = 0.0;
#pragma unroll
            for (int a = 0; a < 5; ++a) gx += bx[a] * src_val(f, eqv, R.src[a * 5 + b]);
            acc += bv[b] * gx;
        }
        v = acc;
    }
    frame[k] = v;
}

__device__ __forceinline__ void flux_acc(double* p, double v, const HierArgs& A)
{
    if (A.first) *p = A.c_flux * v;
    else *p += A.c_flux * v;
}

// Stage tile on one patch of any level (FP64): the x-march of the
// single-level tile over a row segment of a velocity strip; rows and
// columns outside the patch come from its ghost frame.
template <int W, int NT, int KIND>
__device__ __forceinline__ void stage_tile_frame(const HierArgs& A, const AmrTile& tl)
{
    using T = double;
    constexpr int RB = 4;
    constexpr int NSLOT = 8;
    constexpr int TV = NT * W;
    constexpr int LPAD = 2;
    constexpr int RW = ((LPAD + TV + 2 + 3) / 4) * 4;
    __shared__ __attribute__((aligned(16))) T ring[NSLOT][RW];
    __shared__ double aseg[kMaxTx + RB + 2];
    __shared__ T hrow[4][RW];                 // frame rows -2, -1, nx, nx+1; column c <-> j = j0 - 2 + c
    __shared__ T hcol[kMaxTx + 4][4];         // rows i0-2 .. i1+1; columns -2, -1, nv, nv+1

    const HPatch P = A.patches[tl.p];
    const HLevel Lv = A.lv[P.lev];
    const int nx = P.nx, nv = P.nv;
    const int i0 = tl.a * A.tx;
    const int i1 = min(i0 + A.tx, nx);
    const int j0 = tl.b * TV;
    const T* __restrict__ fs = A.fs + P.off;
    const T* __restrict__ fn = A.fn ? A.fn + P.off : nullptr;
    T* __restrict__ acc = A.acc ? A.acc + P.off : nullptr;
    T* __restrict__ fout = A.fout + P.off;
    const double* __restrict__ fr = A.frame + P.frame;
    double* ff = A.ff_acc ? A.ff_acc + P.foff : nullptr;
    const bool do_flux = (KIND != kRhs) && ff != nullptr && A.c_flux != 0.0;

    const int t = threadIdx.x;
    const int jt = j0 + t * W;
    const bool own_in = jt < nv;
    const int jld = own_in ? jt : 0;
    const int c0 = LPAD + t * W;
    const bool has_halo = t < 4;
    const int hj = t < 2 ? j0 - 2 + t : j0 + TV + (t - 2);
    const int hcol_idx = t < 2 ? LPAD - 2 + t : LPAD + TV + (t - 2);
    const bool halo_data = has_halo && hj >= 0 && hj < nv;
    const int hld = halo_data ? hj : jld;

    // the frame cells this tile reads, into LDS
    {
        const int ncols = TV + 4;
        for (int q2 = 0; q2 < 2; ++q2) {
            if (q2 == 0 ? i0 != 0 : i1 != nx) continue;
            for (int k = t; k < 2 * ncols; k += NT) {
                const int q = k / ncols, c = k - q * ncols;
                const int j = j0 - 2 + c;
                hrow[2 * q2 + q][c] = (j >= -2 && j <= nv + 1) ? fr[(size_t)(2 * q2 + q) * (nv + 4) + (j + 2)] : T(0);
            }
        }
        const double* fc = fr + (size_t)4 * (nv + 4);
        for (int k = t; k < 4 * (i1 - i0 + 4); k += NT) {
            const int q = k & 3, rr = k >> 2;
            const int r = i0 - 2 + rr;
            if (r < 0 || r >= nx) continue;
            hcol[rr][q] = fc[(size_t)r * 4 + q];
        }
    }
    auto halo_val = [&](int r, int j) -> T {
        if (j < -2 || j > nv + 1) return T(0);
        if (r < 0) return hrow[r + 2][j - j0 + 2];
        if (r >= nx) return hrow[r - nx + 2][j - j0 + 2];
        return hcol[r - i0 + 2][j < 0 ? j + 2 : j - nv + 2];
    };

    auto slot_of = [&](int r) { return (r - i0 + 2) & (NSLOT - 1); };
    auto load_row = [&](int r, T* v, T& h) {
        const int rc = min(max(r, 0), nx - 1);
        const T* row = fs + (size_t)rc * nv;
        VecIO<T, W>::ld(row + jld, v);
        h = row[hld];
    };
    auto store_row = [&](int r, const T* v, T h) {
        T* dst = &ring[slot_of(r)][0];
        if (r > i1 + 1) {               // past the tile window (last batch): never read
#pragma unroll
            for (int w = 0; w < W; ++w) dst[c0 + w] = T(0);
            if (has_halo) dst[hcol_idx] = T(0);
            return;
        }
        const bool rowdata = r >= 0 && r < nx;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int j = jt + w;
            dst[c0 + w] = (rowdata && j < nv) ? v[w] : halo_val(r, j);
        }
        if (has_halo) dst[hcol_idx] = (rowdata && halo_data) ? h : halo_val(r, hj);
    };
    auto fx_cols = [&](int r, T* Fx) {
        const int sm1 = slot_of(r - 1), s0 = slot_of(r), s1 = slot_of(r + 1), s2 = slot_of(r + 2);
#pragma unroll
        for (int q = 0; q < W + 2; ++q) {
            const int c = c0 - 1 + q;
            Fx[q] = face4<T>(ring[sm1][c], ring[s0][c], ring[s1][c], ring[s2][c]);
        }
    };
    auto fv_faces = [&](int r, T* Fv) {
        const int sl = slot_of(r);
        T u[W + 4];
#pragma unroll
        for (int q = 0; q < W + 4; ++q) u[q] = ring[sl][c0 - 2 + q];
#pragma unroll
        for (int m = 0; m <= W; ++m) Fv[m] = face4<T>(u[m], u[m + 1], u[m + 2], u[m + 3]);
    };

    T vb[W];
#pragma unroll
    for (int w = 0; w < W; ++w) vb[w] = A.v_lo + ((double)(P.gv0 + jt + w) + 0.5) * Lv.dv;
    const T dxi = Lv.dxi, dvi = Lv.dvi, dv24 = Lv.dv24;
    const double dts = A.dt ? *A.dt : 0.0;
    const T cacc = A.dt ? dts * A.c_acc : A.c_acc, cnext = A.dt ? dts * A.c_next : A.c_next;
    const double* __restrict__ al = A.a + Lv.a_off;

    __syncthreads();                          // frame cells in LDS
    {
        T v[4][W], h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) load_row(i0 - 2 + q, v[q], h[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q) store_row(i0 - 2 + q, v[q], h[q]);
    }
    for (int q = t; q < i1 - i0 + 2; q += NT) aseg[q] = al[wrapi(P.gx0 + i0 - 1 + q, Lv.nx)];
    for (int q = i1 - i0 + 2 + t; q < kMaxTx + RB + 2; q += NT) aseg[q] = 0.0;
    __syncthreads();

    T gx_old[W];
    {
        T Fx[W + 2];
        fx_cols(i0 - 1, Fx);
#pragma unroll
        for (int w = 0; w < W; ++w) gx_old[w] = vb[w] * Fx[w + 1] + dv24 * (Fx[w + 2] - Fx[w]);
    }
    if (do_flux && i0 == 0 && own_in) {
#pragma unroll
        for (int w = 0; w < W; ++w) flux_acc(ff + jt + w, gx_old[w], A);       // x face -1/2
    }
    T fvA[W + 1], fvB[W + 1];
    fv_faces(i0 - 1, fvA);
    fv_faces(i0, fvB);

#pragma unroll 1
    for (int ib = i0; ib < i1; ib += RB) {
        T v[RB][W], h[RB], fnv[RB][W], accv[RB][W];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            load_row(min(ib + 2 + q, i1 + 1), v[q], h[q]);
            const size_t off = (size_t)min(ib + q, i1 - 1) * nv + jld;
            if (KIND == kStage23) VecIO<T, W>::ld(fn + off, fnv[q]);
            if (KIND == kStage23 || KIND == kStage4) VecIO<T, W>::ld(acc + off, accv[q]);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RB; ++q) store_row(ib + 2 + q, v[q], h[q]);
        __syncthreads();

        T o1[RB][W], o2[RB][W];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int i = ib + q;
            const int qa = i - i0;
            const T a_m1 = aseg[qa], a_0 = aseg[qa + 1], a_p1 = aseg[qa + 2];
            T Fx[W + 2];
            fx_cols(i, Fx);
            T fvC[W + 1];
            fv_faces(i + 1, fvC);
            const T da48 = (a_p1 - a_m1) * T(1.0 / 48.0);
            T gv[W + 1];
#pragma unroll
            for (int m = 0; m <= W; ++m) gv[m] = a_0 * fvB[m] + da48 * (fvC[m] - fvA[m]);
            T kk[W], gxn[W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                gxn[w] = vb[w] * Fx[w + 1] + dv24 * (Fx[w + 2] - Fx[w]);
                kk[w] = -(gxn[w] - gx_old[w]) * dxi - (gv[w + 1] - gv[w]) * dvi;
                gx_old[w] = gxn[w];
            }
            if (do_flux && i < i1 && own_in) {
                if (i == nx - 1) {
#pragma unroll
                    for (int w = 0; w < W; ++w) flux_acc(ff + nv + jt + w, gxn[w], A);   // x face nx-1/2
                }
                if (jt == 0) flux_acc(ff + 2 * nv + i, gv[0], A);                       // v face -1/2
                if (jt + W == nv) flux_acc(ff + 2 * nv + nx + i, gv[W], A);             // v face nv-1/2
            }
#pragma unroll
            for (int m = 0; m <= W; ++m) { fvA[m] = fvB[m]; fvB[m] = fvC[m]; }

            if (KIND == kRhs) {
#pragma unroll
                for (int w = 0; w < W; ++w) o1[q][w] = kk[w];
            } else if (KIND == kStage1) {
                const int sl = slot_of(i);
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const T f0 = ring[sl][c0 + w];
                    o1[q][w] = f0 + cacc * kk[w];
                    o2[q][w] = f0 + cnext * kk[w];
                }
            } else if (KIND == kStage23) {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    o1[q][w] = accv[q][w] + cacc * kk[w];
                    o2[q][w] = fnv[q][w] + cnext * kk[w];
                }
            } else {
#pragma unroll
                for (int w = 0; w < W; ++w) o2[q][w] = accv[q][w] + cacc * kk[w];
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
}

// coarse fluxes on a chunk of coarse-fine faces, accumulated with weight b_s;
// every stencil value is a state element or an equilibrium ghost value
template <int NT>
__device__ __forceinline__ void face_chunk(const HierArgs& A, const AmrTile& tl)
{
    for (int q = threadIdx.x; q < tl.a; q += NT) {
        const int fi = tl.p + q;
        const HFace F = A.faces[fi];
        const HLevel Lv = A.lv[F.lev];
        double fx[3];
#pragma unroll
        for (int m = 0; m < 3; ++m)
            fx[m] = face4<double>(src_val(A.fs, A.eqv, F.src[m * 4]), src_val(A.fs, A.eqv, F.src[m * 4 + 1]),
                                  src_val(A.fs, A.eqv, F.src[m * 4 + 2]), src_val(A.fs, A.eqv, F.src[m * 4 + 3]));
        double G;
        if (F.dir == 0) {
            G = F.vb * fx[1] + Lv.dv24 * (fx[2] - fx[0]);
        } else {
            const double ai = A.a[F.ai[1]];
            const double da48 = (A.a[F.ai[2]] - A.a[F.ai[0]]) * (1.0 / 48.0);
            G = ai * fx[1] + da48 * (fx[2] - fx[0]);
        }
        flux_acc(A.cf_acc + fi, G, A);
    }
}

template <int W, int NT, int KIND>
__global__ __launch_bounds__(NT) void k_hier_stage(HierArgs A, int t_begin, int t_end)
{
    for (int t = t_begin + (int)blockIdx.x; t < t_end; t += (int)gridDim.x) {
        const AmrTile tl = A.tiles[t];
        if (tl.kind == kTileFine) {
            stage_tile_frame<W, NT, KIND>(A, tl);
        } else if (KIND != kRhs && A.cf_acc != nullptr && A.c_flux != 0.0) {
            face_chunk<NT>(A, tl);
        }
        __syncthreads();
    }
}

// one wave per row segment of the state (off >= 0) or of the frames
// (off < 0: frame element -1 - off): slots[k] = sum of len[k] values
__global__ __launch_bounds__(256) void k_hier_rowsum(const double* __restrict__ f, const double* __restrict__ frame,
                                                    const long long* __restrict__ off, const int* __restrict__ len,
                                                    int ntasks, double* __restrict__ slots)
{
    const int task = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (task >= ntasks) return;          // uniform per wave
    const long long o = off[task];
    const double* p = o >= 0 ? f + o : frame + (-1 - o);
    const int n = len[task];
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += p[j];
    s = wave_sum(s);
    if (lane == 0) slots[task] = s;
}

// a of every level from the finest field: a_l[i] = (q/m) mean of the rt_l finest values
struct HierInjectLevels {
    int L;
    int a_off[kHierLevels], nx[kHierLevels], rt[kHierLevels];
};

__global__ __launch_bounds__(256) void k_hier_inject(const double* __restrict__ E, HierInjectLevels Z, double qm,
                                                    double* __restrict__ a, int na)
{
    const int k = (int)blockIdx.x * 256 + threadIdx.x;
    if (k >= na) return;
    int l = 0;
    while (l + 1 < Z.L && k >= Z.a_off[l + 1]) ++l;
    const int i = k - Z.a_off[l], rt = Z.rt[l];
    double s = 0.0;
    for (int q = 0; q < rt; ++q) s += E[i * rt + q];
    a[k] = qm * (s / rt);
}

// the end-of-step correction: each uncovered cell next to coarse-fine
// faces takes, on each of them, the mean of the fine accumulated fluxes in
// place of its own accumulated flux
__global__ __launch_bounds__(256) void k_hier_reflux(HierSyncArgs S)
{
    const int k = (int)blockIdx.x * 256 + threadIdx.x;
    if (k >= S.ncorr) return;
    double val = S.f[S.corr_cell[k]];
    for (int e = S.corr_ptr[k]; e < S.corr_ptr[k + 1]; ++e) {
        const int code = S.corr_face[e];
        const bool lower = code < 0;                 // the face is the cell's lower face
        const int fi = lower ? -code - 1 : code;
        const HFace F = S.faces[fi];
        const int nf = S.corr_nfine[fi];
        const double* fine = S.ff_acc + S.corr_fine[fi];
        double s = 0.0;
        for (int q = 0; q < nf; ++q) s += fine[q];
        const double diff = s / nf - S.cf_acc[fi];
        const double h = (S.dt_dev ? *S.dt_dev : S.dt) * (F.dir == 0 ? S.lv[F.lev].dxi : S.lv[F.lev].dvi);
        val += lower ? h * diff : -h * diff;
    }
    S.f[S.corr_cell[k]] = val;
}

// the adaptive run's time step on the device: the stability rate of every
// patch of every level, max(|v| at its velocity faces) / dx + |a| / dv over
// its configuration columns (a maximum, so its order does not matter; the
// products and sums rounded one by one, as the host rule computes them),
// then dt and t; one block
struct HierDtArgs {
    const double* a;
    const HPatch* patches;
    int npatch;
    HLevel lv[kHierLevels];
    double v_lo, courant, cfl, growth, dt_initial;
    int first;
    double* state;             // [dt, t]
};

__global__ __launch_bounds__(256) void k_hier_dt(HierDtArgs D)
{
    __shared__ double red[4];
    double rate = 0.0;
    for (int p = 0; p < D.npatch; ++p) {
        const HPatch P = D.patches[p];
        const HLevel& v = D.lv[P.lev];
        const double v0 = __dadd_rn(D.v_lo, __dmul_rn((double)P.gv0, v.dv));
        const double v1 = __dadd_rn(D.v_lo, __dmul_rn((double)(P.gv0 + P.nv), v.dv));
        const double vt = __dmul_rn(fmax(fabs(v0), fabs(v1)), v.dxi);
        const double* al = D.a + v.a_off + P.gx0;
        for (int i = threadIdx.x; i < P.nx; i += 256) rate = fmax(rate, __dadd_rn(vt, __dmul_rn(fabs(al[i]), v.dvi)));
    }
    for (int m = 32; m >= 1; m >>= 1) rate = fmax(rate, __shfl_xor(rate, m, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rate;
    __syncthreads();
    if (threadIdx.x == 0) {
        rate = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        const double lim = D.courant / rate;
        const double cap = D.first ? D.dt_initial : __dmul_rn(D.growth, D.state[0]);
        const double dt = fmin(cap, __dmul_rn(D.cfl, lim));
        D.state[0] = dt;
        D.state[1] = __dadd_rn(D.state[1], dt);
    }
}

__global__ __launch_bounds__(256) void k_hier_average(HierAvgArgs S)
{
    const int k = (int)blockIdx.x * 256 + threadIdx.x;
    if (k >= S.n) return;
    const double* base = S.f + S.src[k];
    const int stride = S.stride[k];
    double s = 0.0;
    for (int a = 0; a < S.rx; ++a)
        for (int b = 0; b < S.rv; ++b) s += base[(size_t)a * stride + b];
    S.f[S.dst[k]] = s / (S.rx * S.rv);
}

template <int W, int NT>
hipError_t launch_hier_t(int kind, const HierArgs& a, int t0, int t1, int grid, hipStream_t stream)
{
    const dim3 g(grid), b(NT);
    switch (kind) {
    case kRhs: hipLaunchKernelGGL((k_hier_stage<W, NT, kRhs>), g, b, 0, stream, a, t0, t1); break;
    case kStage1: hipLaunchKernelGGL((k_hier_stage<W, NT, kStage1>), g, b, 0, stream, a, t0, t1); break;
    case kStage23: hipLaunchKernelGGL((k_hier_stage<W, NT, kStage23>), g, b, 0, stream, a, t0, t1); break;
    default: hipLaunchKernelGGL((k_hier_stage<W, NT, kStage4>), g, b, 0, stream, a, t0, t1); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_hier_fill(const double* f, const int2* desc, const HInterp* rec, const double* wts,
                            const int* wofs, const double* eqv, double* frame, int n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hier_fill, dim3((n + 255) / 256), dim3(256), 0, stream, f, desc, rec, wts, wofs, eqv, frame,
                       n);
    return hipGetLastError();
}

hipError_t launch_hier_stage(int w, int nt, int kind, const HierArgs& a, int t_begin, int t_end, int grid,
                             hipStream_t stream)
{
    if (t_end <= t_begin) return hipSuccess;
    if (w == 2 && nt == 64) return launch_hier_t<2, 64>(kind, a, t_begin, t_end, grid, stream);
    if (w == 2 && nt == 128) return launch_hier_t<2, 128>(kind, a, t_begin, t_end, grid, stream);
    if (w == 1 && nt == 64) return launch_hier_t<1, 64>(kind, a, t_begin, t_end, grid, stream);
    if (w == 1 && nt == 128) return launch_hier_t<1, 128>(kind, a, t_begin, t_end, grid, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_hier_rowsum(const double* f, const double* frame, const long long* task_off, const int* task_len,
                              int ntasks, double* slots, hipStream_t stream)
{
    if (ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hier_rowsum, dim3((ntasks + 3) / 4), dim3(256), 0, stream, f, frame, task_off, task_len,
                       ntasks, slots);
    return hipGetLastError();
}

hipError_t launch_hier_inject(const double* E, const HLevel* lv, int L, double qm, double* a, int na,
                              hipStream_t stream)
{
    if (na <= 0) return hipSuccess;
    HierInjectLevels Z{};
    Z.L = L;
    for (int l = 0; l < L; ++l) {
        Z.a_off[l] = lv[l].a_off;
        Z.nx[l] = lv[l].nx;
        Z.rt[l] = lv[l].rt;
    }
    hipLaunchKernelGGL(k_hier_inject, dim3((na + 255) / 256), dim3(256), 0, stream, E, Z, qm, a, na);
    return hipGetLastError();
}

hipError_t launch_hier_dt(const double* a, const HPatch* patches, int npatch, const HLevel* lv, int L, double v_lo,
                          double courant, double cfl, double growth, double dt_initial, int first, double* state,
                          hipStream_t stream)
{
    HierDtArgs D{};
    D.a = a;
    D.patches = patches;
    D.npatch = npatch;
    for (int l = 0; l < L; ++l) D.lv[l] = lv[l];
    D.v_lo = v_lo;
    D.courant = courant;
    D.cfl = cfl;
    D.growth = growth;
    D.dt_initial = dt_initial;
    D.first = first;
    D.state = state;
    hipLaunchKernelGGL(k_hier_dt, dim3(1), dim3(256), 0, stream, D);
    return hipGetLastError();
}

hipError_t launch_hier_reflux(const HierSyncArgs& s, hipStream_t stream)
{
    if (s.ncorr <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hier_reflux, dim3((s.ncorr + 255) / 256), dim3(256), 0, stream, s);
    return hipGetLastError();
}

hipError_t launch_hier_average(const HierAvgArgs& s, hipStream_t stream)
{
    if (s.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hier_average, dim3((s.n + 255) / 256), dim3(256), 0, stream, s);
    return hipGetLastError();
}

}  // namespace vp
