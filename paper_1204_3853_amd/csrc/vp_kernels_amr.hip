// HIP kernels of the two-level (coarse level + level-1 patches) 1D+1V path.
//
// One persistent launch per RK4 stage walks a tile table that holds every
// tile of every patch on both levels: coarse tiles (the single-level stage
// tile on the coarse mesh), fine tiles (the same x-march over a strip of a
// level-1 patch, whose halo cells are filled on the fly by the conservative
// fifth-order sub-cell interpolation of the coarse predictor of the same
// stage, section 3) and chunks of coarse faces on coarse-fine interfaces,
// whose coarse fluxes are accumulated for the end-of-step synchronisation.
// Fine tiles also accumulate the fluxes on their patch boundary.  All
// inputs of a stage were produced by earlier launches, so tiles are
// independent and need no ordering inside the launch.
#include <hip/hip_runtime.h>

#include "vp_internal.hpp"
#include "vp_stage_tile.hpp"

namespace vp {

namespace {

using namespace dev;

// Ghost values are selected as values after an unconditional (clamped) load;
// selecting between a struct member and an array element would make the
// compiler take the argument struct's address and copy it to scratch.
__device__ __forceinline__ double pick_ghost(int j, int n, double g0, double g1, double g2, double g3)
{
    return j == -2 ? g0 : (j == -1 ? g1 : (j == n ? g2 : g3));
}

// coarse value with x periodic and the coarse velocity ghosts
__device__ __forceinline__ double coarse_at(const Stage1DArgs& C, const double* fc, int i, int j, double g0,
                                            double g1, double g2, double g3)
{
    const int jc = min(max(j, 0), C.nv - 1);
    const double x = fc[(size_t)wrapi(i, C.nx) * C.nv + jc];
    return (j >= 0 && j < C.nv) ? x : pick_ghost(j, C.nv, g0, g1, g2, g3);
}

__device__ __forceinline__ void flux_acc(double* p, double v, const AmrArgs& A)
{
    if (A.first) *p = A.c_flux * v;
    else *p += A.c_flux * v;
}

// Stage tile on a level-1 patch (FP64): same march and arithmetic as the
// single-level tile; the halo cells are interpolated from the coarse level
// (x then v, the sub-cell weights b_j(s) of section 3).
template <int W, int NT, int KIND, bool LIM>
__device__ __forceinline__ void stage_tile_fine(const AmrArgs& A, const AmrTile& tl)
{
    using T = double;
    constexpr int RB = 4;
    constexpr int NSLOT = 8;
    constexpr int TV = NT * W;
    constexpr int LPAD = 2;
    constexpr int RW = ((LPAD + TV + 2 + 3) / 4) * 4;
    __shared__ __attribute__((aligned(16))) T ring[NSLOT][RW];
    __shared__ double aseg[kMaxTx + RB + 2];

    const AmrPatch P = A.patches[tl.p];
    const int nx = P.nx, nv = P.nv;
    const int i0 = tl.a * A.tx;
    const int i1 = min(i0 + A.tx, nx);
    const int j0 = tl.b * TV;
    const T* __restrict__ fs = static_cast<const T*>(A.coarse.fs) + P.off;
    const T* __restrict__ fn = static_cast<const T*>(A.coarse.fn) + P.off;
    T* __restrict__ acc = static_cast<T*>(A.coarse.acc) + P.off;
    T* __restrict__ fout = static_cast<T*>(A.coarse.fout) + P.off;
    double* ff = A.ff_acc ? A.ff_acc + P.foff : nullptr;
    const bool do_flux = (KIND != kRhs) && ff != nullptr && A.c_flux != 0.0;

    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int jt = j0 + t * W;
    const bool own_in = jt < nv;
    const int jld = own_in ? jt : 0;
    const int c0 = LPAD + t * W;
    // velocity sums of the tile's new rows, per wave (Alg. mreduce's fine row sums)
    __shared__ double momf[NT / 64][kMaxTx];
    const bool do_mom = KIND != kRhs && A.fpart != nullptr;
    const bool has_halo = t < 4;
    const int hj = t < 2 ? j0 - 2 + t : j0 + TV + (t - 2);
    const int hcol_idx = t < 2 ? LPAD - 2 + t : LPAD + TV + (t - 2);
    const bool halo_data = has_halo && hj >= 0 && hj < nv;
    const int hld = halo_data ? hj : jld;

    auto load_row = [&](int r, T* v, T& h) {
        const int rc = min(max(r, 0), nx - 1);
        const T* row = fs + (size_t)rc * nv;
        VecIO<T, W>::ld(row + jld, v);
        h = row[hld];
    };
    // the first rows of the march and the tile's accelerations, loaded
    // before the halo work so that their latency overlaps it
    T v0[4][W], h0[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) load_row(i0 - 2 + q, v0[q], h0[q]);
    for (int q = t; q < i1 - i0 + 2; q += NT) aseg[q] = A.a_f[wrapi(P.gx0 + i0 - 1 + q, A.nfx)];
    for (int q = i1 - i0 + 2 + t; q < kMaxTx + RB + 2; q += NT) aseg[q] = 0.0;

    // Coarse-fine halo of the tile, interpolated once into LDS before the
    // march: patch rows -2, -1 (first segment) and nx, nx+1 (last segment)
    // over the tile's columns, and columns -2, -1, nv, nv+1 of its rows.
    // For each of these (up to four) regions the coarse cells its stencils
    // touch are first copied into an LDS window (one batch of loads, held
    // in the ring's storage, which the march has not started using), and
    // the interpolation then reads only LDS.
    __shared__ T hrow[4][RW];                 // rows -2, -1, nx, nx+1; column c <-> j = j0 - 2 + c
    __shared__ T hcol[kMaxTx + 4][4];         // rows i0-2 .. i1+1; columns -2, -1, nv, nv+1
    __shared__ double bs[16 * 5];             // b_j(s), s < R
    {
        const Stage1DArgs& C = A.coarse;
        const double* fc = static_cast<const double*>(C.fs);
        const double cg0 = C.vg[0], cg1 = C.vg[1], cg2 = C.vg[2], cg3 = C.vg[3];
        const double fg0 = A.vgf[0], fg1 = A.vgf[1], fg2 = A.vgf[2], fg3 = A.vgf[3];
        const int R = A.R, lr = A.lr;
        for (int k = t; k < R * 5; k += NT) bs[k] = A.B[k];
        double* win = &ring[0][0];
        constexpr int kWinCap = NSLOT * RW;
        const bool top = i0 == 0, bot = i1 == nx;
        const bool left = j0 == 0, right = j0 + TV + 1 >= nv;
        // fine cell (X, V) from the window with origin (wi0, wj0) and row length ww
        auto interp_win = [&](int X, int V, int wi0, int wj0, int ww) -> T {
            if (V < 0 || V >= A.nfv) return pick_ghost(V, A.nfv, fg0, fg1, fg2, fg3);
            const int ci = X >> lr, sx = X & (R - 1);
            const int cj = V >> lr, sv = V & (R - 1);
            const double* w0 = win + (ci - 2 - wi0) * ww + (cj - 2 - wj0);
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < 5; ++b) {
                double gx = 0.0;
#pragma unroll
                for (int a = 0; a < 5; ++a) gx += bs[sx * 5 + a] * w0[a * ww + b];
                acc += bs[sv * 5 + b] * gx;
            }
            return acc;
        };
        // copy coarse rows wi0 .. wi0+wh-1, columns wj0 .. wj0+ww-1 into the window
        auto fill = [&](int wi0, int wj0, int wh, int ww) {
            const int cnt = min(wh * ww, kWinCap);
            for (int k = t; k < cnt; k += NT) {
                const int r = k / ww, c = k - (k / ww) * ww;
                win[k] = coarse_at(C, fc, wi0 + r, wj0 + c, cg0, cg1, cg2, cg3);
            }
        };
        const int vlo = P.gv0 + j0 - 2, vhi = P.gv0 + j0 + TV + 1;
        const int cjlo = max(min(vlo, A.nfv - 1), 0) >> lr, cjhi = max(min(vhi, A.nfv - 1), 0) >> lr;
        __syncthreads();                      // bs visible; the ring is free
        for (int q2 = 0; q2 < 2; ++q2) {      // top rows, then bottom rows
            if (q2 == 0 ? !top : !bot) continue;
            const int X0 = P.gx0 + (q2 == 0 ? -2 : nx);
            const int wi0 = (X0 >> lr) - 2, wj0 = cjlo - 2, ww = cjhi - cjlo + 5;
            const int wh = 5 + ((X0 + 1) >> lr) - (X0 >> lr);
            fill(wi0, wj0, wh, ww);
            __syncthreads();
            // the same sums as interp_win, split: the x sums of every window
            // column for the two rows first (after the window in the ring's
            // storage: (wh + 2) ww <= 8 ww fits), then the v sums per cell
            double* gxr = win + wh * ww;
            for (int k = t; k < 2 * ww; k += NT) {
                const int q = k / ww, cc = k - q * ww;
                const int X = X0 + q, ci = X >> lr, sx = X & (R - 1);
                const double* w0 = win + (ci - 2 - wi0) * ww + cc;
                double gx = 0.0;
#pragma unroll
                for (int a = 0; a < 5; ++a) gx += bs[sx * 5 + a] * w0[a * ww];
                gxr[k] = gx;
            }
            __syncthreads();
            const int ncols = TV + 4;
            for (int k = t; k < 2 * ncols; k += NT) {
                const int q = k / ncols, c = k - q * ncols;
                const int j = j0 - 2 + c;
                const int V = P.gv0 + j;
                T val = T(0);
                if (j >= -2 && j <= nv + 1) {
                    if (V < 0 || V >= A.nfv) {
                        val = pick_ghost(V, A.nfv, fg0, fg1, fg2, fg3);
                    } else {
                        const int cj = V >> lr, sv = V & (R - 1);
                        const double* g0 = gxr + q * ww + (cj - 2 - wj0);
                        double acc = 0.0;
#pragma unroll
                        for (int b = 0; b < 5; ++b) acc += bs[sv * 5 + b] * g0[b];
                        val = acc;
                    }
                }
                hrow[2 * q2 + q][c] = val;
            }
            __syncthreads();
        }
        for (int q2 = 0; q2 < 2; ++q2) {      // left columns, then right columns
            if (q2 == 0 ? !left : !right) continue;
            const int rlo = max(i0 - 2, 0), rhi = min(i1 + 1, nx - 1);
            const int V0 = P.gv0 + (q2 == 0 ? -2 : nv);
            const int cv0 = max(min(V0, A.nfv - 1), 0) >> lr, cv1 = max(min(V0 + 1, A.nfv - 1), 0) >> lr;
            const int wi0 = ((P.gx0 + rlo) >> lr) - 2, wj0 = cv0 - 2, ww = cv1 - cv0 + 5;
            fill(wi0, wj0, ((P.gx0 + rhi) >> lr) - ((P.gx0 + rlo) >> lr) + 5, ww);
            __syncthreads();
            for (int k = t; k < 2 * (i1 - i0 + 4); k += NT) {
                const int q = k & 1, rr = k >> 1;
                const int r = i0 - 2 + rr;
                if (r < 0 || r >= nx) continue;
                const int j = q2 == 0 ? q - 2 : nv + q;
                hcol[rr][2 * q2 + q] = interp_win(P.gx0 + r, P.gv0 + j, wi0, wj0, ww);
            }
            __syncthreads();
        }
        // Halo cells that a level-1 patch holds (a touching patch, also
        // across the periodic x boundary) take its value of the same stage
        // input instead (the exchange of ghost cells on a level); the same
        // regions as above, each cell written by the thread that wrote it.
        if (P.nb1 > P.nb0) {
            const double* fall = static_cast<const double*>(C.fs);
            // the neighbours' records, staged in LDS (the first kNbLds of them)
            constexpr int kNbLds = 8;
            __shared__ AmrPatch nbs[kNbLds];
            const int nnb = P.nb1 - P.nb0;
            for (int e = t; e < min(nnb, kNbLds); e += NT) nbs[e] = A.patches[A.nb[P.nb0 + e]];
            __syncthreads();
            auto held = [&](int X, int V, T& out) -> bool {
                if (V < 0 || V >= A.nfv) return false;
                const int Xw = wrapi(X, A.nfx);
                for (int e = 0; e < nnb; ++e) {
                    const AmrPatch Q = e < kNbLds ? nbs[e] : A.patches[A.nb[P.nb0 + e]];
                    const int dx = Xw - Q.gx0, dv = V - Q.gv0;
                    if (dx >= 0 && dx < Q.nx && dv >= 0 && dv < Q.nv) {
                        out = fall[Q.off + (size_t)dx * Q.nv + dv];
                        return true;
                    }
                }
                return false;
            };
            for (int q2 = 0; q2 < 2; ++q2) {
                if (q2 == 0 ? !top : !bot) continue;
                const int X0 = P.gx0 + (q2 == 0 ? -2 : nx);
                const int ncols = TV + 4;
                for (int k = t; k < 2 * ncols; k += NT) {
                    const int q = k / ncols, c = k - q * ncols;
                    const int j = j0 - 2 + c;
                    T v;
                    if (j >= -2 && j <= nv + 1 && held(X0 + q, P.gv0 + j, v)) hrow[2 * q2 + q][c] = v;
                }
            }
            for (int q2 = 0; q2 < 2; ++q2) {
                if (q2 == 0 ? !left : !right) continue;
                for (int k = t; k < 2 * (i1 - i0 + 4); k += NT) {
                    const int q = k & 1, rr = k >> 1;
                    const int r = i0 - 2 + rr;
                    if (r < 0 || r >= nx) continue;
                    const int j = q2 == 0 ? q - 2 : nv + q;
                    T v;
                    if (held(P.gx0 + r, P.gv0 + j, v)) hcol[rr][2 * q2 + q] = v;
                }
            }
            __syncthreads();
        }
    }
    // value of a cell of the tile window that is not patch data
    auto halo_val = [&](int r, int j) -> T {
        if (j < -2 || j > nv + 1) return T(0);
        if (r < 0) return hrow[r + 2][j - j0 + 2];
        if (r >= nx) return hrow[r - nx + 2][j - j0 + 2];
        return hcol[r - i0 + 2][j < 0 ? j + 2 : j - nv + 2];
    };

    auto slot_of = [&](int r) { return (r - i0 + 2) & (NSLOT - 1); };
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
    // limited faces (section 2, eq. limitedFace): an x face upwinded by the
    // sign of its column's centre velocity (global column, rounded after the
    // product and after the sum), a v face by the sign of a in its row
    bool upx[W + 2];
#pragma unroll
    for (int q = 0; q < W + 2; ++q)
        upx[q] = LIM && centre_unfused(A.v_lo, (double)(P.gv0 + jt - 1 + q) + 0.5, A.dvf) > 0.0;
    auto fx_cols = [&](int r, T* Fx) {
        const int sm1 = slot_of(r - 1), s0 = slot_of(r), s1 = slot_of(r + 1), s2 = slot_of(r + 2);
#pragma unroll
        for (int q = 0; q < W + 2; ++q) {
            const int c = c0 - 1 + q;
            if (LIM) Fx[q] = face_lim<T>(ring[sm1][c], ring[s0][c], ring[s1][c], ring[s2][c], upx[q]);
            else Fx[q] = face4<T>(ring[sm1][c], ring[s0][c], ring[s1][c], ring[s2][c]);
        }
    };
    auto fv_faces = [&](int r, T* Fv) {
        const int sl = slot_of(r);
        T u[W + 4];
#pragma unroll
        for (int q = 0; q < W + 4; ++q) u[q] = ring[sl][c0 - 2 + q];
        const bool upv = LIM && aseg[r - i0 + 1] > 0.0;
#pragma unroll
        for (int m = 0; m <= W; ++m) {
            if (LIM) Fv[m] = face_lim<T>(u[m], u[m + 1], u[m + 2], u[m + 3], upv);
            else Fv[m] = face4<T>(u[m], u[m + 1], u[m + 2], u[m + 3]);
        }
    };

    T vb[W];
#pragma unroll
    for (int w = 0; w < W; ++w) vb[w] = A.v_lo + ((double)(P.gv0 + jt + w) + 0.5) * A.dvf;
    const T dxi = A.dxfi, dvi = A.dvfi, dv24 = A.dvf24;
    const T cacc = A.coarse.c_acc, cnext = A.coarse.c_next;

#pragma unroll
    for (int q = 0; q < 4; ++q) store_row(i0 - 2 + q, v0[q], h0[q]);
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
        if (do_mom) {
            double sm4[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                sm4[q] = 0.0;
                if (own_in) {
#pragma unroll
                    for (int w = 0; w < W; ++w) sm4[q] += o2[q][w];
                }
            }
            const double tot = wave_sum4(sm4, lane);      // row q = lane / 16 of the batch
            const int g = lane >> 4;
            if ((lane & 15) == 0 && ib + g < i1) momf[wave][ib + g - i0] = tot;
        }
    }
    if (do_mom) {
        __syncthreads();
        double* dst = A.fpart + P.fpart + (size_t)tl.b * nx;
        for (int q = t; q < i1 - i0; q += NT) {
            double sm = 0.0;
#pragma unroll
            for (int wv = 0; wv < NT / 64; ++wv) sm += momf[wv][q];
            dst[i0 + q] = sm;
        }
    }
}

// coarse fluxes on a chunk of coarse-fine faces, accumulated with weight b_s
template <int NT, bool LIM>
__device__ __forceinline__ void face_chunk(const AmrArgs& A, const AmrTile& tl)
{
    const Stage1DArgs& C = A.coarse;
    const double* fc = static_cast<const double*>(C.fs);
    const double g0 = C.vg[0], g1 = C.vg[1], g2 = C.vg[2], g3 = C.vg[3];
    auto at = [&](int i, int j) { return coarse_at(C, fc, i, j, g0, g1, g2, g3); };
    for (int q = threadIdx.x; q < tl.a; q += NT) {
        const int fi = tl.p + q;
        const AmrFace F = A.faces[fi];
        double G;
        if (F.dir == 0) {          // x face between (i, j) and (i + 1, j)
            double fx[3];
#pragma unroll
            for (int m = -1; m <= 1; ++m) {
                const int c = F.j + m;
                if (LIM)
                    fx[m + 1] = face_lim<double>(at(F.i - 1, c), at(F.i, c), at(F.i + 1, c), at(F.i + 2, c),
                                                 centre_unfused(C.v_lo, (double)c + 0.5, C.dv) > 0.0);
                else
                    fx[m + 1] = face4<double>(at(F.i - 1, c), at(F.i, c), at(F.i + 1, c), at(F.i + 2, c));
            }
            const double vb = C.v_lo + ((double)F.j + 0.5) * C.dv;
            G = vb * fx[1] + C.dv24 * (fx[2] - fx[0]);
        } else {                   // v face between (i, j) and (i, j + 1)
            double fv[3];
#pragma unroll
            for (int m = -1; m <= 1; ++m) {
                const int r = F.i + m;
                if (LIM)
                    fv[m + 1] = face_lim<double>(at(r, F.j - 1), at(r, F.j), at(r, F.j + 1), at(r, F.j + 2),
                                                 C.a[wrapi(r, C.nx)] > 0.0);
                else
                    fv[m + 1] = face4<double>(at(r, F.j - 1), at(r, F.j), at(r, F.j + 1), at(r, F.j + 2));
            }
            const double ai = C.a[wrapi(F.i, C.nx)];
            const double da48 = (C.a[wrapi(F.i + 1, C.nx)] - C.a[wrapi(F.i - 1, C.nx)]) * (1.0 / 48.0);
            G = ai * fv[1] + da48 * (fv[2] - fv[0]);
        }
        flux_acc(A.cf_acc + fi, G, A);
    }
}

template <int W, int NT, int KIND, bool LIM>
__global__ __launch_bounds__(NT) void k_amr_stage(AmrArgs A, int t_begin, int t_end)
{
    for (int t = t_begin + (int)blockIdx.x; t < t_end; t += (int)gridDim.x) {
        const AmrTile tl = A.tiles[t];
        if (tl.kind == kTileCoarse) {
            stage_tile_uniform<double, W, NT, KIND, LIM>(A.coarse, tl.a);
        } else if (tl.kind == kTileFine) {
            stage_tile_fine<W, NT, KIND, LIM>(A, tl);
        } else if (KIND != kRhs && A.cf_acc != nullptr && A.c_flux != 0.0) {
            face_chunk<NT, LIM>(A, tl);
        }
        __syncthreads();
    }
}

// one wave per row segment: slots[k] = sum of len[k] consecutive values at off[k]
__global__ __launch_bounds__(256) void k_amr_rowsum(const double* __restrict__ f, const long long* __restrict__ off,
                                                   const int* __restrict__ len, int ntasks,
                                                   double* __restrict__ slots)
{
    const int task = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (task >= ntasks) return;          // uniform per wave
    const double* p = f + off[task];
    const int n = len[task];
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s += p[j];
    s = wave_sum(s);
    if (lane == 0) slots[task] = s;
}

// Mask reduction rows (Alg. mreduce): the coarse level is refined in x
// before it is masked, so the sum for target column i of the x-stencil
// offset a runs over row i + a with the coverage mask of column i.  One
// wave per (i, a).
__global__ __launch_bounds__(256) void k_amr_mask_rows(const double* __restrict__ f,
                                                      const unsigned char* __restrict__ covered, int ncx, int ncv,
                                                      double* __restrict__ S)
{
    const int task = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (task >= 5 * ncx) return;         // uniform per wave
    const int i = task / 5, a = task - (task / 5) * 5 - 2;
    const double* row = f + (size_t)wrapi(i + a, ncx) * ncv;
    const unsigned char* m = covered + (size_t)i * ncv;
    double s = 0.0;
    for (int j = lane; j < ncv; j += 64) s += m[j] ? 0.0 : row[j];
    s = wave_sum(s);
    if (lane == 0) S[task] = s;
}

// n_I = sum_k w_k slots[idx_k] over the list of cell I; 16 lanes per cell
// take every 16th entry and combine in a fixed butterfly order
__global__ __launch_bounds__(256) void k_amr_reduce_finalize(const double* __restrict__ slots,
                                                            const int* __restrict__ rowptr,
                                                            const int* __restrict__ idx,
                                                            const double* __restrict__ w, int nfx,
                                                            double* __restrict__ n)
{
    const int I = (int)blockIdx.x * 16 + (int)(threadIdx.x >> 4);
    const int l = threadIdx.x & 15;
    const int Ic = min(I, nfx - 1);                     // lanes of a cell past the end compute and drop
    const int k0 = rowptr[Ic], k1 = rowptr[Ic + 1];
    double s = 0.0;
    for (int k = k0 + l; k < k1; k += 16) s += w[k] * slots[idx[k]];
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) s += __shfl_xor(s, m, 16);
    if (l == 0 && I < nfx) n[I] = s;
}

// Mask reduction (Alg. mreduce) from the stage kernel's row sums.  For the
// target coarse column i and x-stencil offset a, the masked sum over row
// i + a is that row's total (its strip partials) less its cells in the
// velocity intervals level 1 covers in column i (read back from the state:
// a few cells per column); the R fine cells of column i take the
// x-refinement of the five masked sums, times dv_c, plus dv_f times the row
// sums of the patches over them (their strip partials, listed per column).
// One wave per coarse column.  The loads form three rounds (list bounds and
// the coarse partials; list entries; the values they name), each issued
// for all three sums at once, one element per lane; each lane keeps its
// terms per target and each target's total is a wave sum (a fixed butterfly
// order, so the result does not depend on timing).
__global__ __launch_bounds__(256) void k_amr_mask_fused(AmrMaskFusedArgs M)
{
    const int wv = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int i = min(wv, M.ncx - 1);      // waves past the end recompute the last column, store nothing
    const int lane = threadIdx.x & 63;
    int row[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) row[a] = wrapi(i + a - 2, M.ncx);
    const int nc = 5 * M.nstrip;
    const int k0 = M.cov_ptr[i], k1 = M.cov_ptr[i + 1];
    const int e0 = M.fz_ptr[i], e1 = M.fz_ptr[i + 1];
    double T[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // row totals (this lane's strips)
    double c[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // covered cells of column i (this lane's)
    double F[4] = {0.0, 0.0, 0.0, 0.0};        // fine row sums (R is 2 or 4)
    for (int l0 = 0; l0 < max(nc, max(k1 - k0, e1 - e0)); l0 += 64) {
        const int l = l0 + lane;
        // coarse partial l: strip l % nstrip of row l / nstrip
        const int ac = l < nc ? l / M.nstrip : 5;
        const double vc = l < nc ? M.part_c[(size_t)(l - ac * M.nstrip) * M.ncx + row[min(ac, 4)]] : 0.0;
        const int j = k0 + l < k1 ? M.cov_j[k0 + l] : -1;
        const int2 en = e0 + l < e1 ? M.fz_entry[e0 + l] : make_int2(0, -1);
        double cf[5];
#pragma unroll
        for (int a = 0; a < 5; ++a) cf[a] = j >= 0 ? M.f[(size_t)row[a] * M.ncv + j] : 0.0;
        const double vf = en.y >= 0 ? M.part_f[en.x] : 0.0;
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            T[a] += ac == a ? vc : 0.0;
            c[a] += cf[a];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) F[s] += en.y == s ? vf : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        T[a] = wave_sum(T[a]);
        c[a] = wave_sum(c[a]);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if (s < M.R) F[s] = wave_sum(F[s]);
    if (lane >= M.R || wv >= M.ncx) return;
    double n = 0.0;
#pragma unroll
    for (int a = 0; a < 5; ++a) n += M.B[lane * 5 + a] * M.dvc * (T[a] - c[a]);
    double fl = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if (s == lane) fl = F[s];
    M.n[i * M.R + lane] = n + M.dvf * fl;
}

// a_c = (q/m) mean of the R fine E values over each coarse cell, a_f = (q/m) E
__global__ __launch_bounds__(256) void k_amr_inject(const double* __restrict__ E, int ncx, int R, double qm,
                                                   double* __restrict__ a)
{
    const int k = (int)blockIdx.x * 256 + threadIdx.x;
    const int nfx = ncx * R;
    if (k < ncx) {
        double s = 0.0;
        for (int q = 0; q < R; ++q) s += E[k * R + q];
        a[k] = qm * (s / R);
    } else if (k < ncx + nfx) {
        a[k] = qm * E[k - ncx];
    }
}

__global__ __launch_bounds__(256) void k_amr_sync(AmrSyncArgs S)
{
    const int k = (int)blockIdx.x * 256 + threadIdx.x;
    if (k < S.ncorr) {
        const int cell = S.corr_cell[k];
        double val = S.f[cell];
        for (int e = S.corr_ptr[k]; e < S.corr_ptr[k + 1]; ++e) {
            const int code = S.corr_face[e];
            const bool high = code < 0;              // the face is the cell's lower face
            const int fi = high ? -code - 1 : code;
            const AmrFace F = S.faces[fi];
            double fine = 0.0;
            for (int q = 0; q < S.R; ++q) fine += S.ff_acc[F.fine + q];
            const double diff = fine / S.R - S.cf_acc[fi];
            const double h = F.dir == 0 ? S.dtx : S.dtv;
            val += high ? h * diff : -h * diff;
        }
        S.f[cell] = val;
    } else if (k < S.ncorr + S.ncov) {
        const int c = k - S.ncorr;
        const double* base = S.f + S.cov_fine[c];
        const int nvp = S.cov_nv[c];
        double s = 0.0;
        for (int a = 0; a < S.R; ++a)
            for (int b = 0; b < S.R; ++b) s += base[(size_t)a * nvp + b];
        S.f[S.cov_cell[c]] = s / (S.R * S.R);
    }
}

template <int W, int NT, bool LIM>
hipError_t launch_amr_l(int kind, const AmrArgs& a, int t0, int t1, int grid, hipStream_t stream)
{
    const dim3 g(grid), b(NT);
    switch (kind) {
    case kRhs: hipLaunchKernelGGL((k_amr_stage<W, NT, kRhs, LIM>), g, b, 0, stream, a, t0, t1); break;
    case kStage1: hipLaunchKernelGGL((k_amr_stage<W, NT, kStage1, LIM>), g, b, 0, stream, a, t0, t1); break;
    case kStage23: hipLaunchKernelGGL((k_amr_stage<W, NT, kStage23, LIM>), g, b, 0, stream, a, t0, t1); break;
    default: hipLaunchKernelGGL((k_amr_stage<W, NT, kStage4, LIM>), g, b, 0, stream, a, t0, t1); break;
    }
    return hipGetLastError();
}

template <int W, int NT>
hipError_t launch_amr_t(int kind, const AmrArgs& a, int t0, int t1, int grid, hipStream_t stream)
{
    return a.lim ? launch_amr_l<W, NT, true>(kind, a, t0, t1, grid, stream)
                 : launch_amr_l<W, NT, false>(kind, a, t0, t1, grid, stream);
}

}  // namespace

// coarse data of one fine stage of a subcycled step, from the coarse step's
// states h_0 = f^n, h_1 .. h_3 (the stage predictors) and h_4 (the end of
// the step), each `stride` elements apart: out = h_0 + sum_q c_q (h_q - h_0)
__global__ __launch_bounds__(256) void k_amr_substage(const double* __restrict__ h, size_t n, size_t stride,
                                                     double c1, double c2, double c3, double c4,
                                                     double* __restrict__ out)
{
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (size_t)gridDim.x * 256) {
        const double b = h[q];
        const double d1 = h[stride + q] - b, d2 = h[2 * stride + q] - b;
        const double d3 = h[3 * stride + q] - b, d4 = h[4 * stride + q] - b;
        out[q] = b + (c1 * d1 + c2 * d2 + c3 * d3 + c4 * d4);
    }
}

hipError_t launch_amr_stage(int w, int nt, int kind, const AmrArgs& a, int t_begin, int t_end, int grid,
                            hipStream_t stream)
{
    if (t_end <= t_begin) return hipSuccess;
    if (w == 2 && nt == 64) return launch_amr_t<2, 64>(kind, a, t_begin, t_end, grid, stream);
    if (w == 2 && nt == 128) return launch_amr_t<2, 128>(kind, a, t_begin, t_end, grid, stream);
    if (w == 1 && nt == 64) return launch_amr_t<1, 64>(kind, a, t_begin, t_end, grid, stream);
    if (w == 1 && nt == 128) return launch_amr_t<1, 128>(kind, a, t_begin, t_end, grid, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_amr_rowsum(const double* f, const long long* task_off, const int* task_len, int ntasks,
                             double* slots, hipStream_t stream)
{
    if (ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_amr_rowsum, dim3((ntasks + 3) / 4), dim3(256), 0, stream, f, task_off, task_len, ntasks,
                       slots);
    return hipGetLastError();
}

hipError_t launch_amr_reduce_finalize(const double* slots, const int* rowptr, const int* idx, const double* w,
                                      int nfx, double* n, hipStream_t stream)
{
    hipLaunchKernelGGL(k_amr_reduce_finalize, dim3((nfx + 15) / 16), dim3(256), 0, stream, slots, rowptr, idx,
                       w, nfx, n);
    return hipGetLastError();
}

hipError_t launch_amr_mask_rows(const double* f, const unsigned char* covered, int ncx, int ncv, double* S,
                                hipStream_t stream)
{
    hipLaunchKernelGGL(k_amr_mask_rows, dim3((5 * ncx + 3) / 4), dim3(256), 0, stream, f, covered, ncx, ncv, S);
    return hipGetLastError();
}

hipError_t launch_amr_mask_fused(const AmrMaskFusedArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_amr_mask_fused, dim3((a.ncx + 3) / 4), dim3(256), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_amr_inject(const double* E, int ncx, int R, double qm, double* a, hipStream_t stream)
{
    const int n = ncx + ncx * R;
    hipLaunchKernelGGL(k_amr_inject, dim3((n + 255) / 256), dim3(256), 0, stream, E, ncx, R, qm, a);
    return hipGetLastError();
}

hipError_t launch_amr_substage(const double* hist, size_t n, size_t stride, const double c[4], double* out,
                               hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_amr_substage, dim3(grid), dim3(256), 0, stream, hist, n, stride, c[0], c[1], c[2], c[3],
                       out);
    return hipGetLastError();
}

hipError_t launch_amr_sync(const AmrSyncArgs& s, hipStream_t stream)
{
    const int n = s.ncorr + s.ncov;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_amr_sync, dim3((n + 255) / 256), dim3(256), 0, stream, s);
    return hipGetLastError();
}

}  // namespace vp
