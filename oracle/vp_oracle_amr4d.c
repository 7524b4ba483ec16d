/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Two-level 2D+2V Vlasov-Poisson step (the AMR of section 3 carried to the
 * 2D+2V phase space that section 5 leaves to future work), f stored
 * [x][y][vx][vy] on level 0 and on every level-1 patch:
 *
 *   each stage: predictor on both levels; the ghost cells of a patch (two
 *   layers in every direction): a cell that a level-1 patch holds is copied
 *   (x, y periodic), one outside the velocity box takes the fine
 *   equilibrium product, the others are the conservative fifth-order
 *   sub-cell interpolation of level 0 as a tensor product over the four
 *   directions (x, then y, then vx, then vy; the 1D weights of section 3);
 *   the constraint (Mask Reduction, Alg. mreduce: level 0 refined in x and
 *   y to the fine configuration mesh by the tensor sub-cell interpolation,
 *   masked where level 1 covers the coarse cell, summed over velocity; the
 *   patches summed over velocity; the 2D Poisson problem and the field on
 *   the fine configuration mesh; level 0 takes the mean of the R^2 fine
 *   field values of each coarse cell); the fluxes of section 2 extended
 *   direction by direction (as the single-level 2D+2V oracle) on every
 *   patch; F_accum += b_s F.
 *   update: the patches from their accumulated fluxes; level 0 with its
 *   coarse-fine faces taking the mean of the R^3 fine accumulated fluxes
 *   on the coincident fine faces; then covered coarse cells take the mean
 *   of their R^4 fine cells.
 * One refinement ratio R in all four directions; patches are disjoint and
 * may touch (also across the periodic boundaries).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vp_oracle.h"

static int wr(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }
static int fdv(int a, int b) { int q = a / b; return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q; }

typedef struct {
    int lo[4], hi[4];
    long off;
} p4box;

typedef struct {
    int n[4];                  /* level-0 cells */
    int nf[4];                 /* level-1 index space */
    int R, np;
    double h[4], hf[4];        /* cell sizes of both levels */
    double v_lo, qm, x_len, y_len, v_hi;
    double *gxc, *gyc, *gxf, *gyf;   /* 1D equilibria with two ghosts (n + 4) */
    p4box* P;
    long total;
    double B[16][5];
    void* pf;                  /* single-level 2D+2V context on the fine configuration mesh (Poisson, field) */
} vpo_a4;

#define PSIZE(b, d) ((b).hi[d] - (b).lo[d] + 1)

static long idx4(const int* n, int i, int j, int k, int l) { return (((long)i * n[1] + j) * n[2] + k) * n[3] + l; }

/* level-0 cell, x and y periodic, velocity ghosts the coarse equilibrium product */
static double coarse_at(const vpo_a4* c, const double* f, int i, int j, int k, int l)
{
    if (k < 0 || k >= c->n[2] || l < 0 || l >= c->n[3]) return c->gxc[k + 2] * c->gyc[l + 2];
    return f[idx4(c->n, wr(i, c->n[0]), wr(j, c->n[1]), k, l)];
}

/* level-1 cell held by a patch: 1 and its value */
static int fine_held(const vpo_a4* c, const double* f, int I, int J, int K, int L, double* v)
{
    if (K < 0 || K >= c->nf[2] || L < 0 || L >= c->nf[3]) return 0;
    const int X = wr(I, c->nf[0]), Y = wr(J, c->nf[1]);
    for (int p = 0; p < c->np; ++p) {
        const p4box* b = &c->P[p];
        if (X < b->lo[0] || X > b->hi[0] || Y < b->lo[1] || Y > b->hi[1] || K < b->lo[2] || K > b->hi[2] ||
            L < b->lo[3] || L > b->hi[3]) continue;
        const int sz[4] = {PSIZE(*b, 0), PSIZE(*b, 1), PSIZE(*b, 2), PSIZE(*b, 3)};
        *v = f[b->off + idx4(sz, X - b->lo[0], Y - b->lo[1], K - b->lo[2], L - b->lo[3])];
        return 1;
    }
    return 0;
}

/* any level-1 cell: held, fine equilibrium outside the velocity box, else
 * the tensor sub-cell interpolation of level 0 (x, y, vx, vy in turn) */
static double fine_value(const vpo_a4* c, const double* f, int I, int J, int K, int L)
{
    double v;
    if (K < 0 || K >= c->nf[2] || L < 0 || L >= c->nf[3]) return c->gxf[K + 2] * c->gyf[L + 2];
    if (fine_held(c, f, I, J, K, L, &v)) return v;
    const int R = c->R;
    const int ci = fdv(I, R), cj = fdv(J, R), ck = fdv(K, R), cl = fdv(L, R);
    const int si = I - ci * R, sj = J - cj * R, sk = K - ck * R, sl = L - cl * R;
    double acc = 0.0;
    for (int d = -2; d <= 2; ++d) {
        double av = 0.0;
        for (int e = -2; e <= 2; ++e) {
            double ay = 0.0;
            for (int b = -2; b <= 2; ++b) {
                double ax = 0.0;
                for (int a = -2; a <= 2; ++a) ax += c->B[si][a + 2] * coarse_at(c, f, ci + a, cj + b, ck + e, cl + d);
                ay += c->B[sj][b + 2] * ax;
            }
            av += c->B[sk][e + 2] * ay;
        }
        acc += c->B[sl][d + 2] * av;
    }
    return acc;
}

void* vpo_a4_new(const int* ncells, double x_len, double y_len, double v_lo, double v_hi, double qm, int R, int np,
                 const int* boxes, const double* gxc, const double* gyc, const double* gxf, const double* gyf)
{
    vpo_a4* c = (vpo_a4*)calloc(1, sizeof(*c));
    c->R = R; c->np = np;
    c->v_lo = v_lo; c->v_hi = v_hi; c->qm = qm; c->x_len = x_len; c->y_len = y_len;
    for (int d = 0; d < 4; ++d) { c->n[d] = ncells[d]; c->nf[d] = ncells[d] * R; }
    c->h[0] = x_len / c->n[0]; c->h[1] = y_len / c->n[1];
    c->h[2] = (v_hi - v_lo) / c->n[2]; c->h[3] = (v_hi - v_lo) / c->n[3];
    for (int d = 0; d < 4; ++d) c->hf[d] = c->h[d] / R;
    c->gxc = (double*)malloc(sizeof(double) * (c->n[2] + 4)); memcpy(c->gxc, gxc, sizeof(double) * (c->n[2] + 4));
    c->gyc = (double*)malloc(sizeof(double) * (c->n[3] + 4)); memcpy(c->gyc, gyc, sizeof(double) * (c->n[3] + 4));
    c->gxf = (double*)malloc(sizeof(double) * (c->nf[2] + 4)); memcpy(c->gxf, gxf, sizeof(double) * (c->nf[2] + 4));
    c->gyf = (double*)malloc(sizeof(double) * (c->nf[3] + 4)); memcpy(c->gyf, gyf, sizeof(double) * (c->nf[3] + 4));
    c->P = (p4box*)malloc(sizeof(p4box) * (np > 0 ? np : 1));
    long off = (long)c->n[0] * c->n[1] * c->n[2] * c->n[3];
    for (int p = 0; p < np; ++p) {
        for (int d = 0; d < 4; ++d) { c->P[p].lo[d] = boxes[8 * p + d]; c->P[p].hi[d] = boxes[8 * p + 4 + d]; }
        c->P[p].off = off;
        long s = 1;
        for (int d = 0; d < 4; ++d) s *= PSIZE(c->P[p], d);
        off += s;
    }
    c->total = off;
    vpo_interp_weights(R, &c->B[0][0]);
    c->pf = vpo4_ctx_new(c->nf[0], c->nf[1], c->nf[2], c->nf[3], x_len, y_len, v_lo, v_hi, qm, gxf, gyf);
    return c;
}

void vpo_a4_free(void* h)
{
    vpo_a4* c = (vpo_a4*)h;
    if (!c) return;
    free(c->gxc); free(c->gyc); free(c->gxf); free(c->gyf); free(c->P);
    vpo4_ctx_free(c->pf);
    free(c);
}

long vpo_a4_state_size(void* h) { return ((vpo_a4*)h)->total; }
long vpo_a4_patch_offset(void* h, int p) { return p < 0 ? 0 : ((vpo_a4*)h)->P[p].off; }

/* patch p (-1: level 0) with two ghost layers in every direction */
void vpo_a4_fill_ghosts(void* h, const double* f, int p, double* out)
{
    const vpo_a4* c = (const vpo_a4*)h;
    int lo[4], sz[4];
    for (int d = 0; d < 4; ++d) {
        lo[d] = p < 0 ? 0 : c->P[p].lo[d];
        sz[d] = p < 0 ? c->n[d] : PSIZE(c->P[p], d);
    }
    const int g[4] = {sz[0] + 4, sz[1] + 4, sz[2] + 4, sz[3] + 4};
    for (int i = -2; i < sz[0] + 2; ++i)
        for (int j = -2; j < sz[1] + 2; ++j)
            for (int k = -2; k < sz[2] + 2; ++k)
                for (int l = -2; l < sz[3] + 2; ++l) {
                    const int I = lo[0] + i, J = lo[1] + j, K = lo[2] + k, L = lo[3] + l;
                    out[idx4(g, i + 2, j + 2, k + 2, l + 2)] =
                        p < 0 ? coarse_at(c, f, I, J, K, L) : fine_value(c, f, I, J, K, L);
                }
}

static double face4(double um1, double u0, double u1, double u2) { return (7.0 * (u0 + u1) - (um1 + u2)) / 12.0; }

/* fluxes of section 2, direction by direction, on a patch from its ghosted
 * data g: G[0] x faces [(nx+1)][ny][nvx][nvy], G[1] y faces, G[2] vx faces,
 * G[3] vy faces; ae[c][(i+1)*(ny+2) + (j+1)]: component c of a at patch
 * configuration cell (i, j), i = -1 .. nx, j = -1 .. ny */
static void patch_fluxes4(const int* sz, const double* g, const double* h, const double* vlo, const double* ae,
                          double** G)
{
    const int gs[4] = {sz[0] + 4, sz[1] + 4, sz[2] + 4, sz[3] + 4};
#define U(i, j, k, l) g[idx4(gs, (i) + 2, (j) + 2, (k) + 2, (l) + 2)]
#define AE(cc, i, j) ae[(cc) * (sz[0] + 2) * (sz[1] + 2) + ((i) + 1) * (sz[1] + 2) + ((j) + 1)]
    const int nx = sz[0], ny = sz[1], nvx = sz[2], nvy = sz[3];
    for (int i = -1; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            for (int k = 0; k < nvx; ++k)
                for (int l = 0; l < nvy; ++l) {
                    const double fc = face4(U(i - 1, j, k, l), U(i, j, k, l), U(i + 1, j, k, l), U(i + 2, j, k, l));
                    const double fu = face4(U(i - 1, j, k + 1, l), U(i, j, k + 1, l), U(i + 1, j, k + 1, l), U(i + 2, j, k + 1, l));
                    const double fd = face4(U(i - 1, j, k - 1, l), U(i, j, k - 1, l), U(i + 1, j, k - 1, l), U(i + 2, j, k - 1, l));
                    const double vb = vlo[2] + (k + 0.5) * h[2];
                    const int n1[4] = {nx + 1, ny, nvx, nvy};
                    G[0][idx4(n1, i + 1, j, k, l)] = vb * fc + h[2] / 24.0 * (fu - fd);
                }
    for (int i = 0; i < nx; ++i)
        for (int j = -1; j < ny; ++j)
            for (int k = 0; k < nvx; ++k)
                for (int l = 0; l < nvy; ++l) {
                    const double fc = face4(U(i, j - 1, k, l), U(i, j, k, l), U(i, j + 1, k, l), U(i, j + 2, k, l));
                    const double fu = face4(U(i, j - 1, k, l + 1), U(i, j, k, l + 1), U(i, j + 1, k, l + 1), U(i, j + 2, k, l + 1));
                    const double fd = face4(U(i, j - 1, k, l - 1), U(i, j, k, l - 1), U(i, j + 1, k, l - 1), U(i, j + 2, k, l - 1));
                    const double vb = vlo[3] + (l + 0.5) * h[3];
                    const int n1[4] = {nx, ny + 1, nvx, nvy};
                    G[1][idx4(n1, i, j + 1, k, l)] = vb * fc + h[3] / 24.0 * (fu - fd);
                }
#define FVX(i, j, k, l) face4(U(i, j, (k) - 1, l), U(i, j, k, l), U(i, j, (k) + 1, l), U(i, j, (k) + 2, l))
#define FVY(i, j, k, l) face4(U(i, j, k, (l) - 1), U(i, j, k, l), U(i, j, k, (l) + 1), U(i, j, k, (l) + 2))
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            const double ax = AE(0, i, j), dax = AE(0, i + 1, j) - AE(0, i - 1, j), day = AE(0, i, j + 1) - AE(0, i, j - 1);
            const double ay = AE(1, i, j), dbx = AE(1, i + 1, j) - AE(1, i - 1, j), dby = AE(1, i, j + 1) - AE(1, i, j - 1);
            for (int k = -1; k < nvx; ++k)
                for (int l = 0; l < nvy; ++l) {
                    const int n1[4] = {nx, ny, nvx + 1, nvy};
                    G[2][idx4(n1, i, j, k + 1, l)] =
                        ax * FVX(i, j, k, l) + (dax * (FVX(i + 1, j, k, l) - FVX(i - 1, j, k, l)) +
                                                day * (FVX(i, j + 1, k, l) - FVX(i, j - 1, k, l))) / 48.0;
                }
            for (int k = 0; k < nvx; ++k)
                for (int l = -1; l < nvy; ++l) {
                    const int n1[4] = {nx, ny, nvx, nvy + 1};
                    G[3][idx4(n1, i, j, k, l + 1)] =
                        ay * FVY(i, j, k, l) + (dbx * (FVY(i + 1, j, k, l) - FVY(i - 1, j, k, l)) +
                                                dby * (FVY(i, j + 1, k, l) - FVY(i, j - 1, k, l))) / 48.0;
                }
        }
#undef FVX
#undef FVY
#undef U
#undef AE
}

static void divergence4(const int* sz, double* const* G, const double* h, double* k)
{
    const int nx = sz[0], ny = sz[1], nvx = sz[2], nvy = sz[3];
    const int n0[4] = {nx + 1, ny, nvx, nvy}, n1[4] = {nx, ny + 1, nvx, nvy}, n2[4] = {nx, ny, nvx + 1, nvy},
              n3[4] = {nx, ny, nvx, nvy + 1};
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            for (int a = 0; a < nvx; ++a)
                for (int b = 0; b < nvy; ++b)
                    k[idx4(sz, i, j, a, b)] = -(G[0][idx4(n0, i + 1, j, a, b)] - G[0][idx4(n0, i, j, a, b)]) / h[0]
                                              - (G[1][idx4(n1, i, j + 1, a, b)] - G[1][idx4(n1, i, j, a, b)]) / h[1]
                                              - (G[2][idx4(n2, i, j, a + 1, b)] - G[2][idx4(n2, i, j, a, b)]) / h[2]
                                              - (G[3][idx4(n3, i, j, a, b + 1)] - G[3][idx4(n3, i, j, a, b)]) / h[3];
}

static long face_count(const int* sz, int d)
{
    long s = 1;
    for (int e = 0; e < 4; ++e) s *= sz[e] + (e == d);
    return s;
}

static void patch_geom(const vpo_a4* c, int p, int* lo, int* sz, double* h, double* vlo)
{
    for (int d = 0; d < 4; ++d) {
        lo[d] = p < 0 ? 0 : c->P[p].lo[d];
        sz[d] = p < 0 ? c->n[d] : PSIZE(c->P[p], d);
        h[d] = p < 0 ? c->h[d] : c->hf[d];
    }
    vlo[2] = c->v_lo + lo[2] * h[2];
    vlo[3] = c->v_lo + lo[3] * h[3];
}

/* fluxes of patch p (-1: level 0); a = [a_c (2 nx ny)][a_f (2 nfx nfy)], components x then y */
static void fluxes_of(const vpo_a4* c, const double* f, const double* a, int p, double** G)
{
    int lo[4], sz[4];
    double h[4], vlo[4];
    patch_geom(c, p, lo, sz, h, vlo);
    long gsz = 1;
    for (int d = 0; d < 4; ++d) gsz *= sz[d] + 4;
    double* g = (double*)malloc(sizeof(double) * gsz);
    vpo_a4_fill_ghosts((void*)c, f, p, g);
    const int mx = p < 0 ? c->n[0] : c->nf[0], my = p < 0 ? c->n[1] : c->nf[1];
    const double* al = p < 0 ? a : a + 2 * (long)c->n[0] * c->n[1];
    double* ae = (double*)malloc(sizeof(double) * 2 * (sz[0] + 2) * (sz[1] + 2));
    for (int cc = 0; cc < 2; ++cc)
        for (int i = -1; i <= sz[0]; ++i)
            for (int j = -1; j <= sz[1]; ++j)
                ae[cc * (sz[0] + 2) * (sz[1] + 2) + (i + 1) * (sz[1] + 2) + (j + 1)] =
                    al[(long)cc * mx * my + (long)wr(lo[0] + i, mx) * my + wr(lo[1] + j, my)];
    patch_fluxes4(sz, g, h, vlo, ae, G);
    free(ae);
    free(g);
}

/* Mask Reduction onto the fine configuration mesh: n[(I) nfy + J] */
void vpo_a4_reduce_mask(void* h, const double* f, double* n)
{
    const vpo_a4* c = (const vpo_a4*)h;
    const int R = c->R, nfx = c->nf[0], nfy = c->nf[1];
    const double dvc = c->h[2] * c->h[3], dvf = c->hf[2] * c->hf[3];
    for (int I = 0; I < nfx; ++I)
        for (int J = 0; J < nfy; ++J) {
            const int i = I / R, j = J / R, s = I % R, t = J % R;
            double sc = 0.0;
            for (int k = 0; k < c->n[2]; ++k)
                for (int l = 0; l < c->n[3]; ++l) {
                    double dummy;
                    if (fine_held(c, f, i * R, j * R, k * R, l * R, &dummy)) continue;   /* covered */
                    double acc = 0.0;
                    for (int b = -2; b <= 2; ++b) {
                        double ax = 0.0;
                        for (int a = -2; a <= 2; ++a) ax += c->B[s][a + 2] * coarse_at(c, f, i + a, j + b, k, l);
                        acc += c->B[t][b + 2] * ax;
                    }
                    sc += acc;
                }
            double sf = 0.0;
            for (int p = 0; p < c->np; ++p) {
                const p4box* b = &c->P[p];
                if (I < b->lo[0] || I > b->hi[0] || J < b->lo[1] || J > b->hi[1]) continue;
                const int sz[4] = {PSIZE(*b, 0), PSIZE(*b, 1), PSIZE(*b, 2), PSIZE(*b, 3)};
                for (int k = 0; k < sz[2]; ++k)
                    for (int l = 0; l < sz[3]; ++l) sf += f[b->off + idx4(sz, I - b->lo[0], J - b->lo[1], k, l)];
            }
            n[(long)I * nfy + J] = dvc * sc + dvf * sf;
        }
}

/* a = [a_c x][a_c y][a_f x][a_f y]; E on the fine configuration mesh (x then y) */
void vpo_a4_constraints(void* h, const double* f, double* a, double* E_out)
{
    const vpo_a4* c = (const vpo_a4*)h;
    const int R = c->R, nfx = c->nf[0], nfy = c->nf[1], ncx = c->n[0], ncy = c->n[1];
    const long nf = (long)nfx * nfy, nc = (long)ncx * ncy;
    double* n = (double*)malloc(sizeof(double) * nf);
    double* phi = (double*)malloc(sizeof(double) * nf);
    double* E = (double*)malloc(sizeof(double) * 2 * nf);
    vpo_a4_reduce_mask(h, f, n);
    for (long q = 0; q < nf; ++q) n[q] = 1.0 - n[q];
    vpo4_poisson(c->pf, n, phi);
    vpo4_field(c->pf, phi, E);
    for (int cc = 0; cc < 2; ++cc) {
        for (int i = 0; i < ncx; ++i)
            for (int j = 0; j < ncy; ++j) {
                double s = 0.0;
                for (int a = 0; a < R; ++a)
                    for (int b = 0; b < R; ++b) s += E[cc * nf + (long)(i * R + a) * nfy + (j * R + b)];
                a[cc * nc + (long)i * ncy + j] = c->qm * s / (R * R);
            }
        for (long q = 0; q < nf; ++q) a[2 * nc + cc * nf + q] = c->qm * E[cc * nf + q];
    }
    if (E_out) memcpy(E_out, E, sizeof(double) * 2 * nf);
    free(n); free(phi); free(E);
}

static double** alloc_G(const vpo_a4* c, int zero)
{
    double** G = (double**)malloc(sizeof(double*) * 4 * (c->np + 1));
    for (int p = -1; p < c->np; ++p) {
        int lo[4], sz[4];
        double hh[4], vlo[4];
        patch_geom(c, p, lo, sz, hh, vlo);
        for (int d = 0; d < 4; ++d)
            G[4 * (p + 1) + d] = (double*)(zero ? calloc(face_count(sz, d), sizeof(double))
                                                : malloc(sizeof(double) * face_count(sz, d)));
    }
    return G;
}

static void free_G(const vpo_a4* c, double** G)
{
    for (int q = 0; q < 4 * (c->np + 1); ++q) free(G[q]);
    free(G);
}

void vpo_a4_rhs(void* h, const double* f, const double* a, double* k)
{
    const vpo_a4* c = (const vpo_a4*)h;
    double** G = alloc_G(c, 0);
    for (int p = -1; p < c->np; ++p) {
        int lo[4], sz[4];
        double hh[4], vlo[4];
        patch_geom(c, p, lo, sz, hh, vlo);
        fluxes_of(c, f, a, p, G + 4 * (p + 1));
        divergence4(sz, G + 4 * (p + 1), hh, k + (p < 0 ? 0 : c->P[p].off));
    }
    free_G(c, G);
}

/* level-0 cell (i, j, k, l) covered by a patch (coarse indices, x y periodic) */
static int covered(const vpo_a4* c, const double* f, int i, int j, int k, int l)
{
    double d;
    if (k < 0 || k >= c->n[2] || l < 0 || l >= c->n[3]) return 0;
    return fine_held(c, f, i * c->R, j * c->R, k * c->R, l * c->R, &d);
}

void vpo_a4_rk4_step(void* h, const double* f_in, double* f_out, double dt)
{
    static const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    static const double bw[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const vpo_a4* c = (const vpo_a4*)h;
    const long N = c->total;
    const long na = 2 * ((long)c->n[0] * c->n[1] + (long)c->nf[0] * c->nf[1]);
    double* fs = (double*)malloc(sizeof(double) * N);
    double* k = (double*)calloc(N, sizeof(double));
    double* a = (double*)malloc(sizeof(double) * na);
    double** G = alloc_G(c, 0);
    double** A = alloc_G(c, 1);
    for (int s = 0; s < 4; ++s) {
        for (long q = 0; q < N; ++q) fs[q] = f_in[q] + alpha[s] * dt * k[q];
        vpo_a4_constraints(h, fs, a, NULL);
        for (int p = -1; p < c->np; ++p) {
            int lo[4], sz[4];
            double hh[4], vlo[4];
            patch_geom(c, p, lo, sz, hh, vlo);
            fluxes_of(c, fs, a, p, G + 4 * (p + 1));
            divergence4(sz, G + 4 * (p + 1), hh, k + (p < 0 ? 0 : c->P[p].off));
            for (int d = 0; d < 4; ++d)
                for (long q = 0; q < face_count(sz, d); ++q) A[4 * (p + 1) + d][q] += bw[s] * G[4 * (p + 1) + d][q];
        }
    }
    /* ComputeUpdate: patches from their accumulated fluxes */
    for (int p = 0; p < c->np; ++p) {
        int lo[4], sz[4];
        double hh[4], vlo[4];
        patch_geom(c, p, lo, sz, hh, vlo);
        long cnt = (long)sz[0] * sz[1] * sz[2] * sz[3];
        double* kk = (double*)malloc(sizeof(double) * cnt);
        divergence4(sz, A + 4 * (p + 1), hh, kk);
        for (long q = 0; q < cnt; ++q) f_out[c->P[p].off + q] = f_in[c->P[p].off + q] + dt * kk[q];
        free(kk);
    }
    /* coarse faces on coarse-fine interfaces take the mean of the fine accumulated fluxes */
    const int R = c->R;
    const int* n = c->n;
    for (int d = 0; d < 4; ++d) {
        const int nd[4] = {n[0] + (d == 0), n[1] + (d == 1), n[2] + (d == 2), n[3] + (d == 3)};
        for (int i = 0; i < nd[0]; ++i)
            for (int j = 0; j < nd[1]; ++j)
                for (int kk = 0; kk < nd[2]; ++kk)
                    for (int l = 0; l < nd[3]; ++l) {
                        /* face between cell (..) - e_d and cell (..) */
                        int hi[4] = {i, j, kk, l}, lo2[4] = {i, j, kk, l};
                        lo2[d] -= 1;
                        if (d >= 2 && (lo2[d] < 0 || hi[d] >= n[d])) continue;     /* velocity boundary */
                        const int cl = covered(c, f_in, lo2[0], lo2[1], lo2[2], lo2[3]);
                        const int ch = covered(c, f_in, hi[0], hi[1], hi[2], hi[3]);
                        if (cl == ch) continue;
                        /* the covering patch and its face: fine position R * hi[d] */
                        const int* cov = ch ? hi : lo2;
                        double dummy;
                        int q = -1;
                        for (int pp = 0; pp < c->np && q < 0; ++pp) {
                            const p4box* b = &c->P[pp];
                            int in = 1;
                            for (int e = 0; e < 4; ++e) {
                                const int F = (e < 2 ? wr(cov[e], n[e]) : cov[e]) * R;
                                if (F < b->lo[e] || F > b->hi[e]) in = 0;
                            }
                            if (in) q = pp;
                        }
                        (void)dummy;
                        const p4box* b = &c->P[q];
                        const int sz[4] = {PSIZE(*b, 0), PSIZE(*b, 1), PSIZE(*b, 2), PSIZE(*b, 3)};
                        const int nq[4] = {sz[0] + (d == 0), sz[1] + (d == 1), sz[2] + (d == 2), sz[3] + (d == 3)};
                        const int fpos = ch ? 0 : sz[d];       /* the patch's lower or upper face */
                        double s = 0.0;
                        int cnt = 0;
                        int base[4];
                        for (int e = 0; e < 4; ++e) base[e] = (e < 2 ? wr(hi[e], n[e]) : hi[e]) * R - b->lo[e];
                        for (int u0 = 0; u0 < (d == 0 ? 1 : R); ++u0)
                            for (int u1 = 0; u1 < (d == 1 ? 1 : R); ++u1)
                                for (int u2 = 0; u2 < (d == 2 ? 1 : R); ++u2)
                                    for (int u3 = 0; u3 < (d == 3 ? 1 : R); ++u3) {
                                        int ix[4] = {base[0] + u0, base[1] + u1, base[2] + u2, base[3] + u3};
                                        ix[d] = fpos;
                                        s += A[4 * (q + 1) + d][idx4(nq, ix[0], ix[1], ix[2], ix[3])];
                                        ++cnt;
                                    }
                        A[d][idx4(nd, i, j, kk, l)] = s / cnt;
                        /* periodic x, y: face n[d] is face 0 */
                        if (d < 2 && (d == 0 ? i : j) == 0) {
                            int w[4] = {i, j, kk, l};
                            w[d] = n[d];
                            A[d][idx4(nd, w[0], w[1], w[2], w[3])] = s / cnt;
                        }
                        if (d < 2 && (d == 0 ? i : j) == n[d]) {
                            int w[4] = {i, j, kk, l};
                            w[d] = 0;
                            A[d][idx4(nd, w[0], w[1], w[2], w[3])] = s / cnt;
                        }
                    }
    }
    {
        const long nc = (long)n[0] * n[1] * n[2] * n[3];
        double* kk = (double*)malloc(sizeof(double) * nc);
        divergence4(n, A, c->h, kk);
        for (long q = 0; q < nc; ++q) f_out[q] = f_in[q] + dt * kk[q];
        free(kk);
    }
    /* covered coarse cells: mean of their R^4 fine cells */
    for (int p = 0; p < c->np; ++p) {
        const p4box* b = &c->P[p];
        const int sz[4] = {PSIZE(*b, 0), PSIZE(*b, 1), PSIZE(*b, 2), PSIZE(*b, 3)};
        for (int i = b->lo[0] / R; i <= b->hi[0] / R; ++i)
            for (int j = b->lo[1] / R; j <= b->hi[1] / R; ++j)
                for (int kk = b->lo[2] / R; kk <= b->hi[2] / R; ++kk)
                    for (int l = b->lo[3] / R; l <= b->hi[3] / R; ++l) {
                        double s = 0.0;
                        for (int u0 = 0; u0 < R; ++u0)
                            for (int u1 = 0; u1 < R; ++u1)
                                for (int u2 = 0; u2 < R; ++u2)
                                    for (int u3 = 0; u3 < R; ++u3)
                                        s += f_out[b->off + idx4(sz, i * R + u0 - b->lo[0], j * R + u1 - b->lo[1],
                                                                 kk * R + u2 - b->lo[2], l * R + u3 - b->lo[3])];
                        f_out[idx4(n, i, j, kk, l)] = s / ((double)R * R * R * R);
                    }
    }
    free_G(c, G);
    free_G(c, A);
    free(fs); free(k); free(a);
}
