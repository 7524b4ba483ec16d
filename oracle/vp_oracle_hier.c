/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Multi-level (L <= 4) 1D+1V Vlasov-Poisson step on a block-structured
 * phase-space hierarchy with a refinement ratio per level and direction
 * (section 3: the hierarchy G_H of levels L_0 .. L_{L-1} with ratio vectors
 * r_l^{l+1}; section 4 runs ratios [2,4], [4,2], [2,2]), written as the
 * synchronous multi-level algorithm (Algs. ssthu / mspsc / msrhsfa / msfduc
 * / smsvphu, without regridding):
 *
 *   each stage: predictor on every level; ghost cells of every patch of
 *   level l >= 1: a cell that a level-l patch holds is copied from it (the
 *   exchange of ghost cells on a level; x periodic), one outside the
 *   velocity box takes the level's equilibrium, the others are the
 *   conservative fifth-order sub-cell interpolation of level l-1 along x
 *   (ratio r_x) then along v (ratio r_v); the constraint (Mask Reduction,
 *   Alg. mreduce: each patch's data refined in x to the finest
 *   configuration mesh, masked where the next level covers it, summed over
 *   v with the level's velocity cell size; Poisson and field on the finest
 *   configuration mesh; level l takes the mean of the finest field over
 *   each of its cells); fluxes on every patch; F_accum += b_s F.
 *   update: from the finest level down, each patch's faces that are
 *   coarse-fine faces with the next finer level take the mean of the fine
 *   accumulated fluxes on the coincident fine faces, then f_new = f_old +
 *   dt div F_accum; then, from the finest level down, covered cells take
 *   the mean of the cells of the next finer level.
 *
 * Readings (listed with the others in the design notes):
 *   - the sub-cell weights b_j(s) of section 3 with the corrected p_k and
 *     gamma_1 (as in the two-level oracle), one table per ratio;
 *   - the reduction refines level l in x with the one-step interpolation of
 *     ratio prod_{m>l} r_x^m (the operator I^{l,L-1} of the Mask Reduction),
 *     reading level-l ghost cells where the stencil leaves the patch;
 *   - nesting: every cell a ghost interpolation reads on level l-1 is held
 *     by a level-(l-1) patch or lies outside the velocity box (checked at
 *     creation), so no ghost is interpolated from another ghost.
 * Level 0 is patch 0 (the whole domain); boxes[] lists the other patches
 * (level, lo_x, lo_v, hi_x, hi_v in their level's index space), stored in
 * the state after level 0 in the order given.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vp_oracle.h"

#define HMAXL 4

static int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }
static int fdiv(int a, int b) { int q = a / b; return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q; }

typedef struct {
    int lev, xlo, vlo, xhi, vhi;
    long off;
} hpatch;

typedef struct {
    int L, np;                 /* levels; patches including level 0 (patch 0) */
    int nx[HMAXL], nv[HMAXL];  /* index-space sizes per level */
    int rx[HMAXL], rv[HMAXL];  /* ratio from level l-1 to level l (l >= 1) */
    int rt[HMAXL];             /* x ratio from level l to the finest level */
    double dx[HMAXL], dv[HMAXL], v_lo, qm;
    hpatch* P;
    long total;
    double* veq[HMAXL];        /* nv[l] + 4 values, index 0 is j = -2 */
    double* Bx[HMAXL];         /* rx[l] x 5 */
    double* Bv[HMAXL];         /* rv[l] x 5 */
    double* Br[HMAXL];         /* rt[l] x 5 */
    vpo_poisson* Ps;
} vpo_hier;

#define NXP(P) ((P).xhi - (P).xlo + 1)
#define NVP(P) ((P).vhi - (P).vlo + 1)

/* cell (X, V) of level l (X periodic, V inside the velocity box) held by a
 * patch of that level: its index, else -1 */
static int holder(const vpo_hier* h, int l, int X, int V)
{
    const int Xw = wrap(X, h->nx[l]);
    for (int p = 0; p < h->np; ++p) {
        const hpatch* q = &h->P[p];
        if (q->lev == l && Xw >= q->xlo && Xw <= q->xhi && V >= q->vlo && V <= q->vhi) return p;
    }
    return -1;
}

/* value of cell (X, V) on level l if the level holds it or V lies outside
 * the velocity box (the level's equilibrium); returns 0 otherwise */
static int level_value(const vpo_hier* h, const double* f, int l, int X, int V, double* val)
{
    if (V < 0 || V >= h->nv[l]) {
        *val = h->veq[l][V + 2];
        return 1;
    }
    const int p = holder(h, l, X, V);
    if (p < 0) return 0;
    const hpatch* q = &h->P[p];
    *val = f[q->off + (long)(wrap(X, h->nx[l]) - q->xlo) * NVP(*q) + (V - q->vlo)];
    return 1;
}

/* the sub-cell interpolation of level l-1 at cell (X, V) of level l (x then
 * v); *ok is cleared when a stencil cell is not held by level l-1 */
static double interp_parent(const vpo_hier* h, const double* f, int l, int X, int V, int* ok)
{
    const int ci = fdiv(X, h->rx[l]), s = X - ci * h->rx[l];
    const int cj = fdiv(V, h->rv[l]), t = V - cj * h->rv[l];
    double acc = 0.0;
    for (int b = -2; b <= 2; ++b) {
        double gx = 0.0;
        for (int a = -2; a <= 2; ++a) {
            double u = 0.0;
            if (!level_value(h, f, l - 1, ci + a, cj + b, &u)) *ok = 0;
            gx += h->Bx[l][s * 5 + a + 2] * u;
        }
        acc += h->Bv[l][t * 5 + b + 2] * gx;
    }
    return acc;
}

/* any cell of level l (ghost or not): held, equilibrium, else interpolated */
static double cell_value(const vpo_hier* h, const double* f, int l, int X, int V, int* ok)
{
    double v;
    if (level_value(h, f, l, X, V, &v)) return v;
    return interp_parent(h, f, l, X, V, ok);
}

/* level-l cell (i, j) covered by a level-(l+1) patch: its index, else -1 */
static int covered_by(const vpo_hier* h, int l, int i, int j)
{
    if (l + 1 >= h->L || j < 0 || j >= h->nv[l]) return -1;
    return holder(h, l + 1, i * h->rx[l + 1], j * h->rv[l + 1]);
}

void vpo_hier_free(void* ptr)
{
    vpo_hier* h = (vpo_hier*)ptr;
    if (!h) return;
    for (int l = 0; l < HMAXL; ++l) { free(h->veq[l]); free(h->Bx[l]); free(h->Bv[l]); free(h->Br[l]); }
    free(h->P);
    if (h->Ps) vpo_poisson_free(h->Ps);
    free(h);
}

/* error codes: 1 bad sizes or ratios, 2 box outside its level or not
 * aligned, 3 overlapping boxes, 4 nesting violated */
void* vpo_hier_new(int L, int ncx, int ncv, double x_len, double v_lo, double v_hi, double qm, const int* ratios,
                   int nbox, const int* boxes, const double* veq_all, int* err)
{
    *err = 0;
    if (L < 1 || L > HMAXL || ncx < 1 || ncv < 1) { *err = 1; return NULL; }
    vpo_hier* h = (vpo_hier*)calloc(1, sizeof(*h));
    h->L = L;
    h->v_lo = v_lo;
    h->qm = qm;
    h->nx[0] = ncx; h->nv[0] = ncv; h->rx[0] = h->rv[0] = 1;
    for (int l = 1; l < L; ++l) {
        h->rx[l] = ratios[2 * (l - 1)];
        h->rv[l] = ratios[2 * (l - 1) + 1];
        if (h->rx[l] < 1 || h->rx[l] > 16 || h->rv[l] < 1 || h->rv[l] > 16) { *err = 1; vpo_hier_free(h); return NULL; }
        h->nx[l] = h->nx[l - 1] * h->rx[l];
        h->nv[l] = h->nv[l - 1] * h->rv[l];
    }
    for (int l = 0; l < L; ++l) {
        h->rt[l] = 1;
        for (int m = l + 1; m < L; ++m) h->rt[l] *= h->rx[m];
        h->dx[l] = x_len / h->nx[l];
        h->dv[l] = (v_hi - v_lo) / h->nv[l];
    }
    long vo = 0;
    for (int l = 0; l < L; ++l) {
        h->veq[l] = (double*)malloc(sizeof(double) * (h->nv[l] + 4));
        memcpy(h->veq[l], veq_all + vo, sizeof(double) * (h->nv[l] + 4));
        vo += h->nv[l] + 4;
        h->Bx[l] = (double*)malloc(sizeof(double) * 5 * h->rx[l]);
        h->Bv[l] = (double*)malloc(sizeof(double) * 5 * h->rv[l]);
        h->Br[l] = (double*)malloc(sizeof(double) * 5 * h->rt[l]);
        vpo_interp_weights(h->rx[l], h->Bx[l]);
        vpo_interp_weights(h->rv[l], h->Bv[l]);
        vpo_interp_weights(h->rt[l], h->Br[l]);
    }
    h->np = nbox + 1;
    h->P = (hpatch*)calloc(h->np, sizeof(hpatch));
    h->P[0] = (hpatch){0, 0, 0, ncx - 1, ncv - 1, 0};
    long off = (long)ncx * ncv;
    for (int q = 0; q < nbox; ++q) {
        hpatch b = {boxes[5 * q], boxes[5 * q + 1], boxes[5 * q + 2], boxes[5 * q + 3], boxes[5 * q + 4], off};
        const int l = b.lev;
        if (l < 1 || l >= L || b.xlo < 0 || b.vlo < 0 || b.xhi >= h->nx[l] || b.vhi >= h->nv[l] || b.xlo > b.xhi ||
            b.vlo > b.vhi || b.xlo % h->rx[l] || (b.xhi + 1) % h->rx[l] || b.vlo % h->rv[l] ||
            (b.vhi + 1) % h->rv[l]) {
            *err = 2; vpo_hier_free(h); return NULL;
        }
        for (int r = 1; r <= q; ++r) {
            const hpatch* o = &h->P[r];
            if (o->lev == l && b.xlo <= o->xhi && o->xlo <= b.xhi && b.vlo <= o->vhi && o->vlo <= b.vhi) {
                *err = 3; vpo_hier_free(h); return NULL;
            }
        }
        h->P[q + 1] = b;
        off += (long)NXP(b) * NVP(b);
    }
    h->total = off;
    /* nesting: every interpolated ghost cell's stencil is held by the parent
     * level (the values do not matter here, only the flag) */
    double* zero = (double*)calloc(h->total, sizeof(double));
    int ok = 1;
    for (int p = 1; p < h->np && ok; ++p) {
        const hpatch* q = &h->P[p];
        for (int r = -2; r < NXP(*q) + 2 && ok; ++r)
            for (int c = -2; c < NVP(*q) + 2 && ok; ++c) {
                if (r >= 0 && r < NXP(*q) && c >= 0 && c < NVP(*q)) continue;
                (void)cell_value(h, zero, q->lev, q->xlo + r, q->vlo + c, &ok);
            }
    }
    free(zero);
    if (!ok) { *err = 4; vpo_hier_free(h); return NULL; }
    h->Ps = vpo_poisson_new(h->nx[L - 1]);
    return h;
}

long vpo_hier_state_size(void* ptr) { return ((vpo_hier*)ptr)->total; }
long vpo_hier_patch_offset(void* ptr, int p) { return ((vpo_hier*)ptr)->P[p + 1].off; }

/* patch p (0 = level 0, else boxes[p-1]) with two ghost layers:
 * (nx + 4) x (nv + 4) */
void vpo_hier_fill_ghosts(void* ptr, const double* f, int p, double* out)
{
    const vpo_hier* h = (const vpo_hier*)ptr;
    const hpatch* q = &h->P[p];
    const int nx = NXP(*q), nv = NVP(*q), W = nv + 4;
    int ok = 1;
    for (int r = -2; r < nx + 2; ++r)
        for (int c = -2; c < nv + 2; ++c)
            out[(long)(r + 2) * W + (c + 2)] = cell_value(h, f, q->lev, q->xlo + r, q->vlo + c, &ok);
}

/* Mask Reduction (Alg. mreduce) onto the finest configuration mesh */
void vpo_hier_reduce_mask(void* ptr, const double* f, double* n)
{
    const vpo_hier* h = (const vpo_hier*)ptr;
    const int nfx = h->nx[h->L - 1];
    for (int I = 0; I < nfx; ++I) n[I] = 0.0;
    for (int p = 0; p < h->np; ++p) {
        const hpatch* q = &h->P[p];
        const int l = q->lev, rt = h->rt[l];
        for (int i = q->xlo; i <= q->xhi; ++i)
            for (int s = 0; s < rt; ++s) {
                double sum = 0.0;
                for (int j = q->vlo; j <= q->vhi; ++j) {
                    if (covered_by(h, l, i, j) >= 0) continue;
                    double fx = 0.0;
                    int ok = 1;
                    for (int a = -2; a <= 2; ++a) fx += h->Br[l][s * 5 + a + 2] * cell_value(h, f, l, i + a, j, &ok);
                    sum += fx;
                }
                n[i * rt + s] += h->dv[l] * sum;
            }
    }
}

/* a on every level, [a_0 (nx_0)][a_1 (nx_1)]..; E on the finest mesh */
void vpo_hier_constraints(void* ptr, const double* f, double* a, double* E_out)
{
    const vpo_hier* h = (const vpo_hier*)ptr;
    const int nfx = h->nx[h->L - 1];
    double* n = (double*)malloc(sizeof(double) * nfx);
    double* rho = (double*)malloc(sizeof(double) * nfx);
    double* phi = (double*)malloc(sizeof(double) * nfx);
    double* E = (double*)malloc(sizeof(double) * nfx);
    vpo_hier_reduce_mask(ptr, f, n);
    for (int I = 0; I < nfx; ++I) rho[I] = 1.0 - n[I];
    vpo_poisson_solve(h->Ps, h->dx[h->L - 1], rho, phi);
    vpo_field(nfx, h->dx[h->L - 1], phi, E);
    long o = 0;
    for (int l = 0; l < h->L; ++l) {
        const int rt = h->rt[l];
        for (int i = 0; i < h->nx[l]; ++i) {
            double s = 0.0;
            for (int q = 0; q < rt; ++q) s += E[i * rt + q];
            a[o + i] = h->qm * (s / rt);
        }
        o += h->nx[l];
    }
    if (E_out) memcpy(E_out, E, sizeof(double) * nfx);
    free(n); free(rho); free(phi); free(E);
}

static long level_a_offset(const vpo_hier* h, int l)
{
    long o = 0;
    for (int m = 0; m < l; ++m) o += h->nx[m];
    return o;
}

/* fluxes of patch p from its ghosted data */
static void fluxes_of(const vpo_hier* h, const double* f, const double* a, int p, double* Gx, double* Gv)
{
    const hpatch* q = &h->P[p];
    const int l = q->lev, nx = NXP(*q), nv = NVP(*q);
    double* g = (double*)malloc(sizeof(double) * (long)(nx + 4) * (nv + 4));
    vpo_hier_fill_ghosts((void*)h, f, p, g);
    double* ae = (double*)malloc(sizeof(double) * (nx + 2));
    const double* al = a + level_a_offset(h, l);
    for (int i = -1; i <= nx; ++i) ae[i + 1] = al[wrap(q->xlo + i, h->nx[l])];
    vpo_patch_fluxes(nx, nv, g, h->dv[l], h->v_lo + q->vlo * h->dv[l], ae, Gx, Gv);
    free(ae);
    free(g);
}

static void alloc_fluxes(const vpo_hier* h, double*** Gx, double*** Gv, int zero)
{
    *Gx = (double**)malloc(sizeof(double*) * h->np);
    *Gv = (double**)malloc(sizeof(double*) * h->np);
    for (int p = 0; p < h->np; ++p) {
        const long nx = NXP(h->P[p]), nv = NVP(h->P[p]);
        (*Gx)[p] = (double*)(zero ? calloc((nx + 1) * nv, sizeof(double)) : malloc(sizeof(double) * (nx + 1) * nv));
        (*Gv)[p] = (double*)(zero ? calloc(nx * (nv + 1), sizeof(double)) : malloc(sizeof(double) * nx * (nv + 1)));
    }
}

static void free_fluxes(const vpo_hier* h, double** Gx, double** Gv)
{
    for (int p = 0; p < h->np; ++p) { free(Gx[p]); free(Gv[p]); }
    free(Gx);
    free(Gv);
}

/* k = L(f; a) on every patch */
void vpo_hier_rhs(void* ptr, const double* f, const double* a, double* k)
{
    const vpo_hier* h = (const vpo_hier*)ptr;
    double **Gx, **Gv;
    alloc_fluxes(h, &Gx, &Gv, 0);
    for (int p = 0; p < h->np; ++p) {
        const hpatch* q = &h->P[p];
        fluxes_of(h, f, a, p, Gx[p], Gv[p]);
        vpo_divergence(NXP(*q), NVP(*q), Gx[p], Gv[p], h->dx[q->lev], h->dv[q->lev], k + q->off);
    }
    free_fluxes(h, Gx, Gv);
}

/* ComputeUpdate (Alg. msfduc) from the stage-weighted accumulated fluxes */
static void hier_update(const vpo_hier* h, const double* fn, double** Ax, double** Av, double* f_out, double dt)
{
    for (int l = h->L - 1; l >= 0; --l) {
        for (int p = 0; p < h->np; ++p) {
            const hpatch* q = &h->P[p];
            if (q->lev != l) continue;
            const int nx = NXP(*q), nv = NVP(*q);
            if (l + 1 < h->L) {
                const int rx = h->rx[l + 1], rv = h->rv[l + 1];
                /* x faces: face fi of the patch lies between cells xlo+fi-1 and xlo+fi */
                for (int fi = 0; fi <= nx; ++fi)
                    for (int j = q->vlo; j <= q->vhi; ++j) {
                        const int cl = covered_by(h, l, wrap(q->xlo + fi - 1, h->nx[l]), j);
                        const int cr = covered_by(h, l, wrap(q->xlo + fi, h->nx[l]), j);
                        if ((cl < 0) == (cr < 0)) continue;
                        const int g = cl >= 0 ? cl : cr;
                        const hpatch* G = &h->P[g];
                        const int gnv = NVP(*G);
                        /* covered on the right: the fine patch's lower face; else its upper face */
                        const int ff = cr >= 0 ? 0 : NXP(*G);
                        double s = 0.0;
                        for (int t = 0; t < rv; ++t) s += Ax[g][(long)ff * gnv + (j * rv + t - G->vlo)];
                        Ax[p][(long)fi * nv + (j - q->vlo)] = s / rv;
                    }
                /* v faces: face c lies between cells vlo+c-1 and vlo+c (inside the velocity box only) */
                for (int i = q->xlo; i <= q->xhi; ++i)
                    for (int c = 0; c <= nv; ++c) {
                        const int jb = q->vlo + c - 1, ja = q->vlo + c;
                        if (jb < 0 || ja >= h->nv[l]) continue;
                        const int cb = covered_by(h, l, i, jb), ca = covered_by(h, l, i, ja);
                        if ((cb < 0) == (ca < 0)) continue;
                        const int g = cb >= 0 ? cb : ca;
                        const hpatch* G = &h->P[g];
                        const int gnv = NVP(*G);
                        const int ff = ca >= 0 ? 0 : gnv;
                        double s = 0.0;
                        for (int t = 0; t < rx; ++t) s += Av[g][(long)(i * rx + t - G->xlo) * (gnv + 1) + ff];
                        Av[p][(long)(i - q->xlo) * (nv + 1) + c] = s / rx;
                    }
            }
            double* k = (double*)malloc(sizeof(double) * (long)nx * nv);
            vpo_divergence(nx, nv, Ax[p], Av[p], h->dx[l], h->dv[l], k);
            for (long e = 0; e < (long)nx * nv; ++e) f_out[q->off + e] = fn[q->off + e] + dt * k[e];
            free(k);
        }
    }
    /* covered cells take the mean of the next finer level's cells, finest first */
    for (int l = h->L - 2; l >= 0; --l) {
        const int rx = h->rx[l + 1], rv = h->rv[l + 1];
        for (int p = 0; p < h->np; ++p) {
            const hpatch* G = &h->P[p];
            if (G->lev != l + 1) continue;
            const int gnv = NVP(*G);
            for (int ci = G->xlo / rx; ci <= G->xhi / rx; ++ci)
                for (int cj = G->vlo / rv; cj <= G->vhi / rv; ++cj) {
                    double s = 0.0;
                    for (int a = 0; a < rx; ++a)
                        for (int b = 0; b < rv; ++b)
                            s += f_out[G->off + (long)(ci * rx + a - G->xlo) * gnv + (cj * rv + b - G->vlo)];
                    const int pc = holder(h, l, ci, cj);
                    const hpatch* C = &h->P[pc];
                    f_out[C->off + (long)(ci - C->xlo) * NVP(*C) + (cj - C->vlo)] = s / (rx * rv);
                }
        }
    }
}

/* one synchronous RK4 step of the hierarchy (Alg. smsvphu without regridding) */
void vpo_hier_rk4_step(void* ptr, const double* f_in, double* f_out, double dt)
{
    static const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    static const double bw[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const vpo_hier* h = (const vpo_hier*)ptr;
    const long N = h->total;
    long na = 0;
    for (int l = 0; l < h->L; ++l) na += h->nx[l];
    double* fs = (double*)malloc(sizeof(double) * N);
    double* k = (double*)calloc(N, sizeof(double));
    double* a = (double*)malloc(sizeof(double) * na);
    double **Gx, **Gv, **Ax, **Av;
    alloc_fluxes(h, &Gx, &Gv, 0);
    alloc_fluxes(h, &Ax, &Av, 1);
    for (int s = 0; s < 4; ++s) {
        for (long e = 0; e < N; ++e) fs[e] = f_in[e] + alpha[s] * dt * k[e];
        vpo_hier_constraints(ptr, fs, a, NULL);
        for (int p = 0; p < h->np; ++p) {
            const hpatch* q = &h->P[p];
            const long nx = NXP(*q), nv = NVP(*q);
            fluxes_of(h, fs, a, p, Gx[p], Gv[p]);
            vpo_divergence((int)nx, (int)nv, Gx[p], Gv[p], h->dx[q->lev], h->dv[q->lev], k + q->off);
            for (long e = 0; e < (nx + 1) * nv; ++e) Ax[p][e] += bw[s] * Gx[p][e];
            for (long e = 0; e < nx * (nv + 1); ++e) Av[p][e] += bw[s] * Gv[p][e];
        }
    }
    hier_update(h, f_in, Ax, Av, f_out, dt);
    free_fluxes(h, Gx, Gv);
    free_fluxes(h, Ax, Av);
    free(fs); free(k); free(a);
}

/* ---- regridding of a multi-level hierarchy (section 3) ------------------ */

/* The refinement criterion of section 3 on every cell that a level-l patch
 * holds (delta1 f + delta2 f over x and v with the level's cell sizes;
 * neighbours outside the patch are its ghost cells), in the operation order
 * of vpo_tag_value; values[nx_l * nv_l] is NaN where level l has no patch. */
void vpo_hier_tag_values(void* ptr, const double* f, int l, double* values)
{
    const vpo_hier* h = (const vpo_hier*)ptr;
    const int nx = h->nx[l], nv = h->nv[l];
    const double dx = h->dx[l], dv = h->dv[l];
    for (long e = 0; e < (long)nx * nv; ++e) values[e] = NAN;
    for (int p = 0; p < h->np; ++p) {
        const hpatch* q = &h->P[p];
        if (q->lev != l) continue;
        for (int i = q->xlo; i <= q->xhi; ++i)
            for (int j = q->vlo; j <= q->vhi; ++j) {
                int ok = 1;
                const double c = cell_value(h, f, l, i, j, &ok);
                const double xm = cell_value(h, f, l, i - 1, j, &ok), xp = cell_value(h, f, l, i + 1, j, &ok);
                const double vm = cell_value(h, f, l, i, j - 1, &ok), vp = cell_value(h, f, l, i, j + 1, &ok);
                const double gx = xp - xm, gv = vp - vm;
                const double d1 = sqrt(0.5 * (dx * (gx * gx) + dv * (gv * gv)));
                const double sx = (xp - 2.0 * c) + xm, sv = (vp - 2.0 * c) + vm;
                const double d2 = 0.5 * ((dx * dx) * fabs(sx) + (dv * dv) * fabs(sv));
                values[(long)i * nv + j] = d1 + d2;
            }
    }
}

/* Conservative limited WENO5 prolongation (section 3, eqs. aux1, aux2,
 * interp_r_avg) of level l-1 into the level-l box [x0, x1] x [v0, v1]
 * (aligned to the level pair's ratios): x first with r_x (parent rows
 * cj-2 .. cj+2), then v with r_v; parent cells are read where level l-1
 * holds them, the level's equilibrium outside the velocity box.  out is
 * [x1 - x0 + 1][v1 - v0 + 1]; returns 0 when a parent cell is not held. */
int vpo_hier_prolong_box(void* ptr, const double* f, int l, int x0, int v0, int x1, int v1, double* out)
{
    const vpo_hier* h = (const vpo_hier*)ptr;
    const int rx = h->rx[l], rv = h->rv[l];
    const int cx0 = x0 / rx, cx1 = x1 / rx, cv0 = v0 / rv, cv1 = v1 / rv;
    const int nfx = x1 - x0 + 1, nfv = v1 - v0 + 1, nvt = cv1 - cv0 + 5;
    double* T = (double*)malloc(sizeof(double) * (size_t)nfx * nvt);
    int ok = 1;
    for (int cx = cx0; cx <= cx1; ++cx)
        for (int q = 0; q < nvt; ++q) {
            double u[5], o[64];
            for (int e = 0; e < 5; ++e)
                if (!level_value(h, f, l - 1, cx - 2 + e, cv0 - 2 + q, &u[e])) ok = 0;
            vpo_prolong1d(u, rx, o);
            for (int s = 0; s < rx; ++s) T[(size_t)((cx - cx0) * rx + s) * nvt + q] = o[s];
        }
    for (int x = 0; x < nfx; ++x)
        for (int cv = cv0; cv <= cv1; ++cv) {
            double u[5], o[64];
            for (int e = 0; e < 5; ++e) u[e] = T[(size_t)x * nvt + (cv - cv0) + e];
            vpo_prolong1d(u, rv, o);
            for (int s = 0; s < rv; ++s) out[(size_t)x * nfv + (cv - cv0) * rv + s] = o[s];
        }
    free(T);
    return ok;
}
