/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Two-level (coarse level + level-1 patches) 1D+1V Vlasov-Poisson step,
 * written as the paper's synchronous multi-level algorithm (section 3,
 * Algs. ssthu / mspsc / msrhsfa / msfduc / smsvphu, without regridding):
 *
 *   for each stage: predictor on every level; fine ghost cells filled by
 *   conservative sub-cell interpolation from the coarse predictor of the
 *   same stage; the constraint (Mask Reduction of section 3 -> periodic
 *   Poisson on the finest configuration mesh -> field -> injection);
 *   fluxes on every patch; F_accum += b_s F.
 *   update: every level from its accumulated fluxes, with the coarse
 *   fluxes on coarse-fine faces replaced by the mean of the fine ones
 *   (coarsened fluxes), then covered coarse cells take the average of the
 *   fine cells (restriction is plain summation).
 *
 * Readings (listed with the others in the design notes):
 *   - sub-cell interpolation: the linear fifth-order cell-average formula of
 *     section 3 with p_k(s) = ((s+1)^{k+1} - s^{k+1}) / R^k and the cubic
 *     coefficient of gamma_1 equal to 20 (the printed p_k and 40 break
 *     conservation and the partition of unity);
 *   - two dimensions: x first, then v (dimension by dimension);
 *   - the coarse field is the mean of the R fine field values;
 *   - fine ghosts outside the velocity domain hold the fine equilibrium.
 * Patches are disjoint and may touch, also across the periodic x boundary:
 * fine ghost cells held by a patch are copied from it, so the two patches
 * on a fine-fine face compute its flux from the same values (the flux
 * exchange of Alg. msrhsfa then changes nothing) and only coarse-fine faces
 * take coarsened fluxes.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vp_oracle.h"

static int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }
static int fdiv(int a, int b) { int q = a / b; return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q; }

/* b_j(s), j = -2..2 at out[s*5 + j + 2]: fine-cell averages of the
 * fifth-order interpolant, u^f_{Ri+s} = sum_j b_j(s) u_{i+j} */
void vpo_interp_weights(int R, double* out)
{
    for (int s = 0; s < R; ++s) {
        double p[5];
        p[0] = 1.0;
        for (int k = 1; k <= 4; ++k)
            p[k] = (pow(s + 1.0, k + 1) - pow((double)s, k + 1)) / pow((double)R, k);
        out[s * 5 + 0] = (p[4] - 5 * p[3] + 5 * p[2] + 5 * p[1] - 6) / 120.0;
        out[s * 5 + 1] = (-4 * p[4] + 15 * p[3] + 10 * p[2] - 75 * p[1] + 54) / 120.0;
        out[s * 5 + 2] = (6 * p[4] - 15 * p[3] - 40 * p[2] + 75 * p[1] + 94) / 120.0;
        out[s * 5 + 3] = (-4 * p[4] + 5 * p[3] + 30 * p[2] - 5 * p[1] - 26) / 120.0;
        out[s * 5 + 4] = (p[4] - 5 * p[2] + 4) / 120.0;
    }
}

typedef struct {
    int ncx, ncv, R, nfx, nfv, np;
    double dxc, dvc, dxf, dvf, v_lo, qm;
    int* box;             /* np x 4: lo_x, lo_v, hi_x, hi_v (fine index space) */
    long* off;            /* np + 1 element offsets, off[0] = coarse size */
    unsigned char* cov;   /* coarse cell covered by a patch */
    double* veq_c;        /* ncv + 4 */
    double* veq_f;        /* nfv + 4 */
    double B[16][5];      /* R <= 16 */
    vpo_poisson* P;
    long total;
    int limited;          /* face averages: 0 centred, 1 limited (section 2, eq. limitedFace) */
} vpo_amr;

void* vpo_amr_new(int ncx, int ncv, double x_len, double v_lo, double v_hi, double qm, int R, int np,
                  int* boxes, double* veq_c, double* veq_f)
{
    vpo_amr* c = (vpo_amr*)calloc(1, sizeof(*c));
    c->ncx = ncx; c->ncv = ncv; c->R = R; c->nfx = ncx * R; c->nfv = ncv * R; c->np = np;
    c->dxc = x_len / ncx; c->dvc = (v_hi - v_lo) / ncv;
    c->dxf = c->dxc / R; c->dvf = c->dvc / R;
    c->v_lo = v_lo; c->qm = qm;
    c->box = (int*)malloc(sizeof(int) * 4 * (np > 0 ? np : 1));
    memcpy(c->box, boxes, sizeof(int) * 4 * np);
    c->off = (long*)malloc(sizeof(long) * (np + 1));
    long o = (long)ncx * ncv;
    for (int p = 0; p < np; ++p) {
        c->off[p] = o;
        o += (long)(boxes[4 * p + 2] - boxes[4 * p] + 1) * (boxes[4 * p + 3] - boxes[4 * p + 1] + 1);
    }
    c->off[np] = o;
    c->total = o;
    c->cov = (unsigned char*)calloc((size_t)ncx * ncv, 1);
    for (int p = 0; p < np; ++p)
        for (int i = boxes[4 * p] / R; i <= boxes[4 * p + 2] / R; ++i)
            for (int j = boxes[4 * p + 1] / R; j <= boxes[4 * p + 3] / R; ++j) c->cov[(size_t)i * ncv + j] = 1;
    c->veq_c = (double*)malloc(sizeof(double) * (ncv + 4));
    memcpy(c->veq_c, veq_c, sizeof(double) * (ncv + 4));
    c->veq_f = (double*)malloc(sizeof(double) * (c->nfv + 4));
    memcpy(c->veq_f, veq_f, sizeof(double) * (c->nfv + 4));
    vpo_interp_weights(R, &c->B[0][0]);
    c->P = vpo_poisson_new(c->nfx);
    return c;
}

void vpo_amr_free(void* h)
{
    vpo_amr* c = (vpo_amr*)h;
    if (!c) return;
    free(c->box); free(c->off); free(c->cov); free(c->veq_c); free(c->veq_f);
    vpo_poisson_free(c->P);
    free(c);
}

long vpo_amr_state_size(void* h) { return ((vpo_amr*)h)->total; }
long vpo_amr_patch_offset(void* h, int p) { vpo_amr* c = (vpo_amr*)h; return p < 0 ? 0 : c->off[p]; }

#define NXP(c, p) ((c)->box[4 * (p) + 2] - (c)->box[4 * (p)] + 1)
#define NVP(c, p) ((c)->box[4 * (p) + 3] - (c)->box[4 * (p) + 1] + 1)

/* coarse value with x periodic and the coarse velocity ghosts */
static double coarse_at(const vpo_amr* c, const double* f, int i, int j)
{
    if (j < 0 || j >= c->ncv) return c->veq_c[j + 2];
    return f[(size_t)wrap(i, c->ncx) * c->ncv + j];
}

/* fine-cell value at global fine indices (I, J) interpolated from the coarse
 * level: first along x, then along v */
static double interp_fine(const vpo_amr* c, const double* f, int I, int J)
{
    if (J < 0 || J >= c->nfv) return c->veq_f[J + 2];
    const int R = c->R;
    int ci = fdiv(I, R), s = I - ci * R;
    int cj = fdiv(J, R), t = J - cj * R;
    double acc = 0.0;
    for (int b = -2; b <= 2; ++b) {
        double gx = 0.0;
        for (int a = -2; a <= 2; ++a) gx += c->B[s][a + 2] * coarse_at(c, f, ci + a, cj + b);
        acc += c->B[t][b + 2] * gx;
    }
    return acc;
}

/* fine cell (I, J) (I periodic) held by a level-1 patch: 1 and its value in
 * *val, else 0 (ghost cells for inter-patch communication, section 3) */
static int same_level_at(const vpo_amr* c, const double* f, int I, int J, double* val)
{
    if (J < 0 || J >= c->nfv) return 0;
    const int Iw = wrap(I, c->nfx);
    for (int p = 0; p < c->np; ++p) {
        const int x0 = c->box[4 * p], v0 = c->box[4 * p + 1];
        if (Iw < x0 || Iw > c->box[4 * p + 2] || J < v0 || J > c->box[4 * p + 3]) continue;
        *val = f[c->off[p] + (size_t)(Iw - x0) * NVP(c, p) + (J - v0)];
        return 1;
    }
    return 0;
}

/* patch p with two ghost layers: (nxp + 4) x (nvp + 4).  A ghost cell that a
 * level-1 patch holds (a touching patch, also across the periodic x
 * boundary, or the patch itself when it spans the whole x range) takes that
 * value (the exchange of ghost cells on a level, Alg. mspsc); the others
 * are interpolated from the coarse level */
void vpo_amr_fill_ghosts(void* h, double* f, int p, double* out)
{
    vpo_amr* c = (vpo_amr*)h;
    int nxp = NXP(c, p), nvp = NVP(c, p), x0 = c->box[4 * p], v0 = c->box[4 * p + 1];
    int W = nvp + 4;
    const double* fp = f + c->off[p];
    for (int r = -2; r < nxp + 2; ++r)
        for (int q = -2; q < nvp + 2; ++q) {
            double v;
            if (r >= 0 && r < nxp && q >= 0 && q < nvp) v = fp[(size_t)r * nvp + q];
            else if (!same_level_at(c, f, x0 + r, v0 + q, &v)) v = interp_fine(c, f, x0 + r, v0 + q);
            out[(size_t)(r + 2) * W + (q + 2)] = v;
        }
}

/* Mask Reduction (section 3): refine coarse data in x, mask covered coarse
 * cells, sum over v; add the fine patches' sums; n on the finest x mesh */
void vpo_amr_reduce_mask(void* h, double* f, double* n)
{
    vpo_amr* c = (vpo_amr*)h;
    const int R = c->R;
    for (int I = 0; I < c->nfx; ++I) {
        int i = I / R, s = I % R;
        double sc = 0.0;
        for (int j = 0; j < c->ncv; ++j) {
            double fx = 0.0;
            for (int a = -2; a <= 2; ++a) fx += c->B[s][a + 2] * coarse_at(c, f, i + a, j);
            if (!c->cov[(size_t)i * c->ncv + j]) sc += fx;
        }
        double sf = 0.0;
        for (int p = 0; p < c->np; ++p) {
            int x0 = c->box[4 * p], x1 = c->box[4 * p + 2];
            if (I < x0 || I > x1) continue;
            int nvp = NVP(c, p);
            const double* row = f + c->off[p] + (size_t)(I - x0) * nvp;
            for (int q = 0; q < nvp; ++q) sf += row[q];
        }
        n[I] = c->dvc * sc + c->dvf * sf;
    }
}

/* a on both levels: [a_c (ncx)][a_f (nfx)]; E on the fine mesh */
void vpo_amr_constraints(void* h, double* f, double* a, double* E_out)
{
    vpo_amr* c = (vpo_amr*)h;
    int nfx = c->nfx, R = c->R;
    double* n = (double*)malloc(sizeof(double) * nfx);
    double* rho = (double*)malloc(sizeof(double) * nfx);
    double* phi = (double*)malloc(sizeof(double) * nfx);
    double* E = (double*)malloc(sizeof(double) * nfx);
    vpo_amr_reduce_mask(h, f, n);
    for (int I = 0; I < nfx; ++I) rho[I] = 1.0 - n[I];
    vpo_poisson_solve(c->P, c->dxf, rho, phi);
    vpo_field(nfx, c->dxf, phi, E);
    for (int i = 0; i < c->ncx; ++i) {
        double s = 0.0;
        for (int q = 0; q < R; ++q) s += E[i * R + q];
        a[i] = c->qm * s / R;
    }
    for (int I = 0; I < nfx; ++I) a[c->ncx + I] = c->qm * E[I];
    if (E_out) memcpy(E_out, E, sizeof(double) * nfx);
    free(n); free(rho); free(phi); free(E);
}

static double face4(double um1, double u0, double u1, double u2)
{
    return (7.0 * (u0 + u1) - (um1 + u2)) / 12.0;
}

/* Fluxes of section 2 on one patch from its ghosted data g ((nx+4) x (nv+4)):
 * Gx[(nx+1) x nv] for x faces -1/2 .. nx-1/2, Gv[nx x (nv+1)] for v faces
 * -1/2 .. nv-1/2.  a_ext[i + 1] = a at patch row i, i = -1 .. nx. */
void vpo_patch_fluxes(int nx, int nv, const double* g, double dv, double v0, const double* a_ext,
                      double* Gx, double* Gv)
{
    int W = nv + 4;
#define G(i, j) g[(size_t)((i) + 2) * W + ((j) + 2)]
    for (int i = -1; i < nx; ++i)           /* face i + 1/2 */
        for (int j = 0; j < nv; ++j) {
            double fc = face4(G(i - 1, j), G(i, j), G(i + 1, j), G(i + 2, j));
            double fu = face4(G(i - 1, j + 1), G(i, j + 1), G(i + 1, j + 1), G(i + 2, j + 1));
            double fd = face4(G(i - 1, j - 1), G(i, j - 1), G(i + 1, j - 1), G(i + 2, j - 1));
            double vb = v0 + (j + 0.5) * dv;
            Gx[(size_t)(i + 1) * nv + j] = vb * fc + dv / 24.0 * (fu - fd);
        }
    for (int i = 0; i < nx; ++i) {
        double ai = a_ext[i + 1], da = a_ext[i + 2] - a_ext[i];
        for (int j = -1; j < nv; ++j) {      /* face j + 1/2 */
            double fc = face4(G(i, j - 1), G(i, j), G(i, j + 1), G(i, j + 2));
            double fp = face4(G(i + 1, j - 1), G(i + 1, j), G(i + 1, j + 1), G(i + 1, j + 2));
            double fm = face4(G(i - 1, j - 1), G(i - 1, j), G(i - 1, j + 1), G(i - 1, j + 2));
            Gv[(size_t)i * (nv + 1) + (j + 1)] = ai * fc + da / 48.0 * (fp - fm);
        }
    }
#undef G
}

/* The same fluxes with the limited face averages of section 2 (eq.
 * limitedFace) in place of every centred one, the neighbouring ones of the
 * product-rule corrections included: an x face is upwinded by the sign of
 * the centre velocity of its column, v_lo + (col0 + j + 1/2) dv with col0
 * the level's global index of local column 0, a v face by the sign of a in
 * its row. */
void vpo_patch_fluxes_limited(int nx, int nv, const double* g, double dv, double v_lo, int col0,
                              const double* a_ext, double* Gx, double* Gv)
{
    int W = nv + 4;
#define G(i, j) g[(size_t)((i) + 2) * W + ((j) + 2)]
#define VC(j) (v_lo + ((double)(col0 + (j)) + 0.5) * dv)
    for (int i = -1; i < nx; ++i)           /* face i + 1/2 */
        for (int j = 0; j < nv; ++j) {
            double fc = vpo_face_limited(G(i - 1, j), G(i, j), G(i + 1, j), G(i + 2, j), VC(j) > 0.0);
            double fu = vpo_face_limited(G(i - 1, j + 1), G(i, j + 1), G(i + 1, j + 1), G(i + 2, j + 1),
                                         VC(j + 1) > 0.0);
            double fd = vpo_face_limited(G(i - 1, j - 1), G(i, j - 1), G(i + 1, j - 1), G(i + 2, j - 1),
                                         VC(j - 1) > 0.0);
            Gx[(size_t)(i + 1) * nv + j] = VC(j) * fc + dv / 24.0 * (fu - fd);
        }
    for (int i = 0; i < nx; ++i) {
        double ai = a_ext[i + 1], da = a_ext[i + 2] - a_ext[i];
        for (int j = -1; j < nv; ++j) {      /* face j + 1/2 */
            double fc = vpo_face_limited(G(i, j - 1), G(i, j), G(i, j + 1), G(i, j + 2), a_ext[i + 1] > 0.0);
            double fp = vpo_face_limited(G(i + 1, j - 1), G(i + 1, j), G(i + 1, j + 1), G(i + 1, j + 2),
                                         a_ext[i + 2] > 0.0);
            double fm = vpo_face_limited(G(i - 1, j - 1), G(i - 1, j), G(i - 1, j + 1), G(i - 1, j + 2),
                                         a_ext[i] > 0.0);
            Gv[(size_t)i * (nv + 1) + (j + 1)] = ai * fc + da / 48.0 * (fp - fm);
        }
    }
#undef VC
#undef G
}

void vpo_amr_set_limited(void* h, int on) { ((vpo_amr*)h)->limited = on != 0; }

/* flux divergence: k_ij = -(Gx_{i+1/2} - Gx_{i-1/2})/dx - (Gv_{j+1/2} - Gv_{j-1/2})/dv */
void vpo_divergence(int nx, int nv, const double* Gx, const double* Gv, double dx, double dv, double* k)
{
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < nv; ++j)
            k[(size_t)i * nv + j] = -(Gx[(size_t)(i + 1) * nv + j] - Gx[(size_t)i * nv + j]) / dx
                                    - (Gv[(size_t)i * (nv + 1) + j + 1] - Gv[(size_t)i * (nv + 1) + j]) / dv;
}

/* all fluxes of the hierarchy for state f and accelerations a */
/* fluxes of the coarse level: one periodic patch with velocity ghosts */
static void coarse_fluxes(const vpo_amr* c, const double* f, const double* a, double* Gx, double* Gv)
{
    int ncx = c->ncx, ncv = c->ncv;
    int W = ncv + 4;
    double* g = (double*)malloc(sizeof(double) * (size_t)(ncx + 4) * W);
    for (int i = -2; i < ncx + 2; ++i)
        for (int j = -2; j < ncv + 2; ++j) g[(size_t)(i + 2) * W + j + 2] = coarse_at(c, f, i, j);
    double* ae = (double*)malloc(sizeof(double) * (ncx + 2));
    for (int i = -1; i <= ncx; ++i) ae[i + 1] = a[wrap(i, ncx)];
    if (c->limited) vpo_patch_fluxes_limited(ncx, ncv, g, c->dvc, c->v_lo, 0, ae, Gx, Gv);
    else vpo_patch_fluxes(ncx, ncv, g, c->dvc, c->v_lo, ae, Gx, Gv);
    free(ae);
    free(g);
}

/* fluxes of level-1 patch p, its ghost cells filled from the coarse part of f */
static void fine_patch_fluxes(const vpo_amr* c, double* f, const double* a, int p, double* Gx, double* Gv)
{
    int nxp = NXP(c, p), nvp = NVP(c, p), x0 = c->box[4 * p], v0 = c->box[4 * p + 1];
    double* g = (double*)malloc(sizeof(double) * (size_t)(nxp + 4) * (nvp + 4));
    vpo_amr_fill_ghosts((void*)c, f, p, g);
    double* ae = (double*)malloc(sizeof(double) * (nxp + 2));
    for (int i = -1; i <= nxp; ++i) ae[i + 1] = a[c->ncx + wrap(x0 + i, c->nfx)];
    if (c->limited) vpo_patch_fluxes_limited(nxp, nvp, g, c->dvf, c->v_lo, v0, ae, Gx, Gv);
    else vpo_patch_fluxes(nxp, nvp, g, c->dvf, c->v_lo + v0 * c->dvf, ae, Gx, Gv);
    free(ae);
    free(g);
}

static void hierarchy_fluxes(const vpo_amr* c, double* f, const double* a, double** Gx, double** Gv)
{
    coarse_fluxes(c, f, a, Gx[0], Gv[0]);
    for (int p = 0; p < c->np; ++p) fine_patch_fluxes(c, f, a, p, Gx[p + 1], Gv[p + 1]);
}

/* k = L(f; a) on every patch of the hierarchy (the ComputeRHS fluxes and
 * divergence of one stage, without accumulation) */
void vpo_amr_rhs(void* h, double* f, double* a, double* k)
{
    vpo_amr* c = (vpo_amr*)h;
    const int np = c->np;
    double **Gx = (double**)malloc(sizeof(double*) * (np + 1)), **Gv = (double**)malloc(sizeof(double*) * (np + 1));
    for (int p = 0; p <= np; ++p) {
        int nx = p == 0 ? c->ncx : NXP(c, p - 1), nv = p == 0 ? c->ncv : NVP(c, p - 1);
        Gx[p] = (double*)malloc(sizeof(double) * (size_t)(nx + 1) * nv);
        Gv[p] = (double*)malloc(sizeof(double) * (size_t)nx * (nv + 1));
    }
    hierarchy_fluxes(c, f, a, Gx, Gv);
    for (int p = 0; p <= np; ++p) {
        int nx = p == 0 ? c->ncx : NXP(c, p - 1), nv = p == 0 ? c->ncv : NVP(c, p - 1);
        double dx = p == 0 ? c->dxc : c->dxf, dv = p == 0 ? c->dvc : c->dvf;
        vpo_divergence(nx, nv, Gx[p], Gv[p], dx, dv, k + (p == 0 ? 0 : c->off[p - 1]));
        free(Gx[p]);
        free(Gv[p]);
    }
    free(Gx);
    free(Gv);
}

/* one synchronous RK4 step of the two-level hierarchy (Alg. smsvphu) */
/* ComputeUpdate of the two-level step from the stage-weighted accumulated
 * fluxes Ax, Av (k: scratch of the state size): the fine levels first
 * (skipped when update_fine is 0: f_out already holds them), then the coarse
 * level with its coarse-fine faces carrying the mean of the fine fluxes,
 * then covered coarse cells take the average of their fine cells */
static void amr_update(const vpo_amr* c, const double* fn, double** Ax, double** Av, double* k, double* f_out,
                       double dt, int update_fine)
{
    const int np = c->np, ncx = c->ncx, ncv = c->ncv, R = c->R;
    /* ComputeUpdate: finest level first */
    for (int p = 1; p <= np && update_fine; ++p) {
        int nx = NXP(c, p - 1), nv = NVP(c, p - 1);
        vpo_divergence(nx, nv, Ax[p], Av[p], c->dxf, c->dvf, k + c->off[p - 1]);
        for (long q = 0; q < (long)nx * nv; ++q) f_out[c->off[p - 1] + q] = fn[c->off[p - 1] + q] + dt * k[c->off[p - 1] + q];
    }
    /* coarsen the fine accumulated fluxes onto the coarse-fine faces */
    for (int p = 0; p < np; ++p) {
        int x0 = c->box[4 * p], v0 = c->box[4 * p + 1], nxp = NXP(c, p), nvp = NVP(c, p);
        int ci0 = x0 / R, ci1 = (x0 + nxp) / R - 1, cj0 = v0 / R, cj1 = (v0 + nvp) / R - 1;
        for (int cj = cj0; cj <= cj1; ++cj) {       /* x faces at ci0 - 1/2 and ci1 + 1/2 */
            double lo = 0.0, hi = 0.0;
            for (int t = 0; t < R; ++t) {
                int J = cj * R + t - v0;
                lo += Ax[p + 1][(size_t)0 * nvp + J];
                hi += Ax[p + 1][(size_t)nxp * nvp + J];
            }
            Ax[0][(size_t)wrap(ci0, ncx) * ncv + cj] = lo / R;              /* face ci0 - 1/2 */
            Ax[0][(size_t)(wrap(ci1, ncx) + 1) * ncv + cj] = hi / R;        /* face ci1 + 1/2 */
        }
        for (int ci = ci0; ci <= ci1; ++ci) {       /* v faces at cj0 - 1/2 and cj1 + 1/2 */
            double lo = 0.0, hi = 0.0;
            for (int s2 = 0; s2 < R; ++s2) {
                int I = ci * R + s2 - x0;
                lo += Av[p + 1][(size_t)I * (nvp + 1) + 0];
                hi += Av[p + 1][(size_t)I * (nvp + 1) + nvp];
            }
            Av[0][(size_t)ci * (ncv + 1) + cj0] = lo / R;
            Av[0][(size_t)ci * (ncv + 1) + cj1 + 1] = hi / R;
        }
    }
    /* periodic x: coarse face 0 - 1/2 and face ncx - 1/2 are the same face */
    for (int j = 0; j < ncv; ++j) {
        double* f0 = &Ax[0][j];
        double* fN = &Ax[0][(size_t)ncx * ncv + j];
        /* one of the two may have been replaced above; keep them equal */
        if (*f0 != *fN) {
            int left_cov = c->cov[(size_t)(ncx - 1) * ncv + j], right_cov = c->cov[j];
            if (left_cov != right_cov) { double v = left_cov ? *fN : *f0; *f0 = v; *fN = v; }
        }
    }
    vpo_divergence(ncx, ncv, Ax[0], Av[0], c->dxc, c->dvc, k);
    for (long q = 0; q < (long)ncx * ncv; ++q) f_out[q] = fn[q] + dt * k[q];
    /* average fine data down onto covered coarse cells */
    for (int p = 0; p < np; ++p) {
        int x0 = c->box[4 * p], v0 = c->box[4 * p + 1], nxp = NXP(c, p), nvp = NVP(c, p);
        for (int ci = x0 / R; ci < (x0 + nxp) / R; ++ci)
            for (int cj = v0 / R; cj < (v0 + nvp) / R; ++cj) {
                double sum = 0.0;
                for (int s2 = 0; s2 < R; ++s2)
                    for (int t = 0; t < R; ++t)
                        sum += f_out[c->off[p] + (size_t)(ci * R + s2 - x0) * nvp + (cj * R + t - v0)];
                f_out[(size_t)ci * ncv + cj] = sum / (R * R);
            }
    }
}

void vpo_amr_rk4_step(void* h, double* f_in, double* f_out, double dt)
{
    static const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    static const double bw[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    vpo_amr* c = (vpo_amr*)h;
    const int np = c->np, ncx = c->ncx, ncv = c->ncv;
    const long N = c->total;
    double* fn = (double*)malloc(sizeof(double) * N);
    double* fs = (double*)malloc(sizeof(double) * N);
    double* k = (double*)calloc(N, sizeof(double));
    double* a = (double*)malloc(sizeof(double) * (ncx + c->nfx));
    memcpy(fn, f_in, sizeof(double) * N);
    double **Gx = (double**)malloc(sizeof(double*) * (np + 1)), **Gv = (double**)malloc(sizeof(double*) * (np + 1));
    double **Ax = (double**)malloc(sizeof(double*) * (np + 1)), **Av = (double**)malloc(sizeof(double*) * (np + 1));
    for (int p = 0; p <= np; ++p) {
        int nx = p == 0 ? ncx : NXP(c, p - 1), nv = p == 0 ? ncv : NVP(c, p - 1);
        Gx[p] = (double*)malloc(sizeof(double) * (size_t)(nx + 1) * nv);
        Gv[p] = (double*)malloc(sizeof(double) * (size_t)nx * (nv + 1));
        Ax[p] = (double*)calloc((size_t)(nx + 1) * nv, sizeof(double));
        Av[p] = (double*)calloc((size_t)nx * (nv + 1), sizeof(double));
    }
    for (int s = 0; s < 4; ++s) {
        /* ComputePredictorState on every level */
        for (long q = 0; q < N; ++q) fs[q] = fn[q] + alpha[s] * dt * k[q];
        /* ComputeInstantaneousConstraints */
        vpo_amr_constraints(h, fs, a, NULL);
        /* ComputeRHS: fluxes, divergence, flux accumulation */
        hierarchy_fluxes(c, fs, a, Gx, Gv);
        for (int p = 0; p <= np; ++p) {
            int nx = p == 0 ? ncx : NXP(c, p - 1), nv = p == 0 ? ncv : NVP(c, p - 1);
            double dx = p == 0 ? c->dxc : c->dxf, dv = p == 0 ? c->dvc : c->dvf;
            vpo_divergence(nx, nv, Gx[p], Gv[p], dx, dv, k + (p == 0 ? 0 : c->off[p - 1]));
            for (size_t q = 0; q < (size_t)(nx + 1) * nv; ++q) Ax[p][q] += bw[s] * Gx[p][q];
            for (size_t q = 0; q < (size_t)nx * (nv + 1); ++q) Av[p][q] += bw[s] * Gv[p][q];
        }
    }
    amr_update(c, fn, Ax, Av, k, f_out, dt, 1);
    for (int p = 0; p <= np; ++p) { free(Gx[p]); free(Gv[p]); free(Ax[p]); free(Av[p]); }
    free(Gx); free(Gv); free(Ax); free(Av);
    free(fn); free(fs); free(k); free(a);
}

/* Several species, each on its own two-level hierarchy, with the same
 * finest configuration mesh (section 1: one phase-space hierarchy per
 * species, the species coupled only through the field).  The constraint:
 * rho = background + sum_s charge_s n_s with n_s the Mask Reduction of
 * species s, the periodic Poisson solve and field on the finest
 * configuration mesh, a_s injected with the species' own q/m (coarse: the
 * mean of the R fine values). */
void vpo_amr_species_constraints(int ns, void* const* hs, double* const* fs, const double* charge,
                                 double background, double* const* a)
{
    const vpo_amr* c0 = (const vpo_amr*)hs[0];
    const int nfx = c0->nfx;
    double* n = (double*)malloc(sizeof(double) * nfx);
    double* rho = (double*)malloc(sizeof(double) * nfx);
    double* phi = (double*)malloc(sizeof(double) * nfx);
    double* E = (double*)malloc(sizeof(double) * nfx);
    for (int I = 0; I < nfx; ++I) rho[I] = background;
    for (int s = 0; s < ns; ++s) {
        vpo_amr_reduce_mask(hs[s], fs[s], n);
        for (int I = 0; I < nfx; ++I) rho[I] += charge[s] * n[I];
    }
    vpo_poisson_solve(c0->P, c0->dxf, rho, phi);
    vpo_field(nfx, c0->dxf, phi, E);
    for (int s = 0; s < ns; ++s) {
        const vpo_amr* c = (const vpo_amr*)hs[s];
        const int R = c->R;
        for (int i = 0; i < c->ncx; ++i) {
            double sum = 0.0;
            for (int q = 0; q < R; ++q) sum += E[i * R + q];
            a[s][i] = c->qm * sum / R;
        }
        for (int I = 0; I < nfx; ++I) a[s][c->ncx + I] = c->qm * E[I];
    }
    free(n); free(rho); free(phi); free(E);
}

/* One synchronous RK4 step of every species' hierarchy (the steps of
 * vpo_amr_rk4_step per species), the field of all species' predictor
 * states at every stage. */
void vpo_amr_species_rk4_step(int ns, void* const* hs, double* const* f_in, double* const* f_out,
                              const double* charge, double background, double dt)
{
    static const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    static const double bw[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    double **fn = (double**)malloc(sizeof(double*) * ns), **fs = (double**)malloc(sizeof(double*) * ns);
    double **k = (double**)malloc(sizeof(double*) * ns), **a = (double**)malloc(sizeof(double*) * ns);
    double ***Gx = (double***)malloc(sizeof(double**) * ns), ***Gv = (double***)malloc(sizeof(double**) * ns);
    double ***Ax = (double***)malloc(sizeof(double**) * ns), ***Av = (double***)malloc(sizeof(double**) * ns);
    for (int s = 0; s < ns; ++s) {
        vpo_amr* c = (vpo_amr*)hs[s];
        const long N = c->total;
        const int np = c->np;
        fn[s] = (double*)malloc(sizeof(double) * N);
        fs[s] = (double*)malloc(sizeof(double) * N);
        k[s] = (double*)calloc(N, sizeof(double));
        a[s] = (double*)malloc(sizeof(double) * (c->ncx + c->nfx));
        memcpy(fn[s], f_in[s], sizeof(double) * N);
        Gx[s] = (double**)malloc(sizeof(double*) * (np + 1));
        Gv[s] = (double**)malloc(sizeof(double*) * (np + 1));
        Ax[s] = (double**)malloc(sizeof(double*) * (np + 1));
        Av[s] = (double**)malloc(sizeof(double*) * (np + 1));
        for (int p = 0; p <= np; ++p) {
            int nx = p == 0 ? c->ncx : NXP(c, p - 1), nv = p == 0 ? c->ncv : NVP(c, p - 1);
            Gx[s][p] = (double*)malloc(sizeof(double) * (size_t)(nx + 1) * nv);
            Gv[s][p] = (double*)malloc(sizeof(double) * (size_t)nx * (nv + 1));
            Ax[s][p] = (double*)calloc((size_t)(nx + 1) * nv, sizeof(double));
            Av[s][p] = (double*)calloc((size_t)nx * (nv + 1), sizeof(double));
        }
    }
    for (int st = 0; st < 4; ++st) {
        for (int s = 0; s < ns; ++s) {
            const long N = ((vpo_amr*)hs[s])->total;
            for (long q = 0; q < N; ++q) fs[s][q] = fn[s][q] + alpha[st] * dt * k[s][q];
        }
        vpo_amr_species_constraints(ns, hs, fs, charge, background, a);
        for (int s = 0; s < ns; ++s) {
            vpo_amr* c = (vpo_amr*)hs[s];
            hierarchy_fluxes(c, fs[s], a[s], Gx[s], Gv[s]);
            for (int p = 0; p <= c->np; ++p) {
                int nx = p == 0 ? c->ncx : NXP(c, p - 1), nv = p == 0 ? c->ncv : NVP(c, p - 1);
                double dx = p == 0 ? c->dxc : c->dxf, dv = p == 0 ? c->dvc : c->dvf;
                vpo_divergence(nx, nv, Gx[s][p], Gv[s][p], dx, dv, k[s] + (p == 0 ? 0 : c->off[p - 1]));
                for (size_t q = 0; q < (size_t)(nx + 1) * nv; ++q) Ax[s][p][q] += bw[st] * Gx[s][p][q];
                for (size_t q = 0; q < (size_t)nx * (nv + 1); ++q) Av[s][p][q] += bw[st] * Gv[s][p][q];
            }
        }
    }
    for (int s = 0; s < ns; ++s) {
        vpo_amr* c = (vpo_amr*)hs[s];
        amr_update(c, fn[s], Ax[s], Av[s], k[s], f_out[s], dt, 1);
        for (int p = 0; p <= c->np; ++p) { free(Gx[s][p]); free(Gv[s][p]); free(Ax[s][p]); free(Av[s][p]); }
        free(Gx[s]); free(Gv[s]); free(Ax[s]); free(Av[s]);
        free(fn[s]); free(fs[s]); free(k[s]); free(a[s]);
    }
    free(Gx); free(Gv); free(Ax); free(Av); free(fn); free(fs); free(k); free(a);
}

/* ------------------------------------------------------------------------
 * Subcycled two-level step (the asynchronous time stepping that section 5
 * names as future work).  Reading, stated in full because the paper gives
 * no algorithm for it:
 *   1. the coarse level takes one RK4 step of dt on its own, with the field
 *      of its own velocity moment on the coarse configuration mesh (covered
 *      coarse cells hold the mean of their fine cells), keeping its four
 *      stage slopes K1..K4 and its stage-weighted fluxes;
 *   2. the fine patches take R RK4 substeps of dt/R.  The coarse level in
 *      time is the continuous extension of the coarse RK4 step,
 *      P(theta) = f_c^n + dt sum_q b_q(theta) K_q with b_1 = theta -
 *      3 theta^2/2 + 2 theta^3/3, b_2 = b_3 = theta^2 - 2 theta^3/3,
 *      b_4 = -theta^2/2 + 2 theta^3/3 (the third-order dense output of the
 *      classical scheme).  For the four stages of the substep starting at
 *      theta0 = m/R, with eta = 1/R and P1, P2, P3 the first three
 *      theta-derivatives of P at theta0, the coarse data are the values the
 *      RK4 stages take on the Taylor expansion of P (the construction of
 *      McCorquodale and Colella for high-order subcycling):
 *        P,  P + eta/2 P1,  P + eta/2 P1 + eta^2/4 P2,
 *        P + eta P1 + eta^2/2 P2 + eta^3/4 P3
 *      (on y' = lambda y these are the RK4 stage values of a step of eta
 *      started from P); the fine ghost cells come from these coarse data by
 *      the sub-cell interpolation, and the field from the composite moment
 *      of them and the fine predictor (the synchronous constraint);
 *   3. the coarse update takes, on every coarse-fine face, the mean over
 *      the R fine faces of the fine fluxes averaged over the substeps
 *      (stage-weighted), then covered coarse cells take the mean of their
 *      fine cells.
 * ------------------------------------------------------------------------ */

/* field of the coarse level alone: velocity moment of the coarse cells, the
 * periodic Poisson solve and field on the ncx-cell configuration mesh */
static void coarse_level_field(const vpo_amr* c, const vpo_poisson* Pc, const double* fc, double* ac)
{
    const int ncx = c->ncx;
    double* n = (double*)malloc(sizeof(double) * ncx);
    double* phi = (double*)malloc(sizeof(double) * ncx);
    double* E = (double*)malloc(sizeof(double) * ncx);
    vpo_moment(ncx, c->ncv, c->dvc, fc, n);
    for (int i = 0; i < ncx; ++i) n[i] = 1.0 - n[i];      /* rho = 1 - n */
    vpo_poisson_solve(Pc, c->dxc, n, phi);
    vpo_field(ncx, c->dxc, phi, E);
    for (int i = 0; i < ncx; ++i) ac[i] = c->qm * E[i];
    free(n); free(phi); free(E);
}

/* weights of the continuous extension of the classical RK4 step */
void vpo_rk4_dense_weights(double theta, double* b)
{
    const double t2 = theta * theta, t3 = t2 * theta;
    b[0] = theta - 1.5 * t2 + 2.0 * t3 / 3.0;
    b[1] = t2 - 2.0 * t3 / 3.0;
    b[2] = b[1];
    b[3] = -0.5 * t2 + 2.0 * t3 / 3.0;
}

/* weights w_q of the coarse data of fine stage s (0..3) of the substep that
 * starts at theta0 with length eta (in units of the coarse step):
 * f_c = f_c^n + dt sum_q w_q K_q */
void vpo_rk4_substage_weights(double theta0, double eta, int s, double* w)
{
    const double t = theta0, t2 = t * t;
    const double d0[4] = {t - 1.5 * t2 + 2.0 * t2 * t / 3.0, t2 - 2.0 * t2 * t / 3.0, t2 - 2.0 * t2 * t / 3.0,
                          -0.5 * t2 + 2.0 * t2 * t / 3.0};
    const double d1[4] = {1.0 - 3.0 * t + 2.0 * t2, 2.0 * t - 2.0 * t2, 2.0 * t - 2.0 * t2, -t + 2.0 * t2};
    const double d2[4] = {-3.0 + 4.0 * t, 2.0 - 4.0 * t, 2.0 - 4.0 * t, -1.0 + 4.0 * t};
    const double d3[4] = {4.0, -4.0, -4.0, 4.0};
    static const double c1[4] = {0.0, 0.5, 0.5, 1.0}, c2[4] = {0.0, 0.0, 0.25, 0.5}, c3[4] = {0.0, 0.0, 0.0, 0.25};
    for (int q = 0; q < 4; ++q)
        w[q] = d0[q] + c1[s] * eta * d1[q] + c2[s] * eta * eta * d2[q] + c3[s] * eta * eta * eta * d3[q];
}

void vpo_amr_subcycle_step(void* h, double* f_in, double* f_out, double dt)
{
    static const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    static const double bw[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    vpo_amr* c = (vpo_amr*)h;
    const int np = c->np, ncx = c->ncx, ncv = c->ncv, R = c->R;
    const long Nc = (long)ncx * ncv, N = c->total;
    const double hs = dt / R;
    double* K[4];
    for (int s = 0; s < 4; ++s) K[s] = (double*)malloc(sizeof(double) * Nc);
    double* fs = (double*)malloc(sizeof(double) * N);
    double* kf = (double*)calloc(N, sizeof(double));
    double* a = (double*)malloc(sizeof(double) * (ncx + c->nfx));
    double **Gx = (double**)malloc(sizeof(double*) * (np + 1)), **Gv = (double**)malloc(sizeof(double*) * (np + 1));
    double **Ax = (double**)malloc(sizeof(double*) * (np + 1)), **Av = (double**)malloc(sizeof(double*) * (np + 1));
    double **Sx = (double**)malloc(sizeof(double*) * (np + 1)), **Sv = (double**)malloc(sizeof(double*) * (np + 1));
    for (int p = 0; p <= np; ++p) {
        int nx = p == 0 ? ncx : NXP(c, p - 1), nv = p == 0 ? ncv : NVP(c, p - 1);
        Gx[p] = (double*)malloc(sizeof(double) * (size_t)(nx + 1) * nv);
        Gv[p] = (double*)malloc(sizeof(double) * (size_t)nx * (nv + 1));
        Ax[p] = (double*)calloc((size_t)(nx + 1) * nv, sizeof(double));
        Av[p] = (double*)calloc((size_t)nx * (nv + 1), sizeof(double));
        Sx[p] = (double*)calloc((size_t)(nx + 1) * nv, sizeof(double));
        Sv[p] = (double*)calloc((size_t)nx * (nv + 1), sizeof(double));
    }
    vpo_poisson* Pc = vpo_poisson_new(ncx);

    /* 1. the coarse level: one RK4 step of dt with its own field */
    for (int s = 0; s < 4; ++s) {
        for (long q = 0; q < Nc; ++q) fs[q] = f_in[q] + (s > 0 ? alpha[s] * dt * K[s - 1][q] : 0.0);
        coarse_level_field(c, Pc, fs, a);
        coarse_fluxes(c, fs, a, Gx[0], Gv[0]);
        vpo_divergence(ncx, ncv, Gx[0], Gv[0], c->dxc, c->dvc, K[s]);
        for (size_t q = 0; q < (size_t)(ncx + 1) * ncv; ++q) Ax[0][q] += bw[s] * Gx[0][q];
        for (size_t q = 0; q < (size_t)ncx * (ncv + 1); ++q) Av[0][q] += bw[s] * Gv[0][q];
    }

    /* 2. the fine patches: R substeps of dt / R; f_out holds the fine state */
    memcpy(f_out, f_in, sizeof(double) * N);
    for (int m = 0; m < R; ++m) {
        for (int p = 1; p <= np; ++p) {
            int nx = NXP(c, p - 1), nv = NVP(c, p - 1);
            memset(Sx[p], 0, sizeof(double) * (size_t)(nx + 1) * nv);
            memset(Sv[p], 0, sizeof(double) * (size_t)nx * (nv + 1));
        }
        for (int s = 0; s < 4; ++s) {
            double b[4];
            vpo_rk4_substage_weights((double)m / R, 1.0 / R, s, b);
            for (long q = 0; q < Nc; ++q)
                fs[q] = f_in[q] + dt * (b[0] * K[0][q] + b[1] * K[1][q] + b[2] * K[2][q] + b[3] * K[3][q]);
            for (long q = Nc; q < N; ++q) fs[q] = f_out[q] + alpha[s] * hs * kf[q];
            vpo_amr_constraints(h, fs, a, NULL);
            for (int p = 1; p <= np; ++p) {
                int nx = NXP(c, p - 1), nv = NVP(c, p - 1);
                fine_patch_fluxes(c, fs, a, p - 1, Gx[p], Gv[p]);
                vpo_divergence(nx, nv, Gx[p], Gv[p], c->dxf, c->dvf, kf + c->off[p - 1]);
                for (size_t q = 0; q < (size_t)(nx + 1) * nv; ++q) Sx[p][q] += bw[s] * Gx[p][q];
                for (size_t q = 0; q < (size_t)nx * (nv + 1); ++q) Sv[p][q] += bw[s] * Gv[p][q];
            }
        }
        for (int p = 1; p <= np; ++p) {
            int nx = NXP(c, p - 1), nv = NVP(c, p - 1);
            double* kp = kf + c->off[p - 1];
            vpo_divergence(nx, nv, Sx[p], Sv[p], c->dxf, c->dvf, kp);
            for (long q = 0; q < (long)nx * nv; ++q) f_out[c->off[p - 1] + q] += hs * kp[q];
            for (size_t q = 0; q < (size_t)(nx + 1) * nv; ++q) Ax[p][q] += Sx[p][q] / R;
            for (size_t q = 0; q < (size_t)nx * (nv + 1); ++q) Av[p][q] += Sv[p][q] / R;
        }
    }

    /* 3. the coarse update with the time-averaged fine fluxes on the
     * coarse-fine faces, then the average-down */
    amr_update(c, f_in, Ax, Av, kf, f_out, dt, 0);

    vpo_poisson_free(Pc);
    for (int p = 0; p <= np; ++p) { free(Gx[p]); free(Gv[p]); free(Ax[p]); free(Av[p]); free(Sx[p]); free(Sv[p]); }
    free(Gx); free(Gv); free(Ax); free(Av); free(Sx); free(Sv);
    for (int s = 0; s < 4; ++s) free(K[s]);
    free(fs); free(kf); free(a);
}
