/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 implementation of the 1D+1V Vlasov-Poisson
 * discretisation of Hittinger & Banks, "Block-Structured Adaptive Mesh
 * Refinement Algorithms for Vlasov Simulation", section 2.  It exists to
 * check the GPU library; only the tests, the smoke check and the CPU
 * baseline of the benchmark load it.  It shares no code with the GPU
 * path.  Every loop is written in the order of the definitions in the
 * paper, with no blocking or fusion.
 *
 * Readings of the paper taken here (each pinned by a test):
 *   - E = -d(phi)/dx, so the cell-averaged field is minus the printed
 *     fourth-order difference of phi (section 2, Poisson equation and
 *     the E stencil; the sign is fixed by the Vlasov equation in flux
 *     form and by the Poisson right-hand side).
 *   - The discrete Poisson right-hand side is 12 dx^2 rho (section 2,
 *     discrete potential equation; the printed 12 dx is a typo, the
 *     fourth-order finite-volume Laplacian carries dx^2).
 *   - The (q/m) E f product-rule correction enters with a plus sign
 *     (section 2, face-averaged fluxes; the product rule for averages of
 *     a product of two linear functions gives +).
 *   - The unlimited (ideal-weight) face average is the centred
 *     fourth-order formula (section 2, limited face average with
 *     w_L = w_R = 1/2).
 *   - Velocity ghost cells hold the exact cell averages of the
 *     unperturbed equilibrium (section 2, characteristic boundary
 *     condition; the incoming values are the equilibrium, outgoing
 *     values are replaced by the same equilibrium).
 *   - rho_i = 1 - dv sum_j f_ij over the interior velocity cells.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vp_oracle.h"

static int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

/* ------------------------------------------------------------------ */
/* Velocity moment (section 2: rho_i = 1 - dv sum_j f_ij).            */
/* ------------------------------------------------------------------ */
void vpo_moment(int nx, int nv, double dv, const double* f, double* n)
{
    for (int i = 0; i < nx; ++i) {
        double s = 0.0;
        for (int j = 0; j < nv; ++j) s += f[(size_t)i * nv + j];
        n[i] = dv * s;
    }
}

/* ------------------------------------------------------------------ */
/* Periodic fourth-order Poisson problem (section 2, discrete          */
/* potential equation):                                                */
/*   30 phi_i - 16 (phi_{i+1} + phi_{i-1}) + (phi_{i+2} + phi_{i-2})   */
/*     = 12 dx^2 rho_i .                                               */
/* The periodic matrix A is singular (constants); the null space is    */
/* handled by the bordered system                                      */
/*   [ A   1 ] [phi]   [12 dx^2 rho]                                   */
/*   [ 1^T 0 ] [lam] = [     0     ]                                   */
/* whose solution has sum(phi) = 0 and lam = -mean(12 dx^2 rho), i.e.   */
/* rho is projected onto zero mean.  As the paper describes, the        */
/* matrix is LU-factored once and the factors are reused for every      */
/* solve.  The unknowns are ordered phi_0..phi_{N-3} (a pentadiagonal  */
/* block B, symmetric positive definite) followed by phi_{N-2},        */
/* phi_{N-1}, lam; block elimination of B leaves a 3x3 Schur complement */
/* that is factored with partial pivoting.                              */
/* ------------------------------------------------------------------ */
static double A_entry(int N, int i, int j)
{
    static const double c[5] = {1.0, -16.0, 30.0, -16.0, 1.0};   /* offsets -2..2 */
    double s = 0.0;
    for (int o = -2; o <= 2; ++o)
        if (wrap(i + o, N) == j) s += c[o + 2];
    return s;
}

struct vpo_poisson {
    int N;
    int nb;            /* size of the banded block B = N - 2 (or 0)  */
    double* band;      /* nb x 5: LU factors of B, columns -2..+2     */
    double* Z;         /* nb x 3: B^{-1} C                            */
    double S[3][3];    /* Schur complement D - R Z, LU in place        */
    int piv[3];
};

/* band storage: element (i, i+o) for o in [-2, 2] at band[i*5 + o + 2] */
static void band_solve(const struct vpo_poisson* P, double* x)
{
    int n = P->nb;
    const double* b = P->band;
    /* forward: L has unit diagonal, sub-diagonals at o = -1, -2 */
    for (int i = 0; i < n; ++i) {
        double s = x[i];
        for (int o = -2; o <= -1; ++o)
            if (i + o >= 0) s -= b[i * 5 + o + 2] * x[i + o];
        x[i] = s;
    }
    /* backward: U has diagonal o = 0 and super-diagonals o = 1, 2 */
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int o = 1; o <= 2; ++o)
            if (i + o < n) s -= b[i * 5 + o + 2] * x[i + o];
        x[i] = s / b[i * 5 + 2];
    }
}

vpo_poisson* vpo_poisson_new(int N)
{
    vpo_poisson* P = (vpo_poisson*)calloc(1, sizeof(*P));
    P->N = N;
    if (N < 2) return P;        /* N == 1: phi = 0 */
    int nb = N - 2;
    P->nb = nb;
    P->band = (double*)calloc((size_t)(nb > 0 ? nb : 1) * 5, sizeof(double));
    P->Z = (double*)calloc((size_t)(nb > 0 ? nb : 1) * 3, sizeof(double));
    for (int i = 0; i < nb; ++i)
        for (int o = -2; o <= 2; ++o)
            if (i + o >= 0 && i + o < nb) P->band[i * 5 + o + 2] = A_entry(N, i, i + o);
    /* Doolittle LU of the band, no pivoting (B is SPD). */
    for (int k = 0; k < nb; ++k) {
        double piv = P->band[k * 5 + 2];
        for (int i = k + 1; i <= k + 2 && i < nb; ++i) {
            double l = P->band[i * 5 + (k - i) + 2] / piv;
            P->band[i * 5 + (k - i) + 2] = l;
            for (int j = k + 1; j <= k + 2 && j < nb; ++j)
                P->band[i * 5 + (j - i) + 2] -= l * P->band[k * 5 + (j - k) + 2];
        }
    }
    /* Z = B^{-1} C, C = columns phi_{N-2}, phi_{N-1}, lam of rows 0..nb-1 */
    double* col = (double*)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
    for (int c = 0; c < 3; ++c) {
        for (int i = 0; i < nb; ++i)
            col[i] = (c < 2) ? A_entry(N, i, N - 2 + c) : 1.0;
        if (nb > 0) band_solve(P, col);
        for (int i = 0; i < nb; ++i) P->Z[i * 3 + c] = col[i];
    }
    free(col);
    /* S = D - R Z */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double d;
            if (r < 2 && c < 2) d = A_entry(N, N - 2 + r, N - 2 + c);
            else if (r == 2 && c == 2) d = 0.0;
            else d = 1.0;
            double s = 0.0;
            for (int i = 0; i < nb; ++i) {
                double rr = (r < 2) ? A_entry(N, N - 2 + r, i) : 1.0;
                s += rr * P->Z[i * 3 + c];
            }
            P->S[r][c] = d - s;
        }
    /* LU with partial pivoting of the 3x3 S */
    for (int k = 0; k < 3; ++k) {
        int p = k;
        for (int i = k + 1; i < 3; ++i)
            if (fabs(P->S[i][k]) > fabs(P->S[p][k])) p = i;
        P->piv[k] = p;
        if (p != k)
            for (int c = 0; c < 3; ++c) { double t = P->S[k][c]; P->S[k][c] = P->S[p][c]; P->S[p][c] = t; }
        for (int i = k + 1; i < 3; ++i) {
            P->S[i][k] /= P->S[k][k];
            for (int c = k + 1; c < 3; ++c) P->S[i][c] -= P->S[i][k] * P->S[k][c];
        }
    }
    return P;
}

void vpo_poisson_free(vpo_poisson* P)
{
    if (!P) return;
    free(P->band);
    free(P->Z);
    free(P);
}

/* One solve of the bordered system with the stored factors: right-hand
 * side b (N values) and constraint value c; returns phi and lam. */
static void bordered_solve(const vpo_poisson* P, const double* b, double c, double* phi, double* lam)
{
    int N = P->N;
    int nb = P->nb;
    double* y = (double*)malloc(sizeof(double) * (size_t)(nb > 0 ? nb : 1));
    for (int i = 0; i < nb; ++i) y[i] = b[i];
    if (nb > 0) band_solve(P, y);
    double q[3] = {b[N - 2], b[N - 1], c};
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int i = 0; i < nb; ++i) {
            double rr = (r < 2) ? A_entry(N, N - 2 + r, i) : 1.0;
            s += rr * y[i];
        }
        q[r] -= s;
    }
    /* solve S w = q: the factorisation swapped whole rows, so apply every
     * interchange to q first, then the unit-lower and upper solves */
    for (int k = 0; k < 3; ++k) {
        int p = P->piv[k];
        if (p != k) { double t = q[k]; q[k] = q[p]; q[p] = t; }
    }
    for (int k = 0; k < 3; ++k)
        for (int i = k + 1; i < 3; ++i) q[i] -= P->S[i][k] * q[k];
    for (int k = 2; k >= 0; --k) {
        double s = q[k];
        for (int cc = k + 1; cc < 3; ++cc) s -= P->S[k][cc] * q[cc];
        q[k] = s / P->S[k][k];
    }
    for (int i = 0; i < nb; ++i)
        phi[i] = y[i] - (P->Z[i * 3 + 0] * q[0] + P->Z[i * 3 + 1] * q[1] + P->Z[i * 3 + 2] * q[2]);
    phi[N - 2] = q[0];
    phi[N - 1] = q[1];
    *lam = q[2];
    free(y);
}

/* phi solves A phi = 12 dx^2 (rho - mean rho) with sum(phi) = 0.
 * The system is the exact definition of phi; its condition number grows
 * like N^2, so the rounding of one LU solve grows with the mesh.  Two
 * steps of iterative refinement (residual of the bordered system in
 * extended precision, correction from the same factors) bring phi to
 * rounding of the exact solution. */
void vpo_poisson_solve(const vpo_poisson* P, double dx, const double* rho, double* phi)
{
    int N = P->N;
    if (N < 2) { if (N == 1) phi[0] = 0.0; return; }
    double* b = (double*)malloc(sizeof(double) * (size_t)N);
    double* r = (double*)malloc(sizeof(double) * (size_t)N);
    double* dphi = (double*)malloc(sizeof(double) * (size_t)N);
    for (int i = 0; i < N; ++i) b[i] = 12.0 * dx * dx * rho[i];
    double lam = 0.0, dlam = 0.0;
    bordered_solve(P, b, 0.0, phi, &lam);
    static const long double c[5] = {1.0L, -16.0L, 30.0L, -16.0L, 1.0L};   /* offsets -2..2 */
    for (int it = 0; it < 2; ++it) {
        long double sphi = 0.0L;
        for (int i = 0; i < N; ++i) {
            long double ap = 0.0L;
            for (int o = -2; o <= 2; ++o) ap += c[o + 2] * (long double)phi[wrap(i + o, N)];
            r[i] = (double)((long double)b[i] - ap - (long double)lam);
            sphi += (long double)phi[i];
        }
        bordered_solve(P, r, (double)(-sphi), dphi, &dlam);
        for (int i = 0; i < N; ++i) phi[i] += dphi[i];
        lam += dlam;
    }
    free(b); free(r); free(dphi);
}

/* E_i = -[8 (phi_{i+1} - phi_{i-1}) - (phi_{i+2} - phi_{i-2})] / (12 dx) */
void vpo_field(int nx, double dx, const double* phi, double* E)
{
    for (int i = 0; i < nx; ++i) {
        double d1 = phi[wrap(i + 1, nx)] - phi[wrap(i - 1, nx)];
        double d2 = phi[wrap(i + 2, nx)] - phi[wrap(i - 2, nx)];
        E[i] = -(8.0 * d1 - d2) / (12.0 * dx);
    }
}

/* ------------------------------------------------------------------ */
/* Right-hand side of the semi-discrete system (section 2):            */
/*   k_ij = -(Gx_{i+1/2,j} - Gx_{i-1/2,j})/dx - (Gv_{i,j+1/2} - Gv_{i,j-1/2})/dv */
/* with the fourth-order face-averaged fluxes                          */
/*   Gx = vbar_j <f>_{i+1/2,j} + dv/24 (<f>_{i+1/2,j+1} - <f>_{i+1/2,j-1}) */
/*   Gv = a_i <f>_{i,j+1/2} + 1/48 (a_{i+1} - a_{i-1})                 */
/*                          (<f>_{i+1,j+1/2} - <f>_{i-1,j+1/2})         */
/* where a = (q/m) E, and the face averages use the ideal weights:     */
/*   <f>_{i+1/2} = (7 (f_i + f_{i+1}) - (f_{i-1} + f_{i+2})) / 12.     */
/* x is periodic; velocity ghosts are the equilibrium cell averages.    */
/* ------------------------------------------------------------------ */
#define GH 2   /* ghost layers reached by the stencil */

static double* ghosted(int nx, int nv, const double* vghost, const double* f)
{
    int W = nv + 2 * GH;
    double* g = (double*)malloc(sizeof(double) * (size_t)(nx + 2 * GH) * W);
    for (int i = -GH; i < nx + GH; ++i) {
        const double* src = f + (size_t)wrap(i, nx) * nv;
        double* dst = g + (size_t)(i + GH) * W;
        dst[0] = vghost[0];                  /* j = -2 */
        dst[1] = vghost[1];                  /* j = -1 */
        for (int j = 0; j < nv; ++j) dst[j + GH] = src[j];
        dst[nv + GH] = vghost[2];            /* j = nv */
        dst[nv + GH + 1] = vghost[3];        /* j = nv + 1 */
    }
    return g;
}

static double face4(double um1, double u0, double u1, double u2)
{
    return (7.0 * (u0 + u1) - (um1 + u2)) / 12.0;
}

void vpo_rhs(int nx, int nv, double dx, double dv, double v_lo,
             const double* vghost, const double* f, const double* a, double* k)
{
    int W = nv + 2 * GH;
    double* g = ghosted(nx, nv, vghost, f);
#define G(i, j) g[(size_t)((i) + GH) * W + ((j) + GH)]
    /* Fx[i][j]: face i+1/2 for i = -1..nx-1, j = -1..nv (stored at [i+1][j+1]) */
    int FxW = nv + 2;
    double* Fx = (double*)malloc(sizeof(double) * (size_t)(nx + 1) * FxW);
    /* Fv[i][j]: face j+1/2 for j = -1..nv-1, i = -1..nx (stored at [i+1][j+1]) */
    int FvW = nv + 1;
    double* Fv = (double*)malloc(sizeof(double) * (size_t)(nx + 2) * FvW);
    #pragma omp parallel for schedule(static)
    for (int i = -1; i < nx; ++i)
        for (int j = -1; j <= nv; ++j)
            Fx[(size_t)(i + 1) * FxW + (j + 1)] = face4(G(i - 1, j), G(i, j), G(i + 1, j), G(i + 2, j));
    #pragma omp parallel for schedule(static)
    for (int i = -1; i <= nx; ++i)
        for (int j = -1; j < nv; ++j)
            Fv[(size_t)(i + 1) * FvW + (j + 1)] = face4(G(i, j - 1), G(i, j), G(i, j + 1), G(i, j + 2));
#define FX(i, j) Fx[(size_t)((i) + 1) * FxW + ((j) + 1)]
#define FV(i, j) Fv[(size_t)((i) + 1) * FvW + ((j) + 1)]
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i) {
        double ai = a[i];
        double da = a[wrap(i + 1, nx)] - a[wrap(i - 1, nx)];
        for (int j = 0; j < nv; ++j) {
            double vb = v_lo + (j + 0.5) * dv;
            double gxr = vb * FX(i, j) + dv / 24.0 * (FX(i, j + 1) - FX(i, j - 1));
            double gxl = vb * FX(i - 1, j) + dv / 24.0 * (FX(i - 1, j + 1) - FX(i - 1, j - 1));
            double gvt = ai * FV(i, j) + da / 48.0 * (FV(i + 1, j) - FV(i - 1, j));
            double gvb = ai * FV(i, j - 1) + da / 48.0 * (FV(i + 1, j - 1) - FV(i - 1, j - 1));
            k[(size_t)i * nv + j] = -(gxr - gxl) / dx - (gvt - gvb) / dv;
        }
    }
#undef G
#undef FX
#undef FV
    free(Fv);
    free(Fx);
    free(g);
}

/* Fluxes through the two velocity-boundary faces (j = -1/2 and nv-1/2) of
 * every x-cell, the only terms by which mass can change:
 * sum_ij k_ij dx dv = -dx sum_i (Gv_{i,nv-1/2} - Gv_{i,-1/2}). */
void vpo_vboundary_flux(int nx, int nv, double dx, double dv,
                        const double* vghost, const double* f, const double* a,
                        double* g_lo, double* g_hi)
{
    (void)dx;
    double* g = ghosted(nx, nv, vghost, f);
    int W = nv + 2 * GH;
#define G(i, j) g[(size_t)((i) + GH) * W + ((j) + GH)]
    for (int i = 0; i < nx; ++i) {
        double ai = a[i];
        double da = a[wrap(i + 1, nx)] - a[wrap(i - 1, nx)];
        for (int side = 0; side < 2; ++side) {
            int j = side == 0 ? -1 : nv - 1;           /* face j + 1/2 */
            double fc = face4(G(i, j - 1), G(i, j), G(i, j + 1), G(i, j + 2));
            double fp = face4(G(i + 1, j - 1), G(i + 1, j), G(i + 1, j + 1), G(i + 1, j + 2));
            double fm = face4(G(i - 1, j - 1), G(i - 1, j), G(i - 1, j + 1), G(i - 1, j + 2));
            double gv = ai * fc + da / 48.0 * (fp - fm);
            if (side == 0) g_lo[i] = gv; else g_hi[i] = gv;
        }
    }
#undef G
    free(g);
}

/* ------------------------------------------------------------------ */
/* Instantaneous constraint and RK4 step.                              */
/* ------------------------------------------------------------------ */
vpo_ctx* vpo_ctx_new(int nx, int nv, double x_len, double v_lo, double v_hi,
                     double qm, const double* vghost)
{
    vpo_ctx* c = (vpo_ctx*)calloc(1, sizeof(*c));
    c->nx = nx; c->nv = nv;
    c->dx = x_len / nx;
    c->dv = (v_hi - v_lo) / nv;
    c->v_lo = v_lo;
    c->qm = qm;
    memcpy(c->vghost, vghost, sizeof(c->vghost));
    c->P = vpo_poisson_new(nx);
    return c;
}

void vpo_ctx_free(vpo_ctx* c)
{
    if (!c) return;
    vpo_poisson_free(c->P);
    free(c);
}

/* Reduction -> Poisson -> field -> injection: a = (q/m) E(f).
 * Any of n, phi, E may be NULL. */
void vpo_constraints(const vpo_ctx* c, const double* f, double* a,
                     double* n_out, double* phi_out, double* E_out)
{
    int nx = c->nx;
    double* n = (double*)malloc(sizeof(double) * nx);
    double* rho = (double*)malloc(sizeof(double) * nx);
    double* phi = (double*)malloc(sizeof(double) * nx);
    double* E = (double*)malloc(sizeof(double) * nx);
    vpo_moment(nx, c->nv, c->dv, f, n);
    for (int i = 0; i < nx; ++i) rho[i] = 1.0 - n[i];
    vpo_poisson_solve(c->P, c->dx, rho, phi);
    vpo_field(nx, c->dx, phi, E);
    for (int i = 0; i < nx; ++i) a[i] = c->qm * E[i];
    if (n_out) memcpy(n_out, n, sizeof(double) * nx);
    if (phi_out) memcpy(phi_out, phi, sizeof(double) * nx);
    if (E_out) memcpy(E_out, E, sizeof(double) * nx);
    free(n); free(rho); free(phi); free(E);
}

/* Classic RK4 (section 2, eq. rk4), alpha = [0, 1/2, 1/2, 1],
 * b = [1/6, 1/3, 1/3, 1/6]; the field is re-solved for every predictor
 * state (the instantaneous constraint).  The operator is autonomous, so
 * the stage times c_s are not needed.  f_out may alias f_in.
 * If stage_f / stage_a are non-NULL they receive the four predictor
 * states (4 * nx * nv) and their accelerations (4 * nx). */
void vpo_rk4_step_stages(const vpo_ctx* c, const double* f_in, double* f_out, double dt,
                         double* stage_f, double* stage_a)
{
    static const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    static const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    size_t N = (size_t)c->nx * c->nv;
    double* fn = (double*)malloc(sizeof(double) * N);
    double* fs = (double*)malloc(sizeof(double) * N);
    double* ks = (double*)malloc(sizeof(double) * N * 4);
    double* a = (double*)malloc(sizeof(double) * c->nx);
    memcpy(fn, f_in, sizeof(double) * N);
    for (int s = 0; s < 4; ++s) {
        for (size_t p = 0; p < N; ++p)
            fs[p] = s == 0 ? fn[p] : fn[p] + alpha[s] * dt * ks[(size_t)(s - 1) * N + p];
        vpo_constraints(c, fs, a, NULL, NULL, NULL);
        if (stage_f) memcpy(stage_f + (size_t)s * N, fs, sizeof(double) * N);
        if (stage_a) memcpy(stage_a + (size_t)s * c->nx, a, sizeof(double) * c->nx);
        vpo_rhs(c->nx, c->nv, c->dx, c->dv, c->v_lo, c->vghost, fs, a, ks + (size_t)s * N);
    }
    for (size_t p = 0; p < N; ++p) {
        double sum = 0.0;
        for (int s = 0; s < 4; ++s) sum += b[s] * ks[(size_t)s * N + p];
        f_out[p] = fn[p] + dt * sum;
    }
    free(fn); free(fs); free(ks); free(a);
}

void vpo_rk4_step(const vpo_ctx* c, const double* f_in, double* f_out, double dt)
{
    vpo_rk4_step_stages(c, f_in, f_out, dt, NULL, NULL);
}

/* RK4 with a prescribed, time-independent acceleration a (no field solve);
 * used for free streaming (a = 0) and static-field convergence tests. */
void vpo_rk4_step_fixed_a(const vpo_ctx* c, const double* f_in, double* f_out,
                          const double* a, double dt)
{
    static const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    static const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    size_t N = (size_t)c->nx * c->nv;
    double* fn = (double*)malloc(sizeof(double) * N);
    double* fs = (double*)malloc(sizeof(double) * N);
    double* ks = (double*)malloc(sizeof(double) * N * 4);
    memcpy(fn, f_in, sizeof(double) * N);
    for (int s = 0; s < 4; ++s) {
        for (size_t p = 0; p < N; ++p)
            fs[p] = s == 0 ? fn[p] : fn[p] + alpha[s] * dt * ks[(size_t)(s - 1) * N + p];
        vpo_rhs(c->nx, c->nv, c->dx, c->dv, c->v_lo, c->vghost, fs, a, ks + (size_t)s * N);
    }
    for (size_t p = 0; p < N; ++p) {
        double sum = 0.0;
        for (int s = 0; s < 4; ++s) sum += b[s] * ks[(size_t)s * N + p];
        f_out[p] = fn[p] + dt * sum;
    }
    free(fn); free(fs); free(ks);
}

/* Threads the OpenMP loops of the oracle use (1 without OpenMP); the
 * setter changes the count for later calls (for timing only). */
#ifdef _OPENMP
#include <omp.h>
int vpo_num_threads(void) { return omp_get_max_threads(); }
void vpo_set_num_threads(int n) { if (n > 0) omp_set_num_threads(n); }
#else
int vpo_num_threads(void) { return 1; }
void vpo_set_num_threads(int n) { (void)n; }
#endif
