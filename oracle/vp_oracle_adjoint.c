/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Discrete adjoint (transpose of the Jacobian) of the unlimited RK4
 * Vlasov-Poisson step computed by vp_oracle.c.  The paper does not
 * derive an adjoint; this is the exact reverse-mode derivative of the
 * discrete step of section 2 (face averages, product-rule fluxes, flux
 * divergence, velocity moment, periodic Poisson solve, field, RK4
 * stages), taken operator by operator in reverse order:
 *
 *   forward  f(s) = f^n + alpha_s dt k_{s-1},  a(s) = K f(s),
 *            k_s  = L(f(s), a(s)),            f^{n+1} = f^n + dt sum b_s k_s
 *   reverse  kbar_s  = dt b_s lam + alpha_{s+1} dt fbar(s+1)
 *            fbar(s) = (dL/df)^T kbar_s + K^T (dL/da)^T kbar_s
 *            lam_n   = lam + sum_s fbar(s)
 *
 * K = (q/m) (-D) S (-dv R) is the moment/Poisson/field chain; the Poisson
 * solution operator S is symmetric and the periodic difference D is
 * antisymmetric, so K^T = (q/m) dv R^T S D.  The velocity ghost values
 * are constants and receive no cotangent.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vp_oracle.h"

static int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

static const double CF[4] = {-1.0 / 12.0, 7.0 / 12.0, 7.0 / 12.0, -1.0 / 12.0};  /* taps o=-1..2 */

static double face4(double um1, double u0, double u1, double u2)
{
    return (7.0 * (u0 + u1) - (um1 + u2)) / 12.0;
}

/* fbar = (dk/df)^T kbar (a fixed), abar = (dk/da)^T kbar (f fixed). */
void vpo_rhs_adjoint(int nx, int nv, double dx, double dv, double v_lo,
                     const double* vghost, const double* f, const double* a,
                     const double* kbar, double* fbar, double* abar)
{
    /* forward velocity-face averages Fv(i, j+1/2), i = -2..nx+1, j = -1..nv-1 */
    int FvW = nv + 1;
    double* Fv = (double*)malloc(sizeof(double) * (size_t)(nx + 4) * FvW);
#define FV(i, j) Fv[(size_t)((i) + 2) * FvW + ((j) + 1)]
    for (int i = -2; i < nx + 2; ++i) {
        const double* row = f + (size_t)wrap(i, nx) * nv;
        for (int j = -1; j < nv; ++j) {
            double u[4];
            for (int o = -1; o <= 2; ++o) {
                int jj = j + o;
                u[o + 1] = jj < -1 ? vghost[0] : jj == -1 ? vghost[1]
                         : jj == nv ? vghost[2] : jj > nv ? vghost[3] : row[jj];
            }
            FV(i, j) = face4(u[0], u[1], u[2], u[3]);
        }
    }
    /* flux cotangents */
    double* Gxb = (double*)malloc(sizeof(double) * (size_t)nx * nv);   /* face i+1/2, i = 0..nx-1 */
    double* Gvb = (double*)malloc(sizeof(double) * (size_t)nx * FvW);  /* face j+1/2, j = -1..nv-1 */
#define KB(i, j) kbar[(size_t)(i) * nv + (j)]
#define GXB(i, j) Gxb[(size_t)(i) * nv + (j)]
#define GVB(i, j) Gvb[(size_t)wrap(i, nx) * FvW + ((j) + 1)]
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < nv; ++j)
            GXB(i, j) = (KB(wrap(i + 1, nx), j) - KB(i, j)) / dx;
    for (int i = 0; i < nx; ++i)
        for (int j = -1; j < nv; ++j) {
            double up = j + 1 < nv ? KB(i, j + 1) : 0.0;
            double dn = j >= 0 ? KB(i, j) : 0.0;
            GVB(i, j) = (up - dn) / dv;
        }
    for (size_t p = 0; p < (size_t)nx * nv; ++p) fbar[p] = 0.0;
    /* x faces: Fx(i+1/2, j) for j = -1..nv; only interior j feed fbar */
    for (int i = 0; i < nx; ++i)
        for (int j = -1; j <= nv; ++j) {
            double fxb = 0.0;
            if (j >= 0 && j < nv) fxb += (v_lo + (j + 0.5) * dv) * GXB(i, j);
            if (j - 1 >= 0 && j - 1 < nv) fxb += dv / 24.0 * GXB(i, j - 1);
            if (j + 1 >= 0 && j + 1 < nv) fxb -= dv / 24.0 * GXB(i, j + 1);
            if (j < 0 || j >= nv) continue;            /* ghost column: constant */
            for (int o = -1; o <= 2; ++o)
                fbar[(size_t)wrap(i + o, nx) * nv + j] += CF[o + 1] * fxb;
        }
    /* velocity faces */
    for (int i = 0; i < nx; ++i) {
        double ai = a[i];
        double am2 = a[wrap(i - 2, nx)], ap2 = a[wrap(i + 2, nx)];
        for (int j = -1; j < nv; ++j) {
            double fvb = ai * GVB(i, j)
                       + (ai - am2) / 48.0 * GVB(i - 1, j)
                       - (ap2 - ai) / 48.0 * GVB(i + 1, j);
            for (int o = -1; o <= 2; ++o) {
                int jj = j + o;
                if (jj >= 0 && jj < nv) fbar[(size_t)i * nv + jj] += CF[o + 1] * fvb;
            }
        }
    }
    /* acceleration cotangent: a v-reduction */
    for (int i = 0; i < nx; ++i) {
        double s = 0.0;
        for (int j = -1; j < nv; ++j)
            s += FV(i, j) * GVB(i, j)
               + (FV(i, j) - FV(i - 2, j)) / 48.0 * GVB(i - 1, j)
               - (FV(i + 2, j) - FV(i, j)) / 48.0 * GVB(i + 1, j);
        abar[i] = s;
    }
#undef FV
#undef KB
#undef GXB
#undef GVB
    free(Gxb);
    free(Gvb);
    free(Fv);
}

/* fbar += K^T abar, with K the map f -> a of vpo_constraints. */
void vpo_constraints_adjoint(const vpo_ctx* c, const double* abar, double* fbar)
{
    int nx = c->nx, nv = c->nv;
    double* Eb = (double*)calloc(nx, sizeof(double));
    double* phib = (double*)calloc(nx, sizeof(double));
    double* rhob = (double*)malloc(sizeof(double) * nx);
    /* a = qm E */
    for (int i = 0; i < nx; ++i) Eb[i] = c->qm * abar[i];
    /* E = -D phi, D antisymmetric: phibar = D Ebar */
    for (int m = 0; m < nx; ++m) {
        double d1 = Eb[wrap(m + 1, nx)] - Eb[wrap(m - 1, nx)];
        double d2 = Eb[wrap(m + 2, nx)] - Eb[wrap(m - 2, nx)];
        phib[m] = (8.0 * d1 - d2) / (12.0 * c->dx);
    }
    /* phi = S rho with S symmetric: rhobar = S phibar */
    vpo_poisson_solve(c->P, c->dx, phib, rhob);
    /* rho = 1 - n, n_i = dv sum_j f_ij */
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < nv; ++j)
            fbar[(size_t)i * nv + j] += -c->dv * rhob[i];
    free(Eb); free(phib); free(rhob);
}

/* lam_n = (d f^{n+1} / d f^n)^T lam_np1 at the state f_n. */
void vpo_rk4_adjoint_step(const vpo_ctx* c, const double* f_n, const double* lam_np1,
                          double* lam_n, double dt)
{
    static const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    static const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    int nx = c->nx, nv = c->nv;
    size_t N = (size_t)nx * nv;
    double* sf = (double*)malloc(sizeof(double) * N * 4);
    double* sa = (double*)malloc(sizeof(double) * (size_t)nx * 4);
    double* tmp = (double*)malloc(sizeof(double) * N);
    vpo_rk4_step_stages(c, f_n, tmp, dt, sf, sa);
    double* kb = (double*)malloc(sizeof(double) * N);
    double* fb = (double*)malloc(sizeof(double) * N);
    double* ab = (double*)malloc(sizeof(double) * nx);
    double* acc = (double*)malloc(sizeof(double) * N);
    memcpy(acc, lam_np1, sizeof(double) * N);
    for (int s = 3; s >= 0; --s) {
        for (size_t p = 0; p < N; ++p)
            kb[p] = dt * b[s] * lam_np1[p] + (s < 3 ? alpha[s + 1] * dt * fb[p] : 0.0);
        vpo_rhs_adjoint(nx, nv, c->dx, c->dv, c->v_lo, c->vghost,
                        sf + (size_t)s * N, sa + (size_t)s * nx, kb, fb, ab);
        vpo_constraints_adjoint(c, ab, fb);
        for (size_t p = 0; p < N; ++p) acc[p] += fb[p];
    }
    memcpy(lam_n, acc, sizeof(double) * N);
    free(sf); free(sa); free(tmp); free(kb); free(fb); free(ab); free(acc);
}
