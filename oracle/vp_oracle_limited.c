/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * The limited face averages of section 2 (eqs. limitedFace, thirdLeft,
 * thirdRight) for the 1D+1V single-level scheme: each face average is a
 * weighted sum of the left- and right-biased third-order approximations;
 * the provisional weights come from the standard WENO smoothness
 * indicators, and the larger weight is given to the upwind candidate.
 *
 * Readings (the paper defers the provisional weights to its references):
 *   - provisional weights: Jiang-Shu smoothness indicators of the two
 *     three-cell stencils, ideal weights 1/2 and 1/2, epsilon = 1e-6,
 *     power 2;
 *   - the upwind direction of an x face is the sign of the cell-centre
 *     velocity of its column; of a v face, the sign of the acceleration
 *     a = (q/m) E of its row; zero counts as "not positive";
 *   - the product-rule fluxes of section 2 are unchanged, with every face
 *     average (including the neighbouring ones in the correction terms)
 *     replaced by its limited value.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vp_oracle.h"

#define LIM_EPS 1e-6

static int wrapl(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

/* face average between u0 and u1 from u_{-1}, u0, u1, u2; upwind_left
 * when the advection speed through the face is positive */
double vpo_face_limited(double um1, double u0, double u1, double u2, int upwind_left)
{
    const double fl = (-um1 + 5.0 * u0 + 2.0 * u1) / 6.0;
    const double fr = (2.0 * u0 + 5.0 * u1 - u2) / 6.0;
    const double d1 = um1 - 2.0 * u0 + u1, e1 = um1 - u1;
    const double d2 = u0 - 2.0 * u1 + u2, e2 = 3.0 * u0 - 4.0 * u1 + u2;
    const double bl = 13.0 / 12.0 * d1 * d1 + 0.25 * e1 * e1;
    const double br = 13.0 / 12.0 * d2 * d2 + 0.25 * e2 * e2;
    const double al = 0.5 / ((LIM_EPS + bl) * (LIM_EPS + bl));
    const double ar = 0.5 / ((LIM_EPS + br) * (LIM_EPS + br));
    const double wl_hat = al / (al + ar), wr_hat = ar / (al + ar);
    const double wmax = wl_hat > wr_hat ? wl_hat : wr_hat;
    const double wmin = wl_hat > wr_hat ? wr_hat : wl_hat;
    const double wl = upwind_left ? wmax : wmin;
    const double wr = upwind_left ? wmin : wmax;
    return wl * fl + wr * fr;
}

static double ghost_at(int nx, int nv, const double* vghost, const double* f, int i, int j)
{
    if (j < 0) return vghost[j + 2];
    if (j >= nv) return vghost[j - nv + 2];
    return f[(size_t)wrapl(i, nx) * nv + j];
}

/* k = L(f; a) with limited face averages */
void vpo_rhs_limited(int nx, int nv, double dx, double dv, double v_lo, const double* vghost, const double* f,
                     const double* a, double* k)
{
#define F(i, j) ghost_at(nx, nv, vghost, f, (i), (j))
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i) {
        for (int j = 0; j < nv; ++j) {
            double gx[2], gv[2];
            for (int side = 0; side < 2; ++side) {
                const int ii = i - 1 + side;          /* x face ii + 1/2 */
                double fx[3];
                for (int m = -1; m <= 1; ++m) {
                    const int jj = j + m;
                    const double vb = v_lo + (jj + 0.5) * dv;
                    fx[m + 1] = vpo_face_limited(F(ii - 1, jj), F(ii, jj), F(ii + 1, jj), F(ii + 2, jj), vb > 0.0);
                }
                const double vb = v_lo + (j + 0.5) * dv;
                gx[side] = vb * fx[1] + dv / 24.0 * (fx[2] - fx[0]);
                const int jj = j - 1 + side;          /* v face jj + 1/2 */
                double fv[3];
                for (int m = -1; m <= 1; ++m) {
                    const int r = i + m;
                    const double ar = a[wrapl(r, nx)];
                    fv[m + 1] = vpo_face_limited(F(r, jj - 1), F(r, jj), F(r, jj + 1), F(r, jj + 2), ar > 0.0);
                }
                const double ai = a[i], da = a[wrapl(i + 1, nx)] - a[wrapl(i - 1, nx)];
                gv[side] = ai * fv[1] + da / 48.0 * (fv[2] - fv[0]);
            }
            k[(size_t)i * nv + j] = -(gx[1] - gx[0]) / dx - (gv[1] - gv[0]) / dv;
        }
    }
#undef F
}

/* classic RK4 with limited faces; the field is re-solved at every stage
 * (a_fixed == NULL) or held fixed */
static void rk4_lim(const vpo_ctx* c, const double* f_in, double* f_out, const double* a_fixed, double dt)
{
    static const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    static const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    const size_t N = (size_t)c->nx * c->nv;
    double* fs = (double*)malloc(sizeof(double) * N);
    double* k = (double*)calloc(N, sizeof(double));
    double* acc = (double*)malloc(sizeof(double) * N);
    double* a = (double*)malloc(sizeof(double) * c->nx);
    memcpy(acc, f_in, sizeof(double) * N);
    for (int s = 0; s < 4; ++s) {
        for (size_t q = 0; q < N; ++q) fs[q] = f_in[q] + alpha[s] * dt * k[q];
        if (a_fixed) memcpy(a, a_fixed, sizeof(double) * c->nx);
        else vpo_constraints(c, fs, a, NULL, NULL, NULL);
        vpo_rhs_limited(c->nx, c->nv, c->dx, c->dv, c->v_lo, c->vghost, fs, a, k);
        for (size_t q = 0; q < N; ++q) acc[q] += dt * b[s] * k[q];
    }
    memcpy(f_out, acc, sizeof(double) * N);
    free(fs); free(k); free(acc); free(a);
}

void vpo_rk4_step_limited(const vpo_ctx* c, const double* f_in, double* f_out, double dt)
{
    rk4_lim(c, f_in, f_out, NULL, dt);
}

void vpo_rk4_step_fixed_a_limited(const vpo_ctx* c, const double* f_in, double* f_out, const double* a, double dt)
{
    rk4_lim(c, f_in, f_out, a, dt);
}
