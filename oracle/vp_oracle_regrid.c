/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Regridding pieces of section 3 for 1D+1V levels stored [x][v]:
 *
 *   - the refinement criterion (section 3, mesh refinement criteria): a
 *     cell is tagged when delta1 f + delta2 f > tol, with
 *       delta1 f = [ 1/2 sum_d h_d (f(+e_d) - f(-e_d))^2 ]^(1/2),
 *       delta2 f = 1/2 sum_d h_d^2 |f(+e_d) - 2 f + f(-e_d)|,
 *     summed over the phase-space directions d = x, v (h_x = dx, h_v = dv),
 *     taken as printed;
 *   - the conservative, limited, high-order interpolation of section 3
 *     (eqs. aux1, aux2, interp_r_avg and the renormalisation): the fine
 *     cell averages of the three quadratic candidates of WENO5 in one
 *     coarse cell, combined with the nonlinear weights.  Reading: the
 *     printed B^(0) = 2 D_i - D_{i-1} is taken as 2 D_i - D_{i+1}, the value
 *     that the definition (the quadratic with the cell averages of cells
 *     i, i+1, i+2, averaged over the sub-cells) gives; the other printed
 *     coefficients agree with the definition;
 *   - the prolongation of a level into a fine box: in x first (periodic),
 *     then in v (ghost rows are the equilibrium cell averages), each 1D
 *     step conservative.
 *
 * Operation order of the criterion (kept identical by the GPU code so that
 * the tags agree exactly): per direction the squared difference is scaled
 * by h_d, the x term is added to the v term, halved, and the square root
 * taken; the second differences are formed as (f(+) - 2 f) + f(-), their
 * magnitudes scaled by h_d^2, summed x then v, and halved; the two
 * estimates are added.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vp_oracle.h"

static int wrapr(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

static double level_at(int nx, int nv, const double* vghost, const double* f, int i, int j)
{
    if (j < 0) return vghost[j + 2];
    if (j >= nv) return vghost[j - nv + 2];
    return f[(size_t)wrapr(i, nx) * nv + j];
}

double vpo_tag_value(int nx, int nv, double dx, double dv, const double* vghost, const double* f, int i, int j)
{
    const double c = level_at(nx, nv, vghost, f, i, j);
    const double xm = level_at(nx, nv, vghost, f, i - 1, j), xp = level_at(nx, nv, vghost, f, i + 1, j);
    const double vm = level_at(nx, nv, vghost, f, i, j - 1), vp = level_at(nx, nv, vghost, f, i, j + 1);
    const double gx = xp - xm, gv = vp - vm;
    const double d1 = sqrt(0.5 * (dx * (gx * gx) + dv * (gv * gv)));
    const double sx = (xp - 2.0 * c) + xm, sv = (vp - 2.0 * c) + vm;
    const double d2 = 0.5 * ((dx * dx) * fabs(sx) + (dv * dv) * fabs(sv));
    return d1 + d2;
}

void vpo_tag(int nx, int nv, double dx, double dv, const double* vghost, const double* f, double tol,
             unsigned char* tags)
{
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < nv; ++j)
            tags[(size_t)i * nv + j] = vpo_tag_value(nx, nv, dx, dv, vghost, f, i, j) > tol ? 1 : 0;
}

/* R fine cell averages of coarse cell i from u[0..4] = ubar_{i-2..i+2} */
void vpo_prolong1d(const double* u, int R, double* out)
{
    const double eps = 1e-6;
    const double d[3] = {0.3, 0.6, 0.1};
    double D[4];                                   /* D_{i+n}, n = -2..1 */
    for (int n = 0; n < 4; ++n) D[n] = u[n + 1] - u[n];
    double Dl[3];                                  /* Delta_{i+p}, p = -1..1 */
    for (int p = 0; p < 3; ++p) Dl[p] = D[p + 1] - D[p];
    const double Dm2 = D[0], Dm1 = D[1], D0 = D[2], Dp1 = D[3];
    const double Lm1 = Dl[0], L0 = Dl[1], Lp1 = Dl[2];
    const double beta[3] = {
        13.0 / 12.0 * Lp1 * Lp1 + 0.25 * (Dp1 - 3.0 * D0) * (Dp1 - 3.0 * D0),
        13.0 / 12.0 * L0 * L0 + 0.25 * (D0 + Dm1) * (D0 + Dm1),
        13.0 / 12.0 * Lm1 * Lm1 + 0.25 * (3.0 * Dm1 - Dm2) * (3.0 * Dm1 - Dm2),
    };
    double alpha[3], asum = 0.0;
    for (int r = 0; r < 3; ++r) {
        alpha[r] = d[r] / ((eps + beta[r]) * (eps + beta[r]));
        asum += alpha[r];
    }
    const double ui = u[2];
    const double A[3] = {ui + (2.0 * Dp1 - 5.0 * D0) / 6.0, ui - (D0 + 2.0 * Dm1) / 6.0,
                         ui - (4.0 * Dm1 - Dm2) / 6.0};
    const double B[3] = {2.0 * D0 - Dp1, Dm1, Dm1};
    const double C[3] = {Lp1, L0, Lm1};
    for (int s = 0; s < R; ++s) out[s] = 0.0;
    for (int r = 0; r < 3; ++r) {
        double fine[64];
        double sum = 0.0;
        for (int s = 0; s < R; ++s) {
            fine[s] = A[r] + B[r] * ((2.0 * s + 1.0) / (2.0 * R)) + C[r] * ((3.0 * s * s + 3.0 * s + 1.0) / (6.0 * R * R));
            sum += fine[s];
        }
        fine[R - 1] += ui - sum / R;               /* renormalisation: exact conservation */
        const double w = alpha[r] / asum;
        for (int s = 0; s < R; ++s) out[s] += w * fine[s];
    }
}

/* Fine cell averages on the fine box [fx0, fx1] x [fv0, fv1] (level-1
 * indices, aligned to R) from the level-0 array fc[ncx][ncv]; out is
 * [fx1 - fx0 + 1][fv1 - fv0 + 1] */
void vpo_prolong_box(int ncx, int ncv, const double* fc, const double* vghost_c, int R, int fx0, int fv0, int fx1,
                     int fv1, double* out)
{
    const int cx0 = fx0 / R, cx1 = fx1 / R, cv0 = fv0 / R, cv1 = fv1 / R;
    const int nfx = fx1 - fx0 + 1, nfv = fv1 - fv0 + 1;
    const int nvt = cv1 - cv0 + 5;                /* coarse v rows cv0-2 .. cv1+2 */
    double* T = (double*)malloc(sizeof(double) * (size_t)nfx * nvt);
    /* x first: fine in x, coarse in v */
    for (int cx = cx0; cx <= cx1; ++cx)
        for (int q = 0; q < nvt; ++q) {
            const int cv = cv0 - 2 + q;
            double u[5], o[64];
            for (int e = 0; e < 5; ++e) u[e] = level_at(ncx, ncv, vghost_c, fc, cx - 2 + e, cv);
            vpo_prolong1d(u, R, o);
            for (int s = 0; s < R; ++s) T[(size_t)((cx - cx0) * R + s) * nvt + q] = o[s];
        }
    /* then v */
    for (int x = 0; x < nfx; ++x)
        for (int cv = cv0; cv <= cv1; ++cv) {
            double u[5], o[64];
            for (int e = 0; e < 5; ++e) u[e] = T[(size_t)x * nvt + (cv - cv0) + e];
            vpo_prolong1d(u, R, o);
            for (int s = 0; s < R; ++s) out[(size_t)x * nfv + (cv - cv0) * R + s] = o[s];
        }
    free(T);
}
