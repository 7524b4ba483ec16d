/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Single-level 2D+2V Vlasov-Poisson step, FP64, f stored [x][y][vx][vy].
 * The paper states the fourth-order finite-volume method for 1D+1V
 * (section 2) and leaves 2D+2V to future work; this is its direction-by-
 * direction extension:
 *   - face averages: the centred fourth-order formula of section 2 along
 *     the face normal, from cell averages;
 *   - product-rule corrections only along the directions in which the
 *     advection speed varies: on x faces (speed vx) along vx, on y faces
 *     along vy, on vx faces (speed ax(x, y)) along x and y, on vy faces
 *     along x and y, each with the coefficients of section 2 (dv/24 for the
 *     velocity, 1/48 for the acceleration);
 *   - Poisson: the sum of the 1D fourth-order operators of section 2 in x
 *     and y (each scaled by 12 h^2 as in 1D), periodic, zero-mean potential,
 *     solved here by conjugate gradients; E = -D phi per direction with the
 *     1D field stencil;
 *   - velocity ghost cells hold the cell averages of the unperturbed
 *     equilibrium, the product veq_x[k] veq_y[l].
 * Each cell's update is computed from scratch with every face flux written
 * out; no blocking or reuse.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vp_oracle.h"

typedef struct {
    int nx, ny, nvx, nvy;
    double dx, dy, dvx, dvy, v_lo, qm;
    double* gx;   /* nvx + 4 */
    double* gy;   /* nvy + 4 */
} vpo4;

static int wrap4(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

void* vpo4_ctx_new(int nx, int ny, int nvx, int nvy, double x_len, double y_len, double v_lo, double v_hi,
                   double qm, const double* veq_x, const double* veq_y)
{
    vpo4* c = (vpo4*)calloc(1, sizeof(*c));
    c->nx = nx; c->ny = ny; c->nvx = nvx; c->nvy = nvy;
    c->dx = x_len / nx; c->dy = y_len / ny;
    c->dvx = (v_hi - v_lo) / nvx; c->dvy = (v_hi - v_lo) / nvy;
    c->v_lo = v_lo; c->qm = qm;
    c->gx = (double*)malloc(sizeof(double) * (nvx + 4));
    c->gy = (double*)malloc(sizeof(double) * (nvy + 4));
    memcpy(c->gx, veq_x, sizeof(double) * (nvx + 4));
    memcpy(c->gy, veq_y, sizeof(double) * (nvy + 4));
    return c;
}

void vpo4_ctx_free(void* h)
{
    vpo4* c = (vpo4*)h;
    if (!c) return;
    free(c->gx); free(c->gy); free(c);
}

/* cell average with x, y periodic and the equilibrium in velocity ghosts */
static double at(const vpo4* c, const double* f, int i, int j, int k, int l)
{
    if (k < 0 || k >= c->nvx || l < 0 || l >= c->nvy) return c->gx[k + 2] * c->gy[l + 2];
    i = wrap4(i, c->nx);
    j = wrap4(j, c->ny);
    return f[(((size_t)i * c->ny + j) * c->nvx + k) * c->nvy + l];
}

static double face(double um1, double u0, double u1, double u2) { return (7.0 * (u0 + u1) - (um1 + u2)) / 12.0; }

/* n_ij = dvx dvy sum_kl f_ijkl */
void vpo4_moment(void* h, double* f, double* n)
{
    vpo4* c = (vpo4*)h;
    const size_t plane = (size_t)c->nvx * c->nvy;
    for (int p = 0; p < c->nx * c->ny; ++p) {
        double s = 0.0;
        for (size_t q = 0; q < plane; ++q) s += f[p * plane + q];
        n[p] = c->dvx * c->dvy * s;
    }
}

/* (L phi)_ij = (A_x phi)_ij / (12 dx^2) + (A_y phi)_ij / (12 dy^2),
 * A u_i = 30 u_i - 16 (u_{i+1} + u_{i-1}) + (u_{i+2} + u_{i-2}) */
static void apply_L(const vpo4* c, const double* u, double* out)
{
    const int nx = c->nx, ny = c->ny;
    const double sx = 1.0 / (12.0 * c->dx * c->dx), sy = 1.0 / (12.0 * c->dy * c->dy);
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
#define U(a, b) u[(size_t)wrap4(a, nx) * ny + wrap4(b, ny)]
            double ax = 30.0 * U(i, j) - 16.0 * (U(i + 1, j) + U(i - 1, j)) + (U(i + 2, j) + U(i - 2, j));
            double ay = 30.0 * U(i, j) - 16.0 * (U(i, j + 1) + U(i, j - 1)) + (U(i, j + 2) + U(i, j - 2));
#undef U
            out[(size_t)i * ny + j] = sx * ax + sy * ay;
        }
}

/* L phi = rho - mean(rho), mean(phi) = 0, by conjugate gradients (L is
 * symmetric positive semi-definite with the constants as null space and
 * the right-hand side is orthogonal to it).  The residual is kept
 * orthogonal to the constants, the true residual is evaluated at every
 * iteration and the iterate with the smallest one is returned (once CG
 * has converged in exact arithmetic, rounding can make the iteration
 * wander).  Returns that relative residual |b - L phi| / |b|. */
double vpo4_poisson(void* h, double* rho, double* phi)
{
    vpo4* c = (vpo4*)h;
    const int n = c->nx * c->ny;
    double* x = (double*)calloc(n, sizeof(double));
    double* r = (double*)malloc(sizeof(double) * n);
    double* p = (double*)malloc(sizeof(double) * n);
    double* q = (double*)malloc(sizeof(double) * n);
    double* b = (double*)malloc(sizeof(double) * n);
    double mean = 0.0;
    for (int i = 0; i < n; ++i) mean += rho[i];
    mean /= n;
    double bb = 0.0;
    for (int i = 0; i < n; ++i) { b[i] = rho[i] - mean; bb += b[i] * b[i]; r[i] = b[i]; p[i] = b[i]; phi[i] = 0.0; }
    double rr = bb, best = bb;
    int stall = 0;
    for (int it = 0; bb > 0.0 && it < 20 * n + 100; ++it) {
        apply_L(c, p, q);
        double pq = 0.0;
        for (int i = 0; i < n; ++i) pq += p[i] * q[i];
        if (!(pq > 0.0)) break;
        const double alpha = rr / pq;
        double rm = 0.0;
        for (int i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; rm += r[i]; }
        rm /= n;
        double rr2 = 0.0;
        for (int i = 0; i < n; ++i) { r[i] -= rm; rr2 += r[i] * r[i]; }
        apply_L(c, x, q);
        double t = 0.0;
        for (int i = 0; i < n; ++i) { const double d = b[i] - q[i]; t += d * d; }
        if (t < best) { best = t; memcpy(phi, x, sizeof(double) * n); stall = 0; }
        else ++stall;
        if (best <= 1e-30 * bb || stall > 50 || rr2 == 0.0) break;
        const double beta = rr2 / rr;
        rr = rr2;
        for (int i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
    }
    double m = 0.0;
    for (int i = 0; i < n; ++i) m += phi[i];
    m /= n;
    for (int i = 0; i < n; ++i) phi[i] -= m;
    apply_L(c, phi, q);
    double t = 0.0;
    for (int i = 0; i < n; ++i) { const double d = b[i] - q[i]; t += d * d; }
    free(x); free(r); free(p); free(q); free(b);
    return bb > 0.0 ? sqrt(t / bb) : 0.0;
}

/* E = -D phi per direction: E[0 .. nx ny) = Ex, E[nx ny .. 2 nx ny) = Ey */
void vpo4_field(void* h, double* phi, double* E)
{
    vpo4* c = (vpo4*)h;
    const int nx = c->nx, ny = c->ny;
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
#define P(a, b) phi[(size_t)wrap4(a, nx) * ny + wrap4(b, ny)]
            double dx1 = P(i + 1, j) - P(i - 1, j), dx2 = P(i + 2, j) - P(i - 2, j);
            double dy1 = P(i, j + 1) - P(i, j - 1), dy2 = P(i, j + 2) - P(i, j - 2);
#undef P
            E[(size_t)i * ny + j] = -(8.0 * dx1 - dx2) / (12.0 * c->dx);
            E[(size_t)nx * ny + (size_t)i * ny + j] = -(8.0 * dy1 - dy2) / (12.0 * c->dy);
        }
}

/* moment -> rho = 1 - n -> Poisson -> field -> a = (q/m) E (2 nx ny) */
void vpo4_constraints(void* h, double* f, double* a, double* phi_out, double* E_out)
{
    vpo4* c = (vpo4*)h;
    const int n = c->nx * c->ny;
    double* nn = (double*)malloc(sizeof(double) * n);
    double* phi = (double*)malloc(sizeof(double) * n);
    double* E = (double*)malloc(sizeof(double) * 2 * n);
    vpo4_moment(h, f, nn);
    for (int i = 0; i < n; ++i) nn[i] = 1.0 - nn[i];
    vpo4_poisson(h, nn, phi);
    vpo4_field(h, phi, E);
    for (int i = 0; i < 2 * n; ++i) a[i] = c->qm * E[i];
    if (phi_out) memcpy(phi_out, phi, sizeof(double) * n);
    if (E_out) memcpy(E_out, E, sizeof(double) * 2 * n);
    free(nn); free(phi); free(E);
}

/* fluxes through the faces of cell (i, j, k, l) */
static double gx_face(const vpo4* c, const double* f, int i, int j, int k, int l)   /* face i + 1/2 */
{
    double fc = face(at(c, f, i - 1, j, k, l), at(c, f, i, j, k, l), at(c, f, i + 1, j, k, l), at(c, f, i + 2, j, k, l));
    double fu = face(at(c, f, i - 1, j, k + 1, l), at(c, f, i, j, k + 1, l), at(c, f, i + 1, j, k + 1, l),
                     at(c, f, i + 2, j, k + 1, l));
    double fd = face(at(c, f, i - 1, j, k - 1, l), at(c, f, i, j, k - 1, l), at(c, f, i + 1, j, k - 1, l),
                     at(c, f, i + 2, j, k - 1, l));
    double vb = c->v_lo + (k + 0.5) * c->dvx;
    return vb * fc + c->dvx / 24.0 * (fu - fd);
}

static double gy_face(const vpo4* c, const double* f, int i, int j, int k, int l)   /* face j + 1/2 */
{
    double fc = face(at(c, f, i, j - 1, k, l), at(c, f, i, j, k, l), at(c, f, i, j + 1, k, l), at(c, f, i, j + 2, k, l));
    double fu = face(at(c, f, i, j - 1, k, l + 1), at(c, f, i, j, k, l + 1), at(c, f, i, j + 1, k, l + 1),
                     at(c, f, i, j + 2, k, l + 1));
    double fd = face(at(c, f, i, j - 1, k, l - 1), at(c, f, i, j, k, l - 1), at(c, f, i, j + 1, k, l - 1),
                     at(c, f, i, j + 2, k, l - 1));
    double vb = c->v_lo + (l + 0.5) * c->dvy;
    return vb * fc + c->dvy / 24.0 * (fu - fd);
}

static double fvx(const vpo4* c, const double* f, int i, int j, int k, int l)       /* <f> on face k + 1/2 */
{
    return face(at(c, f, i, j, k - 1, l), at(c, f, i, j, k, l), at(c, f, i, j, k + 1, l), at(c, f, i, j, k + 2, l));
}

static double fvy(const vpo4* c, const double* f, int i, int j, int k, int l)       /* <f> on face l + 1/2 */
{
    return face(at(c, f, i, j, k, l - 1), at(c, f, i, j, k, l), at(c, f, i, j, k, l + 1), at(c, f, i, j, k, l + 2));
}

static double A(const vpo4* c, const double* a, int comp, int i, int j)
{
    return a[(size_t)comp * c->nx * c->ny + (size_t)wrap4(i, c->nx) * c->ny + wrap4(j, c->ny)];
}

static double gvx_face(const vpo4* c, const double* f, const double* a, int i, int j, int k, int l)
{
    double ac = A(c, a, 0, i, j);
    double dax = A(c, a, 0, i + 1, j) - A(c, a, 0, i - 1, j);
    double day = A(c, a, 0, i, j + 1) - A(c, a, 0, i, j - 1);
    return ac * fvx(c, f, i, j, k, l) + (dax * (fvx(c, f, i + 1, j, k, l) - fvx(c, f, i - 1, j, k, l)) +
                                         day * (fvx(c, f, i, j + 1, k, l) - fvx(c, f, i, j - 1, k, l))) / 48.0;
}

static double gvy_face(const vpo4* c, const double* f, const double* a, int i, int j, int k, int l)
{
    double ac = A(c, a, 1, i, j);
    double dax = A(c, a, 1, i + 1, j) - A(c, a, 1, i - 1, j);
    double day = A(c, a, 1, i, j + 1) - A(c, a, 1, i, j - 1);
    return ac * fvy(c, f, i, j, k, l) + (dax * (fvy(c, f, i + 1, j, k, l) - fvy(c, f, i - 1, j, k, l)) +
                                         day * (fvy(c, f, i, j + 1, k, l) - fvy(c, f, i, j - 1, k, l))) / 48.0;
}

/* k = -sum over the four directions of (G_{+1/2} - G_{-1/2}) / h */
void vpo4_rhs(void* h, double* f, double* a, double* k_out)
{
    const vpo4* c = (const vpo4*)h;
    const int nx = c->nx, ny = c->ny, nvx = c->nvx, nvy = c->nvy;
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            for (int k = 0; k < nvx; ++k)
                for (int l = 0; l < nvy; ++l) {
                    double r = -(gx_face(c, f, i, j, k, l) - gx_face(c, f, i - 1, j, k, l)) / c->dx
                               - (gy_face(c, f, i, j, k, l) - gy_face(c, f, i, j - 1, k, l)) / c->dy
                               - (gvx_face(c, f, a, i, j, k, l) - gvx_face(c, f, a, i, j, k - 1, l)) / c->dvx
                               - (gvy_face(c, f, a, i, j, k, l) - gvy_face(c, f, a, i, j, k, l - 1)) / c->dvy;
                    k_out[(((size_t)i * ny + j) * nvx + k) * nvy + l] = r;
                }
}

/* classic RK4 (eq. rk4): the field is recomputed at every stage state */
static void rk4(void* h, double* f_in, double* f_out, double dt, const double* a_fixed)
{
    vpo4* c = (vpo4*)h;
    const size_t N = (size_t)c->nx * c->ny * c->nvx * c->nvy;
    const int na = 2 * c->nx * c->ny;
    static const double alpha[4] = {0.0, 0.5, 0.5, 1.0};
    static const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    double* fs = (double*)malloc(sizeof(double) * N);
    double* k = (double*)calloc(N, sizeof(double));
    double* acc = (double*)malloc(sizeof(double) * N);
    double* a = (double*)malloc(sizeof(double) * na);
    memcpy(acc, f_in, sizeof(double) * N);
    for (int s = 0; s < 4; ++s) {
        for (size_t q = 0; q < N; ++q) fs[q] = f_in[q] + alpha[s] * dt * k[q];
        if (a_fixed) memcpy(a, a_fixed, sizeof(double) * na);
        else vpo4_constraints(h, fs, a, NULL, NULL);
        vpo4_rhs(h, fs, a, k);
        for (size_t q = 0; q < N; ++q) acc[q] += dt * b[s] * k[q];
    }
    memcpy(f_out, acc, sizeof(double) * N);
    free(fs); free(k); free(acc); free(a);
}

void vpo4_rk4_step(void* h, double* f_in, double* f_out, double dt) { rk4(h, f_in, f_out, dt, NULL); }

void vpo4_rk4_step_fixed_a(void* h, double* f_in, double* f_out, double* a, double dt)
{
    rk4(h, f_in, f_out, dt, a);
}

/* Refinement criterion of section 3 (mesh refinement criteria) on a 2D+2V
 * mesh: delta1 f + delta2 f with the sums over the four directions x, y,
 * vx, vy (the printed criterion sums over the phase-space directions),
 *   delta1 f = [ 1/2 sum_d h_d (f(+e_d) - f(-e_d))^2 ]^(1/2),
 *   delta2 f = 1/2 sum_d h_d^2 |f(+e_d) - 2 f + f(-e_d)|,
 * x and y periodic, velocity ghosts the equilibrium.  Terms are added in
 * the order x, y, vx, vy. */
double vpo4_tag_value(void* h, double* f, int i, int j, int k, int l)
{
    const vpo4* c = (const vpo4*)h;
    const double hd[4] = {c->dx, c->dy, c->dvx, c->dvy};
    const int e[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
    const double u = at(c, f, i, j, k, l);
    double s1 = 0.0, s2 = 0.0;
    for (int d = 0; d < 4; ++d) {
        const double p = at(c, f, i + e[d][0], j + e[d][1], k + e[d][2], l + e[d][3]);
        const double m = at(c, f, i - e[d][0], j - e[d][1], k - e[d][2], l - e[d][3]);
        const double g = p - m, s = (p - 2.0 * u) + m;
        s1 = d == 0 ? hd[d] * (g * g) : s1 + hd[d] * (g * g);
        s2 = d == 0 ? (hd[d] * hd[d]) * fabs(s) : s2 + (hd[d] * hd[d]) * fabs(s);
    }
    return sqrt(0.5 * s1) + 0.5 * s2;
}

void vpo4_tag(void* h, double* f, double tol, unsigned char* tags, double* values)
{
    const vpo4* c = (const vpo4*)h;
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < c->nx; ++i)
        for (int j = 0; j < c->ny; ++j)
            for (int k = 0; k < c->nvx; ++k)
                for (int l = 0; l < c->nvy; ++l) {
                    const size_t q = (((size_t)i * c->ny + j) * c->nvx + k) * c->nvy + l;
                    const double v = vpo4_tag_value(h, f, i, j, k, l);
                    tags[q] = v > tol ? 1 : 0;
                    if (values) values[q] = v;
                }
}
