// Host runtime of the single-level 2D+2V path: plan tables (equilibrium
// factors, the real Fourier basis of the configuration mesh and the
// inverse symbol of the summed 1D Poisson operators) and the enqueue
// sequence of one RK4 step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "vp_internal.hpp"

namespace vp {

// Real orthonormal Fourier basis of the periodic n-cell mesh, Q[i * n + m]:
// m = 0 the constant, m = 2k - 1 / 2k the cosine / sine of frequency k,
// and for even n the last column the alternating vector.  Every symmetric
// circulant matrix is diagonal in this basis.
std::vector<double> fourier_basis(int n)
{
    std::vector<double> Q((size_t)n * n);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        Q[(size_t)i * n] = 1.0 / std::sqrt((double)n);
        for (int k = 1; 2 * k < n; ++k) {
            const double th = 2.0 * pi * k * i / n;
            Q[(size_t)i * n + 2 * k - 1] = std::sqrt(2.0 / n) * std::cos(th);
            Q[(size_t)i * n + 2 * k] = std::sqrt(2.0 / n) * std::sin(th);
        }
        if (n % 2 == 0 && n > 1) Q[(size_t)i * n + n - 1] = ((i & 1) ? -1.0 : 1.0) / std::sqrt((double)n);
    }
    return Q;
}

// eigenvalue of (30 - 16 (S + S^-1) + (S^2 + S^-2)) / (12 h^2) on basis column m,
// 30 - 32 cos t + 2 cos 2t in its factored form 4 sin^2(t/2) (14 - 2 cos t),
// which keeps full relative accuracy at small t
std::vector<double> fourier_symbol(int n, double h)
{
    const double pi = 3.14159265358979323846;
    std::vector<double> lam(n);
    for (int m = 0; m < n; ++m) {
        const int k = (m + 1) / 2;
        const double th = 2.0 * pi * k / n;
        const double s = std::sin(0.5 * th);
        lam[m] = 4.0 * s * s * (14.0 - 2.0 * std::cos(th)) / (12.0 * h * h);
    }
    return lam;
}

// Q followed by its transpose (the Poisson solve of larger meshes reads both)
std::vector<double> fourier_basis_and_transpose(int n)
{
    std::vector<double> Q = fourier_basis(n);
    Q.resize((size_t)2 * n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Q[(size_t)n * n + (size_t)j * n + i] = Q[(size_t)i * n + j];
    return Q;
}

namespace {

hipError_t upload(double** dst, const std::vector<double>& v)
{
    hipError_t e = hipMalloc(dst, v.size() * sizeof(double));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Stage4DArgs base(const vp_plan* p)
{
    const Plan4D& M = *p->p4;
    Stage4DArgs A{};
    A.nx = M.nx;
    A.ny = M.ny;
    A.nvx = M.nvx;
    A.nvy = M.nvy;
    A.dxi = 1.0 / M.dx;
    A.dyi = 1.0 / M.dy;
    A.dvxi = 1.0 / M.dvx;
    A.dvyi = 1.0 / M.dvy;
    A.dvx24 = M.dvx / 24.0;
    A.dvy24 = M.dvy / 24.0;
    A.vx_lo = M.v_lo;
    A.vy_lo = M.v_lo;
    A.dvx = M.dvx;
    A.dvy = M.dvy;
    A.gx = M.d_gx;
    A.gy = M.d_gy;
    A.mscale = M.dvx * M.dvy;
    return A;
}

char* wsp(void* work, size_t off) { return static_cast<char*>(work) + off; }

}  // namespace

vp_status p4_create(vp_plan* p, const vp_problem* pb)
{
    if (pb->dtype != VP_F64) return fail(VP_ENOTSUP, "2D+2V is supported in FP64");
    if (!pb->veq[0][1]) return fail(VP_EINVAL, "veq[0][1] (equilibrium along vy with ghosts) is required");
    if (pb->v_lo[0] != pb->v_lo[1] || pb->v_hi[0] != pb->v_hi[1])
        return fail(VP_ENOTSUP, "2D+2V needs the same velocity interval in vx and vy");
    Plan4D* M = new Plan4D();
    p->p4 = M;
    M->nx = pb->cells[0];
    M->ny = pb->cells[1];
    M->nvx = pb->cells[2];
    M->nvy = pb->cells[3];
    if (M->nx > kMaxPoisson2D || M->ny > kMaxPoisson2D)
        return fail(VP_ENOTSUP, "2D+2V configuration mesh is limited to 256 x 256 cells");
    if (M->nvx > kMaxVx4D) return fail(VP_ENOTSUP, "2D+2V is limited to 1024 cells along vx");
    if ((double)M->nx * M->ny * M->nvx * M->nvy >= 2147483648.0)
        return fail(VP_ENOTSUP, "2D+2V is limited to 2^31 phase-space cells");
    M->dx = pb->x_len[0] / M->nx;
    M->dy = pb->x_len[1] / M->ny;
    M->dvx = (pb->v_hi[0] - pb->v_lo[0]) / M->nvx;
    M->dvy = (pb->v_hi[1] - pb->v_lo[1]) / M->nvy;
    M->v_lo = pb->v_lo[0];
    std::vector<double> gx(pb->veq[0][0], pb->veq[0][0] + M->nvx + 4);
    std::vector<double> gy(pb->veq[0][1], pb->veq[0][1] + M->nvy + 4);
    const std::vector<double> Qx = fourier_basis(M->nx), Qy = fourier_basis_and_transpose(M->ny);
    const std::vector<double> lx = fourier_symbol(M->nx, M->dx), ly = fourier_symbol(M->ny, M->dy);
    std::vector<double> inv((size_t)M->nx * M->ny);
    for (int l = 0; l < M->ny; ++l)
        for (int k = 0; k < M->nx; ++k) {
            const double s = lx[k] + ly[l];
            inv[(size_t)l * M->nx + k] = (k == 0 && l == 0) ? 0.0 : 1.0 / s;
        }
    VP_HIP(upload(&M->d_gx, gx));
    VP_HIP(upload(&M->d_gy, gy));
    VP_HIP(upload(&M->d_Qx, Qx));
    VP_HIP(upload(&M->d_Qy, Qy));
    VP_HIP(upload(&M->d_invlamT, inv));
    VP_HIP(upload(&M->d_g, std::vector<double>((size_t)2 * M->nx * M->ny, 0.0)));

    p->state_elems = (size_t)M->nx * M->ny * M->nvx * M->nvy;
    const size_t sb = align256(p->state_elems * sizeof(double));
    size_t o = 0;
    p->ws_acc = o; o += sb;
    p->ws_fsa = o; o += sb;
    p->ws_fsb = o; o += sb;
    const size_t nseg = M->nvy > kMaxVy4D ? (size_t)(M->nvy + kSegVy4D - 1) / kSegVy4D : 1;
    M->ws_n = o; o += align256(nseg * M->nx * M->ny * sizeof(double));      // per vy segment
    M->ws_E = o; o += align256((size_t)2 * M->nx * M->ny * sizeof(double));   // Fourier coefficients in rk4
    p->ws_total = o;
    return VP_OK;
}

void p4_destroy(vp_plan* p)
{
    Plan4D* M = p->p4;
    if (!M) return;
    double* ptrs[] = {M->d_gx, M->d_gy, M->d_Qx, M->d_Qy, M->d_invlamT, M->d_g};
    for (double* q : ptrs)
        if (q) (void)hipFree(q);
    delete M;
    p->p4 = nullptr;
}

vp_status p4_rhs(const vp_plan* p, const void* f, const double* a, void* k, hipStream_t stream)
{
    Stage4DArgs A = base(p);
    A.fs = static_cast<const double*>(f);
    A.fout = static_cast<double*>(k);
    A.a = a;
    VP_HIP(timed(p, kTStage, stream, [&] { return launch_stage4d(p->p4->tile_x, p->p4->tile_y, kRhs, A, stream); }));
    return VP_OK;
}

vp_status p4_reduce(const vp_plan* p, const void* f, double* n, hipStream_t stream)
{
    const Plan4D& M = *p->p4;
    VP_HIP(timed(p, kTMoment, stream, [&] {
        return launch_moment4d(static_cast<const double*>(f), M.nx * M.ny, (size_t)M.nvx * M.nvy, M.dvx * M.dvy, n,
                               stream);
    }));
    return VP_OK;
}

vp_status p4_poisson(const vp_plan* p, const double* n, double* phi, double* E, hipStream_t stream)
{
    const Plan4D& M = *p->p4;
    VP_HIP(timed(p, kTField, stream, [&] {
        return launch_poisson2d(n, M.nx, M.ny, M.dx, M.dy, p->pb.qm, M.d_Qx, M.d_Qy, M.d_invlamT, M.d_g, phi, E,
                                nullptr, stream);
    }));
    return VP_OK;
}

vp_status p4_rk4(const vp_plan* p, void* f, double* a, double dt, void* work, hipStream_t stream)
{
    const Plan4D& M = *p->p4;
    double* fd = static_cast<double*>(f);
    double* acc = reinterpret_cast<double*>(wsp(work, p->ws_acc));
    double* s2 = reinterpret_cast<double*>(wsp(work, p->ws_fsa));
    double* s3 = reinterpret_cast<double*>(wsp(work, p->ws_fsb));
    double* n = reinterpret_cast<double*>(wsp(work, M.ws_n));
    double* g = reinterpret_cast<double*>(wsp(work, M.ws_E));
    const double* in[4] = {fd, s2, s3, s2};
    double* out[4] = {s2, s3, s2, fd};
    // the lean stage schedule (2 + 4 + 3 + 3 state words per cell): stage 2
    // adds dt/3 k2 to the accumulator, stage 4 dt/6 k4; the other slopes
    // are read back from the predictors
    const double cacc[4] = {0.0, dt / 3.0, 0.0, dt / 6.0};
    const double cnext[4] = {0.5 * dt, 0.5 * dt, dt, 0.0};
    const int kinds[4] = {kLean1, kLean2, kLean3, kLean4};
    Stage4DArgs A = base(p);
    A.fn = fd;
    A.acc = acc;
    A.a = a;
    A.n = n;
    for (int s = 0; s < 4; ++s) {
        A.fs = in[s];
        A.fout = out[s];
        A.c_acc = cacc[s];
        A.c_next = cnext[s];
        const int kind = kinds[s];
        VP_HIP(timed(p, kTStage, stream, [&] { return launch_stage4d(M.tile_x, M.tile_y, kind, A, stream); }));
        VP_HIP(timed(p, kTField, stream, [&] {
            return launch_poisson2d(n, M.nx, M.ny, M.dx, M.dy, p->pb.qm, M.d_Qx, M.d_Qy, M.d_invlamT, g, nullptr,
                                    nullptr, a, stream);
        }));
    }
    return VP_OK;
}

}  // namespace vp
