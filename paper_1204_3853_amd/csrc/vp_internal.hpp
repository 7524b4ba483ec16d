// Internal declarations shared by the host runtime and the HIP kernels of
// the MI355X Vlasov-Poisson library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "vp.h"

namespace vp {

// ----------------------------------------------------------------- errors

void set_error(const std::string& msg);
vp_status fail(vp_status code, const std::string& msg);
vp_status hip_fail(hipError_t e, const char* what);

#define VP_HIP(call)                                              \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::vp::hip_fail(e_, #call);   \
    } while (0)

// ----------------------------------------------------------------- launch shapes

// Stage kernel tile: NT threads, each owning W consecutive velocity cells,
// march over a segment of TX configuration rows of a TV = NT * W wide
// velocity strip.
struct StageShape {
    int nt;   // threads per block (multiple of 64)
    int w;    // cells per thread along v
    int tx;   // rows per segment
};

constexpr int kMaxTx = 128;          // bound on rows per segment (LDS moment buffer)
constexpr int kPoissonThreads = 256;
constexpr int kMaxPoisson1D = 8192;  // configuration cells handled by the one-block solver
constexpr int kGreenTaps = 16;       // taps of the truncated Green's function: r^17 ~ 3.6e-20

// Arguments of the 1D+1V stage kernels.  Pointers are element pointers of
// the plan dtype T (passed as void* and cast in the launcher).
struct Stage1DArgs {
    int nx, nv, tx, nstrip;
    double dxi, dvi, dv24, v_lo, dv;
    double vg[4];             // velocity ghosts j = -2, -1, nv, nv+1
    const void* fs;           // stage input state (read with halos)
    const void* fn;           // f^n (stages 2 and 3)
    void* acc;                // running f^n + dt sum b_s k_s
    void* fout;               // next predictor, f^{n+1}, or k
    const double* a;          // (q/m) E per x cell
    double* part;             // velocity-moment partial sums [nstrip][nx] (or null)
    double c_acc, c_next;     // dt b_s and dt alpha_{s+1}
};

enum StageKind : int { kRhs = 0, kStage1 = 1, kStage23 = 2, kStage4 = 3 };

// Arguments of the adjoint stage kernel (FP64, single level).
struct Adjoint1DArgs {
    int nx, nv, tx, nstrip;
    double dxi, dvi, dv24, v_lo, dv;
    double vg[4];
    const double* lam;      // cotangent of f^{n+1}
    const double* g_prev;   // g_{s+1} (null for s = 4)
    const double* z_prev;   // z_{s+1}, one value per x row (null for s = 4)
    const double* mu_in;    // running cotangent of f^n (null: start from lam)
    double* mu_out;
    const double* fs;       // stage state f(s)
    const double* a;        // its acceleration a(s)
    double* g_out;          // g_s
    double* part;           // per-strip partial sums of abar_s [nstrip][nx]
    double c1, c2;          // dt b_s, dt alpha_{s+1}
};

// Launchers (defined in vp_kernels_1d.hip).
hipError_t launch_stage1d(int dtype, const StageShape& sh, int kind, const Stage1DArgs& args,
                          hipStream_t stream);
hipError_t launch_moment_rows(int dtype, const void* f, int nx, int nv, double dv, double* n,
                              hipStream_t stream);
hipError_t launch_poisson1d(const double* part, int nstrip, const double* n_in, double dv,
                            int nx, double dx, double qm, const double* green, int gk,
                            double* n_out, double* phi, double* E, double* a,
                            hipStream_t stream);
// z = -dv S D (q/m) abar: the adjoint of the moment -> Poisson -> field chain
// applied to the per-strip partial sums of abar (finalised into abar_out)
// (part == null: abar_out already holds abar)
hipError_t launch_poisson1d_adjoint(const double* part, int nstrip, int nx, double dx, double dv, double qm,
                                    const double* green, int gk, double* abar_out, double* z, hipStream_t stream);
hipError_t launch_row_broadcast(const double* z, int nx, int nv, double* out, hipStream_t stream);
hipError_t launch_adjoint_stage1d(int w, bool first, const Adjoint1DArgs& a, hipStream_t stream);
hipError_t launch_adjoint_final(const double* mu, const double* g, const double* z, int nx, int nv, double* out,
                                hipStream_t stream);
hipError_t launch_scale(const double* x, double s, double* y, int n, hipStream_t stream);
hipError_t poisson1d_prepare();

}  // namespace vp

// ----------------------------------------------------------------- timing

// Per-launch HIP event pairs, recorded only while timing is enabled.
struct Timing {
    bool enabled = false;
    std::vector<hipEvent_t> ev;      // 2 * kMaxRecords events, created on enable
    std::vector<int> cls;            // kernel class of each recorded launch
    int used = 0;
    static constexpr int kMaxRecords = 8192;
};

// ----------------------------------------------------------------- the plan

struct vp_plan {
    vp_problem pb;
    std::vector<double> veq[VP_MAX_LEVELS][2];
    int ndim = 1, dtype = VP_F64, nlev = 1;
    size_t esize = 8;

    // single level 1D+1V geometry
    int nx = 0, nv = 0;
    double dx = 0, dv = 0, v_lo = 0;
    double vg[4] = {0, 0, 0, 0};

    vp::StageShape shape{128, 2, 32};
    int nstrip = 1;

    // periodic Green's function of the tridiagonal factor of the Poisson
    // operator (device), gk taps on each side
    double* d_green = nullptr;
    int gk = 0;

    // workspace layout (byte offsets)
    size_t ws_acc = 0, ws_fsa = 0, ws_fsb = 0, ws_part = 0, ws_cfg = 0, ws_total = 0;
    size_t ws_tmpf = 0, ws_stages = 0, ws_tmpa = 0;   // adjoint recompute (f_n copy, stage record)
    size_t state_elems = 0;

    mutable Timing timing;
};

namespace vp {
// Runs `launch` (returning hipError_t) bracketed by timing events of class cls.
template <typename F>
hipError_t timed(const vp_plan* p, int cls, hipStream_t stream, F&& launch)
{
    Timing& T = p->timing;
    if (!T.enabled || T.used >= Timing::kMaxRecords) return launch();
    const int r = T.used++;
    T.cls[r] = cls;
    hipError_t e = hipEventRecord(T.ev[2 * r], stream);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    return hipEventRecord(T.ev[2 * r + 1], stream);
}
enum TimingClass : int { kTStage = 0, kTField = 1, kTMoment = 2, kTSync = 3, kTAdjoint = 4, kTOther = 5 };
}  // namespace vp
