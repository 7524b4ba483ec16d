// Internal declarations shared by the host runtime and the HIP kernels of
// the MI355X Vlasov-Poisson library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstring>
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
constexpr int kMinStripCells = 64;   // the narrowest velocity strip of a two-level tile (64 threads x 1 cell)
constexpr int kPoissonThreads = 256;
constexpr int kMaxPoisson1D = 8192;  // configuration cells handled by the one-block solver
constexpr int kGreenTaps = 16;       // taps of the truncated Green's function: r^17 ~ 3.6e-20
constexpr int kFieldChunk = 256;     // configuration cells per block of the split field solve
constexpr int kFieldSplitMin = 1024; // smallest mesh that takes the split field solve

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
    int lim;                  // limited face averages (section 2) instead of the centred ones
};

// Stage kernels.  kStage1/23/4: the accumulator schedule (the accumulator
// is updated at every stage; 3 + 5 + 5 + 3 state words per cell and step).
// kLean1..4: the same classical RK4 step with 2 + 4 + 3 + 3 words, using
// that the predictors already hold the earlier slopes:
//   stage 1: f(2) = f^n + dt/2 k1
//   stage 2: f(3) = f^n + dt/2 k2,  acc = (f^n + f(2))/3 + dt/3 k2
//   stage 3: f(4) = f^n + dt k3
//   stage 4: f^{n+1} = acc + f(4)/3 + dt/6 k4
// since f(2)/3 = f^n/3 + dt/6 k1 and f(4)/3 = f^n/3 + dt/3 k3 (the three
// thirds of f^n add up to f^n); stage 4 does not read f^n.
enum StageKind : int { kRhs = 0, kStage1 = 1, kStage23 = 2, kStage4 = 3, kLean1 = 4, kLean2 = 5, kLean3 = 6, kLean4 = 7 };

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

// ----------------------------------------------------------------- 2D+2V

constexpr int kMaxPoisson2D = 256;    // configuration cells per direction of the 2D+2V path
constexpr int kPoisson2DSmall = 64;   // up to this many per direction: the two-kernel Poisson solve
constexpr int kMaxVy4D = 64;          // velocity cells along vy with one lane each; more: segments
constexpr int kSegVy4D = 60;          // vy cells per segment (64 lanes with two ghost lanes per side)
constexpr int kMaxVx4D = 1024;        // velocity cells along vx (equilibrium factors staged in LDS)

// Arguments of the 2D+2V stage kernel (FP64).
struct Stage4DArgs {
    int nx, ny, nvx, nvy;
    double dxi, dyi, dvxi, dvyi, dvx24, dvy24, vx_lo, vy_lo, dvx, dvy;
    const double* gx;          // 1D equilibrium along vx with ghosts (nvx + 4), device
    const double* gy;          // 1D equilibrium along vy with ghosts (nvy + 4), device
    const double* fs;
    const double* fn;
    double* acc;
    double* fout;
    const double* a;           // a_x (nx ny), then a_y
    double* n;                 // velocity moment of the output per configuration cell (or null)
    double c_acc, c_next, mscale;
};

// ----------------------------------------------------------------- two levels

struct AmrPatch {              // one level-1 patch
    long long off;             // element offset of its cells in the state
    long long foff;            // offset of its boundary-flux block: [x lo: nv][x hi: nv][v lo: nx][v hi: nx]
    int gx0, gv0;              // level-1 global index of its cell (0, 0)
    int nx, nv;                // cells
    int nb0, nb1;              // range of its neighbour list: patches holding some of its ghost cells
    long long fpart;           // its row sums per velocity strip in the fine partial buffer, [strip][row]
                               // (room for strips of 64 cells, the narrowest tile)
};

enum AmrTileKind : int { kTileCoarse = 0, kTileFine = 1, kTileFaces = 2 };
struct AmrTile {
    int kind;
    int p;                     // fine: patch; faces: first face
    int a;                     // coarse: tile index; fine: row segment; faces: face count
    int b;                     // fine: velocity strip
};

struct AmrFace {               // coarse face on a coarse-fine interface
    int i, j;                  // coarse cell on the low side ((i, j) | (i+1, j) or (i, j) | (i, j+1))
    int dir;                   // 0: x face, 1: v face
    int fine;                  // index in the fine boundary-flux buffer of the first of R fine faces
};

struct AmrArgs {
    Stage1DArgs coarse;        // the coarse level as a single-level problem (state base pointers)
    const AmrPatch* patches;
    const AmrTile* tiles;
    int ntiles;
    int nfx, nfv;              // level-1 index space
    int R, lr;                 // refinement ratio (same in x and v) and log2 R
    int tx;                    // rows per fine tile
    double dxfi, dvfi, dvf24, dvf, v_lo;
    double vgf[4];             // level-1 velocity ghosts j = -2, -1, nfv, nfv+1
    const double* a_f;         // level-1 acceleration (nfx)
    const double* B;           // sub-cell interpolation weights b_j(s) at B[s * 5 + j + 2] (device)
    const AmrFace* faces;
    const int* nb;             // neighbour lists (AmrPatch::nb0 .. nb1)
    double* cf_acc;            // accumulated coarse fluxes on the listed faces
    double* ff_acc;            // accumulated fine boundary fluxes
    double c_flux;             // b_s (0: no accumulation)
    int first;                 // first stage: store instead of add
    int lim;                   // limited face averages on both levels
    double* fpart;             // fine row sums of the new stage state per velocity strip (or null);
                               // the coarse ones go to coarse.part
};

// ----------------------------------------------------------------- two-level 2D+2V

struct A4Patch {               // level 0 (patch 0) or a level-1 patch of a two-level 2D+2V plan
    long long off;             // state offset, [x][y][vx][vy]
    long long pad;             // offset of its padded copy (two ghost layers per direction)
    long long foff;            // boundary flux blocks: x lo/hi [ny][nvx][nvy], y lo/hi [nx][nvx][nvy],
                               // vx lo/hi [nx][ny][nvy], vy lo/hi [nx][ny][nvx]
    int lo[4], sz[4];          // first cell (level index space) and cells per direction
    int lev, nb0, nb1, pad_;   // level; neighbour list range (patches holding some of its ghost cells)
    double isz[4], ipz[4];     // 1 / sz and 1 / (sz + 4), for index decoding
};

struct A4Level {
    int n[4];                  // index space
    double h[4], hi[4];        // cell sizes and their inverses
    double v_lo;
    int a_off;                 // offset of the level's a: [x component][y component], each n0 n1
};

constexpr int kA4VxRun = 2;  // cells along vx per thread of the two-level 2D+2V stage kernel

struct A4Face {                // a level-0 face on a coarse-fine interface
    int cell[4];               // the low cell (the face is its upper face along dir)
    int dir;
    int pad_;
};

struct A4Args {
    A4Level lv[2];
    const A4Patch* patches;
    const int* nb;
    const int* tiles;          // per tile: patch index and first thread (2 ints); a patch's threads
                               // are its (x, y, run of kA4VxRun vx cells, vy), vy fastest
    int ntiles;
    const double* pad;         // padded copies of the stage input
    const double* fn;
    double* acc;
    double* fout;
    const double* a;
    double* ff_acc;            // accumulated patch boundary fluxes
    const A4Face* faces;       // level-0 faces on coarse-fine interfaces: their fluxes go to cf
    int nfaces;                // (RK4 stages only; blocks after the tiles)
    double* cf;
    double c_acc, c_next, c_flux;
    int first;
};

struct A4Interp {              // separable sub-cell interpolation over one level-1 patch's padded box
    long long o[3];            // scratch offsets of its x, then y, then vx pass results
    int plo[4], pn[4];         // padded box: first fine cell and cells per direction
    int clo[4], cn[4];         // level-0 cells the passes read (stencils included)
    double ipn[4], icn[4];     // 1 / pn and 1 / cn, for index decoding
};

struct A4PadTiles {            // blocks of 256 elements of one patch: (patch, its first element)
    const int2* pad;           // padded copies, every patch in list order
    int npad;
    const int2* pass[3];       // interpolation passes: (level-1 patch's A4Interp index, first result)
    int npass[3];
};


hipError_t launch_a4_pad(const double* f, const A4Patch* patches, const int* list, int npatch, long long total,
                         const int* nb, const A4Level* lv_host, const double* B, int R, const double* gxc,
                         const double* gyc, const double* gxf, const double* gyf, const A4Interp* ip,
                         const A4PadTiles& tl, double* scratch, double* pad, hipStream_t stream);
hipError_t launch_a4_stage(int kind, const A4Args& a, hipStream_t stream);
// the Mask reduction's sums: masked plane sums of level 0 (M[t * 25 + s]) and
// level-1 row segments (M[25 ncx ncy + k]), one launch
hipError_t launch_a4_moment_sums(const double* f, const int* rp, const int4* rects, const int* n,
                                const long long* task_off, const int* task_len, int ntasks, double* M,
                                hipStream_t stream);
hipError_t launch_a4_inject(double* a, int ncx, int ncy, int R, hipStream_t stream);
hipError_t launch_a4_reflux(double* f, const long long* cell, const int* ptr, const int* code, const int* fine,
                            int nfine, const double* ff, const double* cf, const A4Face* faces, const double* hdt, double dt,
                            int ncorr, hipStream_t stream);
hipError_t launch_a4_average(double* f, const long long* dst, const long long* src, const int* strides, int R, int n,
                             hipStream_t stream);

// ----------------------------------------------------------------- multi-level hierarchies

constexpr int kHierLevels = VP_MAX_LEVELS;

struct HLevel {                // one level of a multi-level hierarchy
    int nx, nv;                // index space
    int rx, rv;                // ratio from the parent level (1 on level 0)
    int rt;                    // x ratio from this level to the finest
    int a_off;                 // offset of the level's acceleration in a
    double dxi, dvi, dv24, dv;
};

struct HPatch {                // a patch of a multi-level hierarchy (level 0 is patch 0)
    long long off;             // element offset of its cells in the state
    long long frame;           // its ghost frame: rows -2, -1, nx, nx+1 (nv + 4 each, column c <-> j = c - 2),
                               // then columns -2, -1, nv, nv+1 of each interior row
    long long foff;            // boundary-flux block: [x lo: nv][x hi: nv][v lo: nx][v hi: nx]
    int lev, gx0, gv0, nx, nv;
    int pad;
};

// Source of a frame cell or of a face-stencil value: src >= 0 is a state
// element; src < 0 the equilibrium ghost value eqv[-1 - src].
struct HInterp {               // a ghost cell interpolated from the parent level
    int src[25];               // parent cells (ci + a, cj + b) at src[(a + 2) * 5 + b + 2]
    int lev, s, t;             // the fine cell's level and its sub-cell position in x and v
};

struct HFace {                 // a face of level l on a coarse-fine interface with level l + 1
    int src[12];               // x face: cells (i-1 .. i+2) x (j-1 .. j+1) at src[(m + 1) * 4 + q],
                               // v face: cells (i-1 .. i+1) x (j-1 .. j+2) at src[(m + 1) * 4 + q]
    int dir, lev;              // 0: x face, 1: v face
    int ai[3];                 // v face: absolute indices of a at i-1, i, i+1
    int pad;
    double vb;                 // x face: cell-centre velocity of row j
};

struct HierArgs {
    HLevel lv[kHierLevels];
    const HPatch* patches;
    const AmrTile* tiles;
    int tx;                    // rows per tile
    double v_lo;
    const double* fs;          // stage input (whole hierarchy)
    const double* fn;
    double* acc;
    double* fout;
    const double* a;           // acceleration of every level
    const double* frame;       // ghost frames of fs
    const double* eqv;         // equilibrium ghost values, 4 per level (j = -2, -1, nv, nv+1)
    const HFace* faces;
    double* cf_acc;            // accumulated coarse fluxes on the listed faces
    double* ff_acc;            // accumulated patch boundary fluxes
    double c_acc, c_next, c_flux;
    int first;
    const double* dt;          // null: c_acc and c_next are the stage coefficients; else they are
                               // multiplied by the time step held in device memory at dt
};

struct HierSyncArgs {
    double* f;
    HLevel lv[kHierLevels];
    double dt;
    const double* dt_dev;      // non-null: the time step is read there instead
    const HFace* faces;
    const double* cf_acc;
    const double* ff_acc;
    const int* corr_ptr;       // per corrected cell: its faces corr_face[corr_ptr[k] .. corr_ptr[k+1])
    const int* corr_face;      // face index, negative (-1 - index) when the face is the cell's lower face
    const long long* corr_cell;
    const long long* corr_fine;  // per face: first of its fine faces in ff_acc
    const int* corr_nfine;       // per face: number of fine faces
    int ncorr;
};

struct HierAvgArgs {           // covered cells of one level take the mean of the next finer level
    double* f;
    const long long* dst;
    const long long* src;      // first fine cell
    const int* stride;         // fine row length
    int rx, rv, n;
};

// regridding of a multi-level hierarchy (vp_kernels_regrid.hip)
struct HProlongPatch {         // a new patch filled by prolongation of its new parent level
    long long off;             // the new patch's state offset
    int nv;                    // its velocity width
    int pcx, pcv;              // parent cells it covers
    int win;                   // offset of its (pcx + 4) x (pcv + 4) window sources in the source table
};
struct HCopyBlock {            // an intersection of a new patch with an old patch of the same level
    long long dst, src;        // its first cell in the new and in the old state
    int dst_stride, src_stride, nx, nv;
};
hipError_t launch_hier_tag(const double* f, const double* frame, const HPatch* d_patches, const int* d_list, int n,
                           int max_cells, int nv_l, double dx, double dv, double tol, uint8_t* tags, double* values,
                           hipStream_t stream);
hipError_t launch_hier_prolong(double* f, const int* d_win, const HProlongPatch* pp, int n, int max_parent_cells,
                               int rx, int rv, const double* eqv, hipStream_t stream);
hipError_t launch_hier_copy(double* fnew, const double* fold, const HCopyBlock* d_blocks, int n, int max_cells,
                            hipStream_t stream);

hipError_t launch_hier_fill(const double* f, const int2* desc, const HInterp* rec, const double* wts,
                            const int* wofs, const double* eqv, double* frame, int n, hipStream_t stream);
hipError_t launch_hier_stage(int w, int nt, int kind, const HierArgs& a, int t_begin, int t_end, int grid,
                             hipStream_t stream);
hipError_t launch_hier_rowsum(const double* f, const double* frame, const long long* task_off, const int* task_len,
                              int ntasks, double* slots, hipStream_t stream);
hipError_t launch_hier_inject(const double* E, const HLevel* lv, int L, double qm, double* a, int na,
                              hipStream_t stream);
hipError_t launch_hier_reflux(const HierSyncArgs& s, hipStream_t stream);
hipError_t launch_hier_average(const HierAvgArgs& s, hipStream_t stream);

// Optional inputs and outputs of the 1D Poisson kernel for two-level plans:
// the moment taken from a fixed-order weighted list over row-sum slots, and
// the injection onto both levels.
struct PoissonExtra {
    const double* slots;       // null: the kernel reads n
    const int* rowptr;
    const int* idx;
    const double* w;
    int inject_R;              // > 0: a = [(q/m) mean of R fine E per coarse cell][(q/m) E]
    const double* part;        // non-null: n_i = dv sum over the strips of part[s nx + i]
    int nstrip;
    double dv;
    double* n_out;             // non-null (with part): receives that n
    int inject_L;              // > 0: a of every level of a hierarchy, level l at inject_off[l]:
    int inject_off[kHierLevels];  // (q/m) times the mean of the inject_rt[l] fine E values of each cell
    int inject_rt[kHierLevels];
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
// several species on one configuration mesh: per species the per-strip
// partial sums of its velocity moment (or its moment, nstrip = 1) and the
// weight w_s (charge times the velocity cell width, or the charge)
constexpr int kMaxSpecies = 4;
struct SpeciesMoments {
    const double* part[kMaxSpecies];
    int nstrip[kMaxSpecies];
    double w[kMaxSpecies];
    int ns;
    double background;
};
// n_eff = 1 - rho with rho = background + sum_s w_s sum_strips part_s, the
// form the single-species field solves take (rho = 1 - n)
hipError_t launch_species_neff(const SpeciesMoments& m, int nx, double* n_eff, hipStream_t stream);
// arrays the split field solve writes: a[k] = qm[k] E; with inject_R > 0
// also the coarse acceleration of a two-level plan, inject_a[c] = inject_qm
// times the mean of the inject_R fine E values of coarse cell c
struct FieldOutputs {
    double* a[kMaxSpecies + 1];
    double qm[kMaxSpecies + 1];
    int n;
    double* inject_a;
    double inject_qm;
    int inject_R;
};
// moment from strip partials, Poisson, field and a = (q/m) E over many blocks
// (nx >= kFieldSplitMin); work holds nx + 4 ceil(nx / kFieldChunk) doubles
hipError_t launch_field_split(const double* part, int nstrip, int nx, double dv, double dx, double qm,
                              const double* green, double* work, double* a, hipStream_t stream);
// the same from the charge density of several species (rho = background +
// sum_s w_s sum_strips part_s), writing every array of `out`
hipError_t launch_field_split_species(const SpeciesMoments& m, int nx, double dx, const double* green, double* work,
                                      const FieldOutputs& out, hipStream_t stream);
// Poisson, field and the injection onto every level of a hierarchy (L <= 4
// levels; level l's cell holds rt[l] finest cells, its a starts at off[l])
// in one launch, for meshes below kFieldSplitMin cells
hipError_t launch_poisson1d_levels(const double* n_in, int nx, double dx, double qm, const double* green, int gk,
                                   double* E, double* a, int L, const int* off, const int* rt, hipStream_t stream);
// Poisson, field and two-level injection in one launch; the moment is n_in,
// or is finalised from the weighted list of x when x.slots is set
hipError_t launch_poisson1d_inject(const double* n_in, const PoissonExtra& x, int nx, double dx, double qm,
                                   const double* green, int gk, double* E, double* a, hipStream_t stream);
hipError_t poisson1d_prepare();

// 2D+2V launchers (vp_kernels_4d.hip)
// tx x ty configuration cells per block (4x4, 2x4, 4x2, 2x2), one wave per cell
hipError_t launch_stage4d(int tx, int ty, int kind, const Stage4DArgs& a, hipStream_t stream);
hipError_t launch_moment4d(const double* f, int ncfg, size_t plane, double scale, double* n, hipStream_t stream);
// g: 2 nx ny doubles of device scratch (the scaled Fourier coefficients, then
// the potential); Qy: the basis, followed by its transpose; nx, ny <= 256
hipError_t launch_poisson2d(const double* n, int nx, int ny, double dx, double dy, double qm, const double* Qx,
                            const double* Qy, const double* invlamT, double* g, double* phi, double* E, double* a,
                            hipStream_t stream);
// the same, and with a_coarse (R = 2 or 4, nx and ny <= 64, multiples of R) also
// the mean of the R x R fine accelerations over each cell of the coarse mesh
// of nx/R x ny/R cells, components one after the other
hipError_t launch_poisson2d_coarse(const double* n, int nx, int ny, double dx, double dy, double qm,
                                   const double* Qx, const double* Qy, const double* invlamT, double* g, double* phi,
                                   double* E, double* a, int R, double* a_coarse, hipStream_t stream);

// two-level launchers (vp_kernels_amr.hip)
hipError_t launch_amr_stage(int w, int nt, int kind, const AmrArgs& a, int t_begin, int t_end, int grid,
                            hipStream_t stream);
hipError_t launch_amr_rowsum(const double* f, const long long* task_off, const int* task_len, int ntasks,
                             double* slots, hipStream_t stream);
hipError_t launch_amr_reduce_finalize(const double* slots, const int* rowptr, const int* idx, const double* w,
                                      int nfx, double* n, hipStream_t stream);
// Mask reduction: S[i * 5 + a + 2] = sum over uncovered (i, j) of f_coarse(i + a, j)
hipError_t launch_amr_mask_rows(const double* f, const unsigned char* covered, int ncx, int ncv, double* S,
                                hipStream_t stream);
// Mask reduction from the stage kernel's strip partials (see k_amr_mask_fused)
struct AmrMaskFusedArgs {
    const double* f;           // the stage state (coarse level at offset 0)
    const double* part_c;      // coarse row sums, [strip][ncx]
    const double* part_f;      // fine row sums, per patch at AmrPatch::fpart, [strip][row]
    const AmrPatch* patches;
    const int* cov_ptr;        // per coarse column, its covered cells (ncx + 1 entries)
    const int* cov_j;          // their velocity indices
    const int* fz_ptr;         // per coarse column, its fine strip partials (ncx + 1 entries)
    const int2* fz_entry;      // (index in part_f, fine cell of the column 0 .. R-1), in a fixed order
    const double* B;           // b_j(s) at B[s * 5 + j + 2]
    int ncx, ncv, nstrip, R, tv;
    double dvc, dvf;
    double* n;                 // out: n on the fine configuration mesh
};
hipError_t launch_amr_mask_fused(const AmrMaskFusedArgs& a, hipStream_t stream);
hipError_t launch_amr_inject(const double* E, int ncx, int R, double qm, double* a, hipStream_t stream);
// end of step: coarse cells next to coarse-fine faces take the fine
// accumulated fluxes; covered coarse cells take the mean of their fine cells
struct AmrSyncArgs {
    double* f;                 // state (coarse level at offset 0)
    int ncv, R;
    const double* cf_acc;
    const double* ff_acc;
    const AmrFace* faces;
    const int* corr_ptr;       // CSR over corrected coarse cells
    const int* corr_face;      // face index, negated-minus-one when the cell is on the high side
    const int* corr_cell;      // coarse cell index of each CSR row
    int ncorr;
    const int* cov_cell;       // covered coarse cells
    const long long* cov_fine; // element offset of the first fine cell under each covered cell
    const int* cov_nv;         // row stride (patch width) of that fine block
    int ncov;
    double dtx, dtv;           // dt / dx_coarse, dt / dv_coarse
};
hipError_t launch_amr_sync(const AmrSyncArgs& a, hipStream_t stream);
// refinement criterion on a 2D+2V mesh (vp_kernels_regrid.hip)
struct Tag4DArgs {
    const double* f;           // [x][y][vx][vy]
    int nx, ny, nvx, nvy;
    const double* gx;          // vx equilibrium factors with ghosts (nvx + 4)
    const double* gy;          // vy equilibrium factors with ghosts (nvy + 4)
    double h[4];               // dx, dy, dvx, dvy
    double tol;
    unsigned char* tags;
    double* values;            // or null
};
hipError_t launch_tag4d(const Tag4DArgs& a, hipStream_t stream);
// subcycled steps: out = hist + sum_q c[q - 1] (hist[q stride] - hist), q = 1..4, over n elements
hipError_t launch_amr_substage(const double* hist, size_t n, size_t stride, const double c[4], double* out,
                               hipStream_t stream);

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

// ----------------------------------------------------------------- two-level plan

namespace vp {
struct AmrPlan {
    int ncx = 0, ncv = 0, R = 4, lr = 2, nfx = 0, nfv = 0;
    double dxc = 0, dvc = 0, dxf = 0, dvf = 0, v_lo = 0;
    double vgc[4] = {0, 0, 0, 0}, vgf[4] = {0, 0, 0, 0};
    std::vector<AmrPatch> patches;
    std::vector<AmrFace> faces;
    size_t total = 0, fflux = 0;
    // tile shape (threads, cells per thread, rows per tile) and launch mode
    int nt = 64, w = 2, tx = 8;
    int mode = 0;                                    // 0 persistent, 1 one launch per patch
    int ncoarse_tiles = 0, ntiles = 0, nstrip_c = 1;
    std::vector<AmrTile> tiles;
    std::vector<int> patch_tile_begin;               // per patch, plus the face chunks at the end
    std::vector<int> fcol_ptr, fcol_patch;           // the patches over each fine configuration column (CSR)
    int face_tile_begin = 0;
    // device tables: one allocation (d_tables) holds every table but the
    // tile table, which a tile shape change rebuilds
    void* d_tables = nullptr;
    AmrPatch* d_patches = nullptr;
    int* d_nb = nullptr;
    AmrTile* d_tiles = nullptr;
    AmrTile* d_tiles_run = nullptr;                  // the same tiles in the order of the one-launch stage
                                                     // (fine, coarse, faces; in d_tiles' allocation)
    AmrFace* d_faces = nullptr;
    double* d_B = nullptr;
    int ntasks = 0;
    long long* d_task_off = nullptr;
    int* d_task_len = nullptr;
    int* d_rowptr = nullptr;
    int* d_idx = nullptr;
    double* d_w = nullptr;
    int ncorr = 0, ncov = 0;
    int* d_corr_ptr = nullptr;
    int* d_corr_face = nullptr;
    int* d_corr_cell = nullptr;
    int* d_cov_cell = nullptr;
    long long* d_cov_fine = nullptr;
    int* d_cov_nv = nullptr;
    int nsub = 0;                                    // sub-patches of the coarse level (Alg. subdiv)
    // Mask reduction (Alg. mreduce): coverage mask, fixed-order lists over [S (5 ncx) | fine row sums]
    int reduce_mode = VP_REDUCE_FUSED;               // VP_REDUCE_SUBPATCH, VP_REDUCE_MASK or VP_REDUCE_FUSED
    int fine_task0 = 0;                              // first fine-row task in the task list
    unsigned char* d_mask = nullptr;
    int* d_rowptr_m = nullptr;
    int* d_idx_m = nullptr;
    double* d_w_m = nullptr;
    size_t ws_slots_m = 0;
    // the Mask reduction from the stage kernel's row sums: per coarse column
    // its covered cells (covc_ptr, ncx + 1 entries; covc_j their velocity
    // indices) and the fine strip partials of its fine cells (fz, rebuilt
    // with the tile table: the strips are the tiles'); the coarse and fine
    // strip partials in the workspace (ws_pc, ws_pf)
    int* d_covc_ptr = nullptr;
    int* d_covc_j = nullptr;
    void* d_fz = nullptr;
    int* d_fz_ptr = nullptr;
    int2* d_fz_entry = nullptr;
    size_t ws_pc = 0, ws_pf = 0;
    // Poisson table of the coarse configuration mesh (subcycled steps)
    double* d_green_c = nullptr;
    // workspace offsets; ws_hist: the five coarse states of a subcycled
    // step, hist_stride elements apart; ws_nc: the coarse moment
    size_t ws_cf = 0, ws_ff = 0, ws_slots = 0, ws_n = 0, ws_E = 0, ws_fld = 0;
    size_t ws_hist = 0, ws_nc = 0, hist_stride = 0;
};

// two-level 2D+2V plan (vp_amr4d.hip)
struct Amr4DPlan {
    int R = 2;
    int nc[4] = {}, nf[4] = {};
    A4Level lv[2] = {};
    std::vector<A4Patch> patches;                    // patch 0 is level 0
    size_t total = 0, pad_total = 0, fflux = 0;
    int ntiles = 0, nfaces = 0, ncorr = 0, ntasks = 0, navg = 0, ncfg = 0;
    void* d_tables = nullptr;
    A4Patch* d_patches = nullptr;
    int* d_list = nullptr;
    int* d_nb = nullptr;
    int* d_tiles = nullptr;
    double* d_B = nullptr;
    double *d_gxc = nullptr, *d_gyc = nullptr, *d_gxf = nullptr, *d_gyf = nullptr;
    A4Face* d_faces = nullptr;
    A4Interp* d_interp = nullptr;                    // per level-1 patch, the separable interpolation passes
    A4PadTiles ptiles{};                             // block tables of the padded copies and the passes
    double* d_rhs_scratch = nullptr;                 // pass results of vp_rhs calls
    int* d_rect_ptr = nullptr;                       // per level-0 column: its covered velocity rectangles
    int4* d_rects = nullptr;
    long long* d_task_off = nullptr;
    int* d_task_len = nullptr;
    int* d_rowptr = nullptr;
    int* d_idx = nullptr;
    double* d_w = nullptr;
    long long* d_corr_cell = nullptr;
    int* d_corr_ptr = nullptr;
    int* d_corr_code = nullptr;
    int* d_fine = nullptr;                           // per face: its R^3 fine faces in the boundary-flux buffer
    long long* d_avg_dst = nullptr;
    long long* d_avg_src = nullptr;
    int* d_avg_strides = nullptr;
    double *d_Qx = nullptr, *d_Qy = nullptr, *d_inv = nullptr;   // fine configuration mesh Fourier tables
    double* d_rhs_pad = nullptr;                     // padded copies for vp_rhs, which takes no workspace
    double* d_g = nullptr;                           // Fourier coefficients of vp_poisson_periodic calls
    size_t ws_pad = 0, ws_ff = 0, ws_cf = 0, ws_slots = 0, ws_n = 0, ws_g = 0, ws_interp = 0;
};

// multi-level plan (vp_hier.hip): L levels, a ratio per level and direction
struct HierPlan {
    int L = 2;
    bool tag_only = false;                           // patches, frames and level lists only (see hier_create)
    int na = 0;                                      // elements of a: every level's configuration mesh
    double dxf = 0;                                  // finest configuration cell
    HLevel lv[kHierLevels] = {};
    std::vector<HPatch> patches;                     // patch 0 is level 0
    std::vector<double> eqv;                         // 4 per level
    size_t total = 0, frame_elems = 0, fflux = 0;
    int nframe = 0, nfaces = 0;
    int nt = 64, w = 1, tx = 8;
    int ntiles = 0, face_tile_begin = 0;
    std::vector<AmrTile> tiles;
    void* d_tables = nullptr;
    AmrTile* d_tiles = nullptr;
    HPatch* d_patches = nullptr;
    int2* d_desc = nullptr;
    HInterp* d_rec = nullptr;
    double* d_wts = nullptr;
    int* d_wofs = nullptr;                           // per level: offsets of its x and v weight tables in d_wts
    double* d_eqv = nullptr;
    HFace* d_faces = nullptr;
    HLevel* d_lv = nullptr;
    int ntasks = 0;
    long long* d_task_off = nullptr;                 // >= 0: state offset; < 0: frame offset -1 - off
    int* d_task_len = nullptr;
    int* d_rowptr = nullptr;
    int* d_idx = nullptr;
    double* d_w = nullptr;
    int ncorr = 0;
    int* d_corr_ptr = nullptr;
    int* d_corr_face = nullptr;
    long long* d_corr_cell = nullptr;
    long long* d_corr_fine = nullptr;
    int* d_corr_nfine = nullptr;
    struct Avg {
        int rx = 1, rv = 1, n = 0;
        long long* d_dst = nullptr;
        long long* d_src = nullptr;
        int* d_stride = nullptr;
    };
    Avg avg[kHierLevels];                            // avg[l]: level-l cells covered by level l + 1
    double* d_rhs_frame = nullptr;                   // frames for vp_rhs, which takes no workspace
    std::vector<int> level_list;                     // patch indices grouped by level
    int level_begin[kHierLevels + 1] = {};           // level l: level_list[level_begin[l] .. level_begin[l+1])
    int level_max_cells[kHierLevels] = {};           // largest patch of each level, in cells
    int* d_level_list = nullptr;
    size_t ws_frame = 0, ws_cf = 0, ws_ff = 0, ws_slots = 0, ws_n = 0, ws_E = 0, ws_fld = 0;
};
}  // namespace vp

// ----------------------------------------------------------------- 2D+2V plan

namespace vp {
struct Plan4D {
    int nx = 0, ny = 0, nvx = 0, nvy = 0;
    double dx = 0, dy = 0, dvx = 0, dvy = 0, v_lo = 0;
    int tile_x = 4, tile_y = 4;                      // configuration cells per block of the stage kernel
    double* d_gx = nullptr;
    double* d_gy = nullptr;
    double* d_Qx = nullptr;
    double* d_Qy = nullptr;
    double* d_invlamT = nullptr;
    double* d_g = nullptr;                           // Fourier coefficients of vp_poisson_periodic calls
    size_t ws_n = 0, ws_E = 0;
};
}  // namespace vp

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
    int face_scheme = VP_FACE_CENTERED;

    // periodic Green's function of the tridiagonal factor of the Poisson
    // operator (device), gk taps on each side
    double* d_green = nullptr;
    int gk = 0;

    // workspace layout (byte offsets)
    size_t ws_acc = 0, ws_fsa = 0, ws_fsb = 0, ws_part = 0, ws_cfg = 0, ws_total = 0;
    size_t ws_step = 0;   // prefix of the workspace that a forward RK4 step uses (single-level 1D+1V)
    size_t ws_tmpf = 0, ws_stages = 0, ws_tmpa = 0;   // adjoint recompute (f_n copy, stage record)
    size_t state_elems = 0;

    mutable Timing timing;
    vp::AmrPlan* amr = nullptr;
    vp::Plan4D* p4 = nullptr;
    vp::HierPlan* hier = nullptr;
    vp::Amr4DPlan* a4 = nullptr;
};

namespace vp {
// the single-level 1D+1V RK4 step (lean stage schedule) of plan p on state
// f: tile shape, common stage arguments, the stage input and output states
// (the workspace ping-pong buffers, or the stage record st_f), the stage
// coefficients and kinds (vp_api.hip)
struct Rk4Setup1D {
    StageShape sh;
    Stage1DArgs A;
    const void* in[4];
    void* out[4];
    double* part;
    double c_acc[4], c_next[4];
    int kind[4];
};
Rk4Setup1D rk4_setup_1d(const vp_plan* p, void* f, void* work, double dt, void* st_f);
// the arguments of stage s (0..3) with the acceleration a
Stage1DArgs rk4_stage_args_1d(const Rk4Setup1D& R, int s, const double* a);

// host tables packed into one device allocation and one copy: add() records
// each table, commit() allocates, copies and sets the device pointers
struct TableArena {
    struct Item {
        void** dst;
        const void* src;
        size_t bytes, off;
    };
    std::vector<Item> items;
    size_t total = 0;
    template <typename T>
    void add(T** dst, const std::vector<T>& v)
    {
        *dst = nullptr;
        if (v.empty()) return;
        items.push_back(Item{reinterpret_cast<void**>(dst), v.data(), v.size() * sizeof(T), total});
        total += (v.size() * sizeof(T) + 255) & ~size_t(255);
    }
    hipError_t commit(void** base)
    {
        *base = nullptr;
        if (total == 0) return hipSuccess;
        std::vector<char> host(total, 0);
        for (const Item& it : items) std::memcpy(host.data() + it.off, it.src, it.bytes);
        hipError_t e = hipMalloc(base, total);
        if (e != hipSuccess) return e;
        e = hipMemcpy(*base, host.data(), total, hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
        for (const Item& it : items) *it.dst = static_cast<char*>(*base) + it.off;
        return hipSuccess;
    }
};

// two-level 2D+2V host sequences (vp_amr4d.hip)
vp_status a4_create(vp_plan* p, const vp_problem* pb, const vp_box* boxes, int nbox);
void a4_destroy(vp_plan* p);
vp_status a4_rhs(const vp_plan* p, const void* f, const double* a, void* k, hipStream_t stream);
vp_status a4_reduce(const vp_plan* p, const void* f, double* n, void* work, hipStream_t stream);
vp_status a4_poisson(const vp_plan* p, const double* n, double* phi, double* E, hipStream_t stream);
vp_status a4_inject(const vp_plan* p, const double* E, double* a, hipStream_t stream);
vp_status a4_rk4(const vp_plan* p, void* f, double* a, double dt, void* work, hipStream_t stream);
// real orthonormal Fourier basis and the symbol of the 1D fourth-order
// Poisson operator on an n-cell periodic mesh (vp_4d.hip)
std::vector<double> fourier_basis(int n);
std::vector<double> fourier_basis_and_transpose(int n);
std::vector<double> fourier_symbol(int n, double h);

// b_j(s) of the conservative fifth-order sub-cell interpolation for ratio R
// (section 3), R x 5 values at [s * 5 + j + 2] (vp_amr.hip)
std::vector<double> interp_table(int R);

// clustering (vp_regrid.hip): an inclusive box of cells of the level that is
// clustered, and Berger-Rigoutsos on a dense [x][v] tag field
struct CBox {
    int xlo, vlo, xhi, vhi;
    long long area() const { return (long long)(xhi - xlo + 1) * (vhi - vlo + 1); }
};
// summed-area table of a 0/1 mask of nx x nv cells ([x][v]): the cells set
// in a box in four lookups.  With `bounded`, the table covers only the
// bounding box of the set cells (none lie outside it), and a box is
// clipped to it first
struct TagSums {
    int x0 = 0, v0 = 0, nx = 0, nv = 0;              // the table's window: [x0, x0 + nx) x [v0, v0 + nv)
    std::vector<int> s;                              // s[(i + 1)(nv + 1) + j + 1] = cells set in the window's [0, i] x [0, j]
    TagSums(const std::vector<unsigned char>& m, int mx, int mv, bool bounded = false);
    long long count(int xlo, int vlo, int xhi, int vhi) const   // inclusive bounds
    {
        xlo = std::max(xlo - x0, 0);
        vlo = std::max(vlo - v0, 0);
        xhi = std::min(xhi - x0, nx - 1);
        vhi = std::min(vhi - v0, nv - 1);
        if (xlo > xhi || vlo > vhi) return 0;
        const size_t w = (size_t)nv + 1;
        return (long long)s[(xhi + 1) * w + vhi + 1] - s[xlo * w + vhi + 1] - s[(xhi + 1) * w + vlo] + s[xlo * w + vlo];
    }
};
void br_cluster(const std::vector<unsigned char>& tag, int nv, CBox B, double eff, int minw, std::vector<CBox>& out);
void br_cluster(const TagSums& T, CBox B, double eff, int minw, std::vector<CBox>& out);

// multi-level host sequences (vp_hier.hip)
// tag_only: build only what tagging a level and transferring a state into
// the plan need (patches, ghost frames, level lists); such a plan cannot step
vp_status hier_create(vp_plan* p, const vp_problem* pb, const vp_box* boxes, int nbox, bool tag_only = false);
void hier_destroy(vp_plan* p);
vp_status hier_rhs(const vp_plan* p, const void* f, const double* a, void* k, hipStream_t stream);
vp_status hier_reduce(const vp_plan* p, const void* f, double* n, void* work, hipStream_t stream);
vp_status hier_inject(const vp_plan* p, const double* E, double* a, hipStream_t stream);
// dt_dev: non-null, the time step is the value held there in device memory
// (written by an earlier launch on the stream; dt is then unused)
vp_status hier_rk4(const vp_plan* p, void* f, double* a, double dt, void* work, hipStream_t stream,
                   const double* dt_dev = nullptr);
// the time step control of the adaptive run on the device (section 4): the
// largest linearly stable step of a multi-level state's field a, every
// patch of every level over its own velocity faces and configuration
// columns; state[0] = dt = min(first ? dt_initial : growth state[0],
// cfl courant / rate), state[1] += dt
hipError_t launch_hier_dt(const double* a, const HPatch* patches, int npatch, const HLevel* lv, int L, double v_lo,
                          double courant, double cfl, double growth, double dt_initial, int first, double* state,
                          hipStream_t stream);
vp_status hier_set_shape(vp_plan* p, int nt, int w, int tx);
// ghost frames of state f into the workspace frame buffer
vp_status hier_fill_frames(const vp_plan* p, const double* f, void* work, hipStream_t stream);
// multi-level regridding (vp_hier_regrid.hip): the criterion on level l
// (dense [nx_l][nv_l] tags and optionally values, NaN where level l has no
// patch); the state of a new plan from an old one (level 0 copied, every
// finer level from the coarsest: old cells of the same level kept, the others
// prolonged from the new parent level); clustering of level-l tags into
// level-(l+1) boxes nested in plan p's level l
vp_status hier_tag_level(const vp_plan* p, const double* f, int l, double tol, uint8_t* d_tags, double* d_values,
                         void* work, hipStream_t stream);
vp_status hier_transfer(const vp_plan* old_plan, const double* f_old, const vp_plan* new_plan, double* f_new,
                        hipStream_t stream);
vp_status hier_cluster(const vp_plan* p, int l, const uint8_t* tags, int rx, int rv, double efficiency, int min_width,
                       int buffer, int max_x, int max_v, std::vector<vp_box>& out);
// a plan on the multi-level engine whatever its levels and ratios (vp_api.hip)
vp_status hier_plan_create(const vp_problem* pb, const vp_box* boxes, int nbox, vp_plan** out, bool tag_only = false);

// two-level host sequences (vp_amr.hip)
vp_status amr_create(vp_plan* p, const vp_problem* pb, const vp_box* boxes, int nbox);
void amr_destroy(vp_plan* p);
vp_status amr_rhs(const vp_plan* p, const void* f, const double* a, void* k, hipStream_t stream);
// partials: the stage kernel that wrote f also wrote its strip partials
// (amr_stage with partials), so the fused Mask reduction forms n from them
vp_status amr_reduce(const vp_plan* p, const void* f, double* n, void* work, hipStream_t stream,
                     bool partials = false);
vp_status amr_inject(const vp_plan* p, const double* E, double* a, hipStream_t stream);
vp_status amr_rk4(const vp_plan* p, void* f, double* a, double dt, void* work, hipStream_t stream);
// the pieces of amr_rk4: stage s (0..3) reading the acceleration a, its
// output state (the stage-4 output is f itself), and the end-of-step
// coarse-fine synchronisation (flux correction and average-down of f)
// partials: also write the strip partials of the new stage state's rows
// (the coarse ones at ws_pc, the fine ones at ws_pf)
vp_status amr_stage(const vp_plan* p, int s, void* f, const double* a, double dt, void* work, hipStream_t stream,
                    bool partials = false);
// whether stage s of a step takes the fused Mask reduction
bool amr_stage_partials(const vp_plan* p, int s);
void* amr_stage_output(const vp_plan* p, int s, void* f, void* work);
vp_status amr_end_sync(const vp_plan* p, void* f, double dt, void* work, hipStream_t stream);
vp_status amr_set_shape(vp_plan* p, int nt, int w, int tx);
// one subcycled step: the coarse level takes dt, the patches R substeps
vp_status amr_subcycle(const vp_plan* p, void* f, double* a, double dt, void* work, hipStream_t stream);
// Green's-function table of the periodic fourth-order Poisson solve on n cells
std::vector<double> poisson_green_table(int n);
// 2D+2V host sequences (vp_4d.hip)
vp_status p4_create(vp_plan* p, const vp_problem* pb);
void p4_destroy(vp_plan* p);
vp_status p4_rhs(const vp_plan* p, const void* f, const double* a, void* k, hipStream_t stream);
vp_status p4_reduce(const vp_plan* p, const void* f, double* n, hipStream_t stream);
vp_status p4_poisson(const vp_plan* p, const double* n, double* phi, double* E, hipStream_t stream);
vp_status p4_rk4(const vp_plan* p, void* f, double* a, double dt, void* work, hipStream_t stream);
}  // namespace vp

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
