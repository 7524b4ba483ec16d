/*
 * vp.h -- C ABI of the MI355X (gfx950) Vlasov-Poisson library.
 *
 * The library advances the electrostatic Vlasov-Poisson system with
 * immobile ions (Hittinger & Banks, "Block-Structured Adaptive Mesh
 * Refinement Algorithms for Vlasov Simulation", section 2):
 *
 *     df/dt + v . grad_x f + (q/m) E . grad_v f = 0,
 *     E = -grad_x phi,  laplacian(phi) = int f dv - 1,
 *
 * discretised by the fourth-order finite-volume method of section 2
 * (cell averages, face averages with the ideal (unlimited) weights,
 * product-rule flux corrections, flux divergence) and integrated with the
 * classic four-stage RK4 scheme (eq. rk4), with the field re-solved at
 * every predictor state and after the update (Alg. smsvphu).  Phase space
 * is 1D+1V or 2D+2V; x is periodic; the velocity box is truncated.
 *
 * Conventions (every entry point):
 *   - Arrays are caller-owned device memory (e.g. torch tensors), passed
 *     as plain pointers; the library never allocates or frees them.
 *     Phase-space state f is row-major with the velocity index fastest:
 *     1D+1V f[x][v], 2D+2V f[x][y][vx][vy].  Its element type is the
 *     plan's dtype (double for VP_F64, float for VP_F32).  Configuration-
 *     space arrays (n, phi, E, a) are always double.
 *   - Work is only enqueued on `stream`; no call synchronises the device
 *     or the host.  Calls that share a plan may run concurrently only
 *     with distinct `work` buffers.
 *   - No call inside the time loop allocates device memory: scratch comes
 *     from the caller's `work` buffer of at least vp_workspace_bytes().
 *   - Errors: a vp_status is returned; VP_OK is 0.  Argument, shape and
 *     dtype errors are detected on the host before any launch, nothing is
 *     enqueued, and vp_last_error() returns a thread-local message.  No
 *     exception crosses the ABI and the library never aborts.
 */
#ifndef VP_H
#define VP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum vp_status {
    VP_OK = 0,
    VP_EINVAL = 1,     /* bad argument (null pointer, non-positive size, bad box) */
    VP_ESHAPE = 2,     /* sizes inconsistent with the plan                         */
    VP_EDTYPE = 3,     /* unsupported element type for this call                    */
    VP_ENOTSUP = 4,    /* valid request outside what this library supports          */
    VP_EHIP = 5,       /* a HIP runtime call failed                                 */
    VP_ENOMEM = 6      /* plan tables could not be allocated                        */
} vp_status;

typedef enum vp_dtype { VP_F64 = 0, VP_F32 = 1 } vp_dtype;

#define VP_MAX_LEVELS 4

/*
 * Problem statement (section 2 of the paper; the box hierarchy of
 * section 3).  Directions are ordered configuration first, then velocity:
 * 1D+1V (x, v), 2D+2V (x, y, vx, vy).
 *
 *   ndim      N = M, the number of configuration (= velocity) dimensions: 1 or 2
 *   dtype     element type of the phase-space state (vp_dtype)
 *   n_levels  1 (uniform mesh) .. VP_MAX_LEVELS (level 0 plus patches on
 *             levels 1 .. n_levels-1)
 *   cells     level-0 cells per direction
 *   ratio     ratio[l][d]: refinement ratio of level l -> level l+1 along
 *             direction d (configuration directions first, then velocity),
 *             l < n_levels - 1; section 4 runs [2,4], [4,2], [2,2]
 *   x_lo, x_len  periodic configuration box [x_lo, x_lo + x_len) per direction
 *   v_lo, v_hi   truncated velocity box per velocity direction
 *   qm        charge-to-mass ratio of the species (-1 for electrons)
 *   veq[l][d] host pointer: the cell averages of the unperturbed equilibrium
 *             along velocity direction d on level l, including two ghost
 *             cells on each side (cells_v(l) + 4 values, index 0 is j = -2).
 *             The velocity ghost cells of f hold these values (the
 *             characteristic boundary condition of section 2 with the
 *             equilibrium supplied on both ends); in 2D+2V the equilibrium
 *             is the product veq[l][0][j] * veq[l][1][k].  Copied at plan
 *             creation.
 * Single-level 2D+2V plans are FP64 with nx, ny <= 256, nvx <= 1024 and
 * fewer than 2^31 phase-space cells (VP_ENOTSUP otherwise).  Two-level 2D+2V plans (the hierarchy
 * of section 3 in the 2D+2V phase space) are FP64 with one ratio, 2 or 4,
 * in all four directions, the same velocity interval along vx and vy, and
 * a fine configuration mesh of at most 256 x 256 cells; their charge density
 * is the Mask reduction (Alg. mreduce) onto the fine configuration mesh,
 * where the Poisson equation is solved, and a holds [level-0 x][level-0
 * y][level-1 x][level-1 y] components, level 0 taking the mean of its
 * R x R fine values.
 */
typedef struct vp_problem {
    int32_t ndim;
    int32_t dtype;
    int32_t n_levels;
    int32_t cells[4];
    int32_t ratio[VP_MAX_LEVELS - 1][4];
    double x_lo[2];
    double x_len[2];
    double v_lo[2];
    double v_hi[2];
    double qm;
    const double* veq[VP_MAX_LEVELS][2];
} vp_problem;

/*
 * A patch on level `level` >= 1: inclusive cell range [lo, hi] per
 * direction in that level's global index space (section 3, box notation).
 * Level 0 always covers the whole domain and is implicit.  Patches must be
 * inside the domain (no periodic wrap inside one patch), aligned to the
 * refinement ratio of their parent level (lo and hi + 1 multiples of it)
 * and disjoint on their level (VP_EINVAL otherwise); a patch on level
 * l >= 2 must be nested in level l-1 with room for its ghost
 * interpolation.  Patches may touch, also across the periodic x boundary:
 * ghost cells that a neighbouring patch holds are copied from it (ghost
 * cells for inter-patch communication, section 3; Alg. mspsc), the others
 * interpolated from the parent level, so a fine-fine face gets the same
 * flux from both sides and only coarse-fine faces are corrected at the end
 * of a step.  1D+1V: FP64, up to VP_MAX_LEVELS levels with a ratio per
 * level and direction, a finest configuration mesh of at most 8192 cells.
 * 2D+2V: FP64, two levels (lo and hi hold x, y, vx, vy).
 */
typedef struct vp_box {
    int32_t level;
    int32_t lo[4];
    int32_t hi[4];
} vp_box;

typedef struct vp_plan vp_plan;

/* Creates an immutable plan: validates the problem and boxes, builds the
 * device tables (tile tables, coarse-fine maps, Poisson factors).  The
 * plan owns only these tables.  boxes may be NULL when nbox == 0. */
vp_status vp_plan_create(const vp_problem* problem, const vp_box* boxes, int32_t nbox,
                         vp_plan** out);
vp_status vp_plan_destroy(vp_plan* plan);
const char* vp_last_error(void);

/* Sizes derived from the plan.
 *   vp_state_elems   elements of a phase-space state f: level 0 followed by
 *                    each level-1 patch (in box order), each row-major.
 *   vp_patch_offset  element offset of patch p's data in f (p = -1: level 0)
 *   vp_config_elems  doubles of n, phi, E: the finest configuration mesh
 *   vp_field_elems   doubles of the acceleration array a: (q/m) E on every
 *                    level's configuration mesh (level 0 first)
 *   vp_workspace_bytes  minimum size of `work` for every call below
 *   vp_stage_elems   elements of the stage record of vp_rk4_step_record
 */
size_t vp_state_elems(const vp_plan* plan);
int64_t vp_patch_offset(const vp_plan* plan, int32_t patch);
size_t vp_config_elems(const vp_plan* plan);
size_t vp_field_elems(const vp_plan* plan);
size_t vp_workspace_bytes(const vp_plan* plan);
size_t vp_stage_elems(const vp_plan* plan);

/*
 * k = L(f; a): the semi-discrete right-hand side (section 2,
 * eq. semi-discrete) for every cell of every patch.
 *   f  state (plan dtype), vp_state_elems
 *   a  acceleration (q/m) E per level, vp_field_elems (from vp_inject_field)
 *   k  output, same layout and dtype as f; must not alias f
 * Ghost cells are synthesised: x periodic, velocity ghosts from veq, and on
 * level 1 the fifth-order conservative sub-cell interpolation of level 0,
 * along x then along v (section 3); level-1 ghosts outside the velocity
 * box take veq[1][0].
 */
vp_status vp_rhs(const vp_plan* plan, const void* f, const double* a, void* k,
                 hipStream_t stream);

/*
 * n = dv sum_j f_ij: the velocity moment (section 2; section 3,
 * reduction) on the finest configuration mesh.  On two levels the
 * Sub-Patch reduction is used: uncovered coarse columns are summed over
 * velocity, refined in x by the linear fifth-order sub-cell interpolant
 * and added to the fine-patch sums.  rho = 1 - n.
 *   n  output, vp_config_elems doubles
 */
vp_status vp_reduce_moment(const vp_plan* plan, const void* f, double* n, void* work,
                           hipStream_t stream);

/*
 * Face averages of the single-level 1D+1V scheme (section 2):
 *   VP_FACE_CENTERED  the ideal weights 1/2, 1/2: the centred fourth-order
 *                     face average (default)
 *   VP_FACE_LIMITED   eq. limitedFace: the left- and right-biased
 *                     third-order candidates (eqs. thirdLeft, thirdRight)
 *                     weighted by provisional WENO weights (Jiang-Shu
 *                     smoothness of the two stencils, ideal weights 1/2,
 *                     epsilon 1e-6, power 2), the larger weight given to
 *                     the upwind candidate (x faces: sign of the column's
 *                     velocity; v faces: sign of the row's acceleration)
 * The limited scheme is nonlinear: vp_rk4_step_record / vp_adjoint_step
 * return VP_ENOTSUP for it.  Two-level plans take it on both levels (the
 * coarse fluxes on coarse-fine faces included; synchronous and subcycled
 * steps); VP_ENOTSUP for plans of more than two levels and 2D+2V plans.
 * Not safe to call while calls on the plan are being enqueued.
 */
#define VP_FACE_CENTERED 0
#define VP_FACE_LIMITED 1
vp_status vp_face_scheme_set(vp_plan* plan, int32_t scheme);

/*
 * Reduction algorithm of a two-level plan (section 3):
 *   VP_REDUCE_SUBPATCH  Sub-Patch reduction (Alg. spreduce): the uncovered
 *                       coarse region is split into rectangles (Alg.
 *                       subdiv), each grown by two columns in x, summed
 *                       over its velocity range and refined in x
 *   VP_REDUCE_MASK      Mask reduction (Alg. mreduce): every coarse row is
 *                       refined in x, masked by the coverage of the target
 *                       column and summed over velocity
 *   VP_REDUCE_FUSED     the Mask reduction with its row sums formed by the
 *                       stage kernels (default): inside vp_rk4_step the
 *                       stages that produce a predictor also write the
 *                       velocity sums of its coarse and fine rows per tile
 *                       strip, and one kernel forms n from them (the masked
 *                       sum of a coarse row is its total less the cells
 *                       level 1 covers in the target column).  The field
 *                       after the end-of-step synchronisation (which changes
 *                       coarse cells next to coarse-fine faces), subcycled
 *                       steps and vp_reduce_moment compute n as
 *                       VP_REDUCE_SUBPATCH does (the cheaper of the two
 *                       without the stage kernels' sums).
 * All give the same n up to rounding; they differ in cost.  No effect on
 * single-level plans.  Not safe to call while calls on the plan are being
 * enqueued.
 */
#define VP_REDUCE_SUBPATCH 0
#define VP_REDUCE_MASK 1
#define VP_REDUCE_FUSED 2
vp_status vp_reduction_set(vp_plan* plan, int32_t algorithm);

/*
 * Periodic fourth-order Poisson problem of section 2 (discrete potential
 * equation, read with 12 dx^2 on the right-hand side) for rho = 1 - n,
 * with the null space projected out (sum rho = 0, zero-mean phi), and the
 * fourth-order cell-averaged field E = -D phi.
 *   n    input, vp_config_elems
 *   phi  output or NULL
 *   E    output or NULL (vp_config_elems per configuration direction,
 *        direction-major in 2D+2V)
 *   work unused (may be NULL); 2D+2V plans keep the Fourier coefficients
 *        in plan-owned device memory, so calls on one 2D+2V plan must be
 *        ordered on one stream
 */
vp_status vp_poisson_periodic(const vp_plan* plan, const double* n, double* phi, double* E,
                              void* work, hipStream_t stream);

/*
 * Injection (section 3, Alg. inject): a = (q/m) E on every level's
 * configuration mesh; the finest level takes E directly, level 0 the mean
 * of the ratio fine values covering each coarse cell.  The phase-space
 * kernels read a as a per-row scalar (the restricted hierarchy is used
 * directly, no phase-space copy).
 *   E  input, as written by vp_poisson_periodic
 *   a  output, vp_field_elems
 */
vp_status vp_inject_field(const vp_plan* plan, const double* E, double* a, hipStream_t stream);

/*
 * One synchronous RK4 Vlasov-Poisson step (Alg. smsvphu without
 * regridding), in place.
 *   f     state, overwritten with f^{n+1}
 *   a     on entry the acceleration of f (from vp_inject_field or the
 *         previous step); on exit that of f^{n+1} (the post-update
 *         constraint of Alg. smsvphu)
 *   dt    time step
 *   work  >= vp_workspace_bytes
 * On two levels the coarse level is advanced everywhere, the fine ghosts
 * are filled from the coarse predictor of the same stage, and at the end
 * the coarse cells next to coarse-fine faces take the fine accumulated
 * flux and covered coarse cells the average of the fine cells
 * (Alg. msfduc).
 */
vp_status vp_rk4_step(const vp_plan* plan, void* f, double* a, double dt, void* work,
                      hipStream_t stream);

/*
 * vp_rk4_step without a `work` argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It runs the same kernels as
 * vp_rk4_step with their workspace in a static device array of the library
 * (32 MiB, held on each device the library runs on until the process
 * ends), and calls no hipMalloc, hipFree or allocating routine.
 *   f, a, dt  as for vp_rk4_step
 * Single-level 1D+1V plans only (VP_ENOTSUP otherwise); VP_ESHAPE if the
 * step needs more than 32 MiB of workspace (FP64: up to about 1.3M cells,
 * e.g. 1024 x 1024).  Every call on one device shares that device's array
 * and leaves its contents behind: calls that overlap in time on one device
 * (several streams or threads) race and must be serialised by the caller.
 */
vp_status vp_rk4_step_noalloc(const vp_plan* plan, void* f, double* a, double dt,
                              hipStream_t stream);

/*
 * One subcycled step of a two-level plan: asynchronous time stepping, which
 * section 5 names as future work (citing the high-order subcycling of
 * McCorquodale and Colella); the reading taken here:
 *   1. the coarse level takes one RK4 step of dt on its own, with the field
 *      of its own velocity moment solved on the coarse configuration mesh
 *      (covered coarse cells hold the mean of their fine cells);
 *   2. the patches take R RK4 substeps of dt/R.  The coarse data of each
 *      fine stage (the source of the fine ghost cells and of the uncovered
 *      part of the composite moment) are the RK4 stage values taken on the
 *      Taylor expansion, at the substep start, of the third-order continuous
 *      extension of the coarse step; the field is the synchronous
 *      constraint of those coarse data and the fine predictor;
 *   3. the coarse cells next to coarse-fine faces take the fine fluxes
 *      averaged over the R substeps, and covered coarse cells the mean of
 *      their fine cells (Alg. msfduc).
 *   f     hierarchy state (layout of vp_rk4_step), overwritten
 *   a     in: any values (overwritten in the first stage); out: the
 *         acceleration of the new state (the synchronous constraint)
 *   dt    coarse time step (the patches take dt / R)
 *   work  >= vp_workspace_bytes
 * The plan's reduction algorithm (vp_reduction_set) applies to every fine
 * stage's composite moment; the launch mode does not apply (the coarse and
 * the fine tile ranges are each one persistent launch).
 * Errors: VP_EINVAL for a single-level plan, NULL pointers or a non-finite
 * dt.  Enqueued on `stream`; host-side it only sequences launches.
 */
vp_status vp_amr_subcycle_step(const vp_plan* plan, void* f, double* a, double dt, void* work,
                               hipStream_t stream);

/*
 * As vp_rk4_step (single level), and also records the stage states
 * f(2), f(3), f(4) and the four stage accelerations in `stages`
 * (vp_stage_elems elements of the plan dtype; the accelerations are
 * stored as doubles at the end, see vp_stage_elems) for a later
 * vp_adjoint_step.
 */
vp_status vp_rk4_step_record(const vp_plan* plan, void* f, double* a, double dt,
                             void* stages, void* work, hipStream_t stream);

/*
 * Discrete adjoint of one RK4 step (single level, FP64): lam_n =
 * (d f^{n+1} / d f^n)^T lam_np1 at the state f_n, including the adjoint of
 * the moment reduction, the Poisson solve, the field and the injection.
 *   f_n      state at the start of the step
 *   a_n      its acceleration
 *   stages   record written by vp_rk4_step_record from (f_n, a_n), or NULL
 *            to recompute the stages internally
 *   lam_np1  cotangent of f^{n+1}
 *   lam_n    output cotangent of f^n (may alias lam_np1)
 * VP_ENOTSUP for two-level or FP32 plans.
 */
vp_status vp_adjoint_step(const vp_plan* plan, const void* f_n, const double* a_n,
                          const void* stages, const void* lam_np1, void* lam_n, double dt,
                          void* work, hipStream_t stream);

/*
 * Adjoint of the map f -> a = (q/m) E(f) (velocity moment, periodic
 * Poisson solve, field, injection; section 2): fbar_ij = (K^T abar)_i for
 * every velocity cell j, where K f = a.  With the Poisson solution
 * operator S (symmetric) and the field stencil D (antisymmetric),
 * K^T abar = -dv S D (q/m) abar, broadcast over v.  Single level, FP64.
 *   abar  vp_field_elems doubles
 *   fbar  output state (FP64)
 */
vp_status vp_field_adjoint(const vp_plan* plan, const double* abar, void* fbar, void* work,
                           hipStream_t stream);

/*
 * Tile shapes of the stage kernels, for autotuning.  A shape is (threads
 * per block, velocity cells per thread, configuration rows per tile); on
 * 2D+2V plans it is (threads per block, configuration cells of the tile
 * along x, along y), one wavefront per configuration cell.
 * vp_tile_shape_count / _get enumerate the shapes compiled for the plan
 * (its dtype and number of levels); vp_tile_shape_set selects one for
 * every later call on the plan (results agree to rounding for every shape;
 * only speed changes).  On two levels a shape with two cells per thread
 * needs even patch widths in v (VP_EINVAL otherwise).  Not safe to call
 * while other calls on the same plan are being enqueued.
 */
int32_t vp_tile_shape_count(const vp_plan* plan);
vp_status vp_tile_shape_get(const vp_plan* plan, int32_t index, int32_t* threads, int32_t* cells,
                            int32_t* rows);
vp_status vp_tile_shape_set(vp_plan* plan, int32_t index);

/*
 * Launch structure of a two-level stage (the task-parallel overhead of
 * section 4 is what the persistent form removes):
 *   VP_LAUNCH_PERSISTENT  one launch per RK4 stage walks a tile table that
 *                         holds every tile of level 0, of every level-1
 *                         patch and the coarse-fine face chunks (default)
 *   VP_LAUNCH_PER_PATCH   one launch for level 0, one per patch and one for
 *                         the face chunks (the per-patch baseline)
 * Both run the same tiles with the same arithmetic: results are
 * bitwise identical.  No effect on single-level plans.
 */
#define VP_LAUNCH_PERSISTENT 0
#define VP_LAUNCH_PER_PATCH 1
vp_status vp_launch_mode_set(vp_plan* plan, int32_t mode);

/*
 * Autotuner: times `reps` RK4 steps (after one warm-up step) for every
 * tile shape valid for the plan, in three interleaved passes, keeps each
 * shape's fastest pass, selects the fastest shape with vp_tile_shape_set
 * and returns its index and mean step time in ms (either output may be
 * NULL).  f and a are used as scratch: they are advanced by 3 (reps + 1)
 * steps per shape, so pass copies of the state.  Unlike the other calls it
 * synchronises on its own timing events.
 */
vp_status vp_autotune(vp_plan* plan, void* f, double* a, double dt, int32_t reps, void* work,
                      hipStream_t stream, int32_t* best_index, float* best_ms);

/*
 * Kernel timing (a profiling aid, per-routine exclusive timers): while
 * enabled, every launch made by this plan is bracketed by a pair of HIP
 * events recorded on the launch's stream.  vp_timing_read synchronises on
 * those events, returns the accumulated milliseconds and launch counts of
 * each kernel class and clears them.  Classes: 0 stage / right-hand-side
 * kernels, 1 field solve (moment finalisation + Poisson + field),
 * 2 velocity moment, 3 coarse-fine synchronisation, 4 adjoint stage
 * kernels, 5 other.  At most 8192 launches are recorded between reads;
 * later launches run untimed.
 */
#define VP_TIMING_CLASSES 6
vp_status vp_timing_enable(vp_plan* plan, int32_t enable);
vp_status vp_timing_read(vp_plan* plan, double* ms, int64_t* counts, int32_t nclass);

/*
 * Regridding (section 3).
 *
 * vp_tag_cells: the refinement criterion of section 3 (mesh refinement
 * criteria) on level 0 of a 1D+1V FP64 plan (the single level, or the
 * coarse level of two): a cell is tagged when
 *   delta1 f + delta2 f > tol,
 *   delta1 f = [ 1/2 sum_d h_d (f(+e_d) - f(-e_d))^2 ]^(1/2),
 *   delta2 f = 1/2 sum_d h_d^2 |f(+e_d) - 2 f + f(-e_d)|,
 * summed over d = x, v (as printed), x periodic, velocity ghosts the
 * equilibrium; on a 2D+2V plan over d = x, y, vx, vy (the sums run over
 * the phase-space directions), x and y periodic, velocity ghosts the
 * equilibrium product.  The value is formed in a fixed order (directions
 * in the order listed) without fused multiply-adds and with a correctly
 * rounded square root, so that it is reproducible bit for bit.
 *   f       the state (level 0 is read)
 *   tags    output, device uint8 [ncx][ncv] (2D+2V: [nx][ny][nvx][nvy]):
 *           1 where tagged, else 0
 *   values  output or NULL: delta1 f + delta2 f per cell (double)
 * Enqueued on `stream`; VP_ENOTSUP for FP32 plans.
 */
vp_status vp_tag_cells(const vp_plan* plan, const void* f, double tol, uint8_t* tags, double* values,
                       hipStream_t stream);

/*
 * vp_cluster_tags (host, no device work): level-1 boxes that cover the
 * tagged level-0 cells, by Berger-Rigoutsos clustering (the paper leaves
 * the clustering to its AMR library): the bounding box of the tags is
 * split at a hole of a row or column signature, else at the strongest
 * inflection of a signature's second difference, else in the middle of
 * its longer side, until every box holds at least `efficiency` tagged
 * cells per cell or cannot be split into parts of `min_width` cells; every
 * box then grows by `buffer` cells (clipped to the domain), and boxes that
 * then overlap are merged into their bounding box.  Boxes may touch, also
 * across the periodic x boundary (a tagged region across x = x_lo is
 * covered by boxes at both ends of the x range).  The boxes are
 * returned in level-1 indices (level-0 box times `ratio`), sorted by
 * (x, v) origin, and satisfy vp_plan_create's rules.
 *   tags       host uint8 [ncx][ncv]
 *   boxes      output, room for max_boxes; *nbox receives the count
 * VP_EINVAL for bad sizes, efficiency outside (0, 1], or more than
 * max_boxes boxes (*nbox still holds the count).
 */
vp_status vp_cluster_tags(const uint8_t* tags, int32_t ncx, int32_t ncv, int32_t ratio, double efficiency,
                          int32_t min_width, int32_t buffer, vp_box* boxes, int32_t max_boxes, int32_t* nbox);

/*
 * Regridding of a multi-level plan (section 3, mesh refinement criteria;
 * the hierarchy is rebuilt from the coarsest level up, so a new level is
 * clustered from the tags of the new level below it).
 *
 * vp_tag_level: the criterion delta1 f + delta2 f > tol (as vp_tag_cells,
 *   with the level's cell sizes) on every cell that level `level` holds,
 *   neighbours outside a patch taken from its ghost cells.  tags: device
 *   uint8 [nx_l][nv_l] (0 where the level has no patch); values: device
 *   double [nx_l][nv_l] or NULL (NaN where the level has no patch).  work:
 *   the plan's workspace (its ghost-frame buffer is used).  VP_ENOTSUP for
 *   plans that are not multi-level.
 * vp_cluster_level (host): level-(level+1) boxes (level+1 index space,
 *   aligned to the ratios ratio_x, ratio_v of level -> level+1) covering
 *   the tagged level-`level` cells (tags: host uint8 [nx_l][nv_l]) that
 *   nesting allows: a cell is allowed when the plan's level `level` holds it
 *   and every cell within three cells of it (x periodic; outside the
 *   velocity box counts as held), so that the new level can be created
 *   over this plan's levels 0 .. level.  Berger-Rigoutsos as in
 *   vp_cluster_tags (efficiency, min_width and buffer in level-`level`
 *   cells); boxes that then hold disallowed cells are halved along their
 *   longer side until they do not (parts without tags dropped); boxes
 *   larger than max_x x max_v cells of the new level (0: no limit) are split
 *   into near-equal parts.  The boxes may touch.
 */
vp_status vp_tag_level(const vp_plan* plan, const void* f, int32_t level, double tol, uint8_t* tags, double* values,
                       void* work, hipStream_t stream);
vp_status vp_cluster_level(const vp_plan* plan, int32_t level, const uint8_t* tags, int32_t ratio_x, int32_t ratio_v,
                           double efficiency, int32_t min_width, int32_t buffer, int32_t max_x, int32_t max_v,
                           vp_box* boxes, int32_t max_boxes, int32_t* nbox);

/*
 * vp_regrid_transfer: fills the state of new_plan from the state of
 * old_plan after a regrid (section 3): level 0 is copied; every new
 * level-1 cell covered by an old level-1 patch takes the old fine value,
 * the others the conservative, limited, high-order interpolation of
 * level 0 (section 3, eqs. aux1, aux2, interp_r_avg with the
 * renormalisation; B^(0) = 2 D_i - D_{i+1}, the value the definition of
 * the candidate gives), applied in x and then in v.  Both plans are 1D+1V
 * FP64 with the same level 0 (cells, spacing, equilibrium) and the same
 * ratio; either may have one level.  f_old and f_new must not overlap.
 * Enqueued on `stream`.  Multi-level plans (both): level 0 copied, then
 * every finer level of new_plan from the coarsest: the cells an old patch
 * of the same level holds keep the old value, the others are that
 * interpolation of the new parent level with the level pair's ratios in x
 * and in v (anisotropic); VP_EINVAL if a new patch is not nested in its new
 * parent level; synchronises the stream (its tables are freed on return).
 */
vp_status vp_regrid_transfer(const vp_plan* old_plan, const void* f_old, const vp_plan* new_plan, void* f_new,
                             hipStream_t stream);

/*
 * Adaptive two-level run: the time loop of Alg. smsvphu with regridding
 * (section 3) and the time step control of the numerical results
 * (section 4), in the library.  A run owns the plan of its current
 * hierarchy and the device buffers of its state, field and workspace.
 *
 * Time step: dt = min(cap, cfl * L), L the linear stability limit of the
 * fourth-order scheme under RK4, the largest step with
 * dt (max|v| / dx + max|a| / dv) <= 2 sqrt(2) / max_t (8 sin t - sin 2t)/6
 * (about 2.0612) on every level (level 0 over the whole mesh; level 1 per
 * patch, over the patch's velocity faces and configuration columns);
 * cap = dt_initial for the first step, else dt_growth times the previous
 * step.  Regridding after every
 * regrid_interval steps: vp_tag_cells with tol, vp_cluster_tags with
 * efficiency, min_width and buffer, a new plan with the same problem and
 * the new boxes (default tile shape, launch mode and reduction),
 * vp_regrid_transfer, then the field of the new state.  A regrid that
 * finds exactly the current boxes keeps the current plan and state (the
 * transfer would copy every cell unchanged).
 */
typedef struct vp_amr_params {
    double tol;                /* refinement threshold of delta1 f + delta2 f (>= 0)   */
    int32_t regrid_interval;   /* steps between regrids (>= 1)                          */
    double efficiency;         /* clustering: tagged fraction of a box, (0, 1]         */
    int32_t min_width;         /* clustering: smallest split part, level-0 cells (>= 1) */
    int32_t buffer;            /* level-0 cells added around tagged regions (>= 0)     */
    double cfl;                /* fraction of the linear stability limit (> 0; 0.5)    */
    double dt_growth;          /* largest ratio of consecutive steps (>= 1; 1.1)       */
    double dt_initial;         /* first time step (> 0)                                 */
    int32_t max_size[VP_MAX_LEVELS][2];  /* largest patch on level l in its own cells
                                  (x, v); 0: no limit (multi-level runs only)            */
} vp_amr_params;

typedef struct vp_amr_info {
    double t;                  /* time reached                                           */
    double dt;                 /* last time step                                         */
    int64_t steps;             /* steps taken                                            */
    int32_t regrids;           /* regrids done                                           */
    int32_t npatch;            /* level-1 patches of the current hierarchy              */
    int64_t state_elems;       /* elements of the current state (vp_state_elems)        */
    double regrid_seconds;     /* host wall time spent in regrids (tag read-back,
                                  clustering, plan creation, transfer, field)            */
} vp_amr_info;

typedef struct vp_amr_run vp_amr_run;

/* Creates a run from a 1D+1V FP64 problem of two or more levels, its
 * initial boxes and the initial state f0 (device, the layout of
 * vp_plan_create(problem, boxes), copied).  Allocates device memory;
 * enqueues the copy and the field solve on `stream`.  A multi-level
 * problem (more than two levels, or different ratios in x and v) regrids
 * from the coarsest level up: level l of the new hierarchy is tagged
 * (vp_tag_level; level 0 on the old state, finer levels on the new levels
 * below them with their transferred state, or on the old plan and state
 * while those levels are the old ones box for box), clustered into level-(l+1)
 * boxes nested in it (vp_cluster_level with min_width, buffer, efficiency
 * and max_size[l+1]), and the new state transferred from the old one
 * (vp_regrid_transfer).  VP_EINVAL for bad parameters or a problem with
 * one level; plan creation errors as vp_plan_create. */
vp_status vp_amr_run_create(const vp_problem* problem, const vp_box* boxes, int32_t nbox, const void* f0,
                            const vp_amr_params* params, vp_amr_run** out, hipStream_t stream);
/* Advances `steps` time steps on `stream`.  A run of one species on a
 * multi-level plan keeps its time step and time in device memory: each
 * step's time step is computed on the device from the field (the same
 * rule and arithmetic as on the host) and the step's kernels read it
 * there, so the stream is synchronised only at a regrid and at the end of
 * the call.  Two-level plans and several species synchronise every step
 * (the time step needs max|a| on the host).  A regrid that changes the
 * boxes allocates the new plan and state and frees the old ones.  After an error the run should only be
 * destroyed. */
vp_status vp_amr_run_advance(vp_amr_run* run, int32_t steps, hipStream_t stream);
vp_status vp_amr_run_info(const vp_amr_run* run, vp_amr_info* info);
/* The plan of the current hierarchy (owned by the run; replaced at a regrid
 * that changes the boxes). */
const vp_plan* vp_amr_run_plan(const vp_amr_run* run);
/* The current boxes (level-1 index space); *nbox receives the count,
 * VP_EINVAL when it exceeds max_boxes. */
vp_status vp_amr_run_boxes(const vp_amr_run* run, vp_box* boxes, int32_t max_boxes, int32_t* nbox);
/* Copies the current state into dst (device, elems == vp_state_elems of
 * the current plan, else VP_ESHAPE); enqueued on `stream`. */
vp_status vp_amr_run_read_state(const vp_amr_run* run, void* dst, size_t elems, hipStream_t stream);
/* Waits for the device, frees the run's memory and plans.  NULL is a no-op. */
vp_status vp_amr_run_destroy(vp_amr_run* run);

/* A run of several species, each on its own two-level hierarchy that it
 * regrids from its own tags (section 1: one hierarchy per species), coupled
 * through the field of a species group (vp_species_group_create: rho =
 * background + sum_s charge[s] n_s, the same finest configuration mesh).
 * problems[s], boxes[s] (nbox[s] of them), f0[s]: as vp_amr_run_create per
 * species.  The time step takes the stability limit over every level of
 * every species.  vp_amr_run_info sums patches and state elements over the
 * species; the calls without a species index address species 0. */
vp_status vp_amr_run_create_species(int32_t nspecies, const vp_problem* const* problems, const vp_box* const* boxes,
                                    const int32_t* nbox, const void* const* f0, const double* charge,
                                    double background, const vp_amr_params* params, vp_amr_run** out,
                                    hipStream_t stream);
int32_t vp_amr_run_species_count(const vp_amr_run* run);
const vp_plan* vp_amr_run_plan_of(const vp_amr_run* run, int32_t species);
vp_status vp_amr_run_boxes_of(const vp_amr_run* run, int32_t species, vp_box* boxes, int32_t max_boxes,
                              int32_t* nbox);
vp_status vp_amr_run_read_state_of(const vp_amr_run* run, int32_t species, void* dst, size_t elems,
                                   hipStream_t stream);

/*
 * Several kinetic species on one configuration mesh.  Each species has its
 * own velocity range and mesh and, in the paper's design, its own
 * phase-space hierarchy; without collisions the species interact only
 * through the field (section 1, the motivation for one hierarchy per
 * species).  A group ties together 1D+1V plans of one dtype, single-level
 * or two-level (one hierarchy per species), whose finest configuration
 * meshes agree (cells, x_lo, x_len); each plan keeps its velocity mesh,
 * boxes, equilibrium ghost values and charge-to-mass ratio qm.
 * The charge density is
 *   rho = background + sum_s charge[s] n_s,   n_s the velocity moment of f_s,
 * (background: a uniform neutralising density; 1 with immobile ions of unit
 * density, 0 when every species is evolved), the field comes from rho by the
 * periodic Poisson solve and field stencil of section 2, and species s is
 * accelerated by a_s = qm_s E.  The group keeps pointers to the plans,
 * which must outlive it.  VP_EINVAL for NULL pointers, 0 or more than
 * VP_MAX_SPECIES species, non-finite charges or background, or plans that
 * differ in dtype or finest configuration mesh; VP_ENOTSUP for 2D+2V plans.
 */
#define VP_MAX_SPECIES 4
typedef struct vp_species_group vp_species_group;
vp_status vp_species_group_create(const vp_plan* const* plans, const double* charge, int32_t nspecies,
                                  double background, vp_species_group** out);
vp_status vp_species_group_destroy(vp_species_group* group);
/* bytes of the group workspace `gwork` of the calls below */
size_t vp_species_workspace_bytes(const vp_species_group* group);
/* a[s] = qm_s E of the states f[s] (f[s]: plan s's layout and dtype;
 * a[s]: vp_field_elems of plan s); enqueued on `stream`.  work may be NULL
 * when no species has two levels, else work[s] is plan s's workspace. */
vp_status vp_species_field(const vp_species_group* group, const void* const* f, double* const* a, void* const* work,
                           void* gwork, hipStream_t stream);
/* One RK4 step of every species in place (the lean stage schedule of
 * vp_rk4_step per species, one field solve from all species after every
 * stage).  a[s] in: the field of f (vp_species_field); out: the field of
 * the new states.  work[s]: plan s's workspace (vp_workspace_bytes).  A
 * two-level species takes the stages of vp_rk4_step and its end-of-step
 * synchronisation, its moment from its plan's reduction; its a[s] is the
 * injected [coarse][fine] array (vp_field_elems). */
vp_status vp_species_rk4_step(const vp_species_group* group, void* const* f, double* const* a, double dt,
                              void* const* work, void* gwork, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* VP_H */
