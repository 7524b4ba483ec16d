/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.  Declarations of the plain
 * FP64 reference implementation; not used by the GPU library.
 * Arrays are row-major [x][v] (v contiguous), all sizes in cells.
 */
#ifndef VP_ORACLE_H
#define VP_ORACLE_H

typedef struct vpo_poisson vpo_poisson;
typedef struct vpo_ctx {
    int nx, nv;
    double dx, dv, v_lo, qm;
    double vghost[4];      /* equilibrium cell averages at j = -2, -1, nv, nv+1 */
    vpo_poisson* P;
} vpo_ctx;

int vpo_num_threads(void);
void vpo_set_num_threads(int n);
void vpo_moment(int nx, int nv, double dv, const double* f, double* n);
vpo_poisson* vpo_poisson_new(int N);
void vpo_poisson_free(vpo_poisson* P);
void vpo_poisson_solve(const vpo_poisson* P, double dx, const double* rho, double* phi);
void vpo_field(int nx, double dx, const double* phi, double* E);
void vpo_rhs(int nx, int nv, double dx, double dv, double v_lo,
             const double* vghost, const double* f, const double* a, double* k);
void vpo_vboundary_flux(int nx, int nv, double dx, double dv,
                        const double* vghost, const double* f, const double* a,
                        double* g_lo, double* g_hi);

vpo_ctx* vpo_ctx_new(int nx, int nv, double x_len, double v_lo, double v_hi,
                     double qm, const double* vghost);
void vpo_ctx_free(vpo_ctx* c);
void vpo_constraints(const vpo_ctx* c, const double* f, double* a,
                     double* n_out, double* phi_out, double* E_out);
void vpo_rk4_step_stages(const vpo_ctx* c, const double* f_in, double* f_out, double dt,
                         double* stage_f, double* stage_a);
void vpo_rk4_step(const vpo_ctx* c, const double* f_in, double* f_out, double dt);
void vpo_rk4_step_fixed_a(const vpo_ctx* c, const double* f_in, double* f_out,
                          const double* a, double dt);

void vpo_rhs_adjoint(int nx, int nv, double dx, double dv, double v_lo,
                     const double* vghost, const double* f, const double* a,
                     const double* kbar, double* fbar, double* abar);
void vpo_constraints_adjoint(const vpo_ctx* c, const double* abar, double* fbar);
void vpo_rk4_adjoint_step(const vpo_ctx* c, const double* f_n, const double* lam_np1,
                          double* lam_n, double dt);

/* two-level hierarchy (vp_oracle_amr.c) */
void vpo_interp_weights(int R, double* out);
void* vpo_amr_new(int ncx, int ncv, double x_len, double v_lo, double v_hi, double qm, int R, int np,
                  int* boxes, double* veq_c, double* veq_f);
void vpo_amr_free(void* h);
long vpo_amr_state_size(void* h);
long vpo_amr_patch_offset(void* h, int p);
void vpo_amr_fill_ghosts(void* h, double* f, int p, double* out);
void vpo_amr_reduce_mask(void* h, double* f, double* n);
void vpo_amr_constraints(void* h, double* f, double* a, double* E_out);
void vpo_amr_rhs(void* h, double* f, double* a, double* k);
void vpo_amr_set_limited(void* h, int on);
void vpo_patch_fluxes_limited(int nx, int nv, const double* g, double dv, double v_lo, int col0,
                              const double* a_ext, double* Gx, double* Gv);
/* fluxes of section 2 on one patch from its data with two ghost layers g
 * ((nx+4) x (nv+4)): Gx[(nx+1) x nv], Gv[nx x (nv+1)]; a_ext[i+1] = a at row
 * i = -1 .. nx; and their divergence */
void vpo_patch_fluxes(int nx, int nv, const double* g, double dv, double v0, const double* a_ext,
                      double* Gx, double* Gv);
void vpo_divergence(int nx, int nv, const double* Gx, const double* Gv, double dx, double dv, double* k);

/* L-level hierarchy with per-level, per-direction ratios (vp_oracle_hier.c);
 * ratios[2(l-1)], ratios[2(l-1)+1]: x and v ratio of level l-1 -> l;
 * boxes: nbox x (level, lo_x, lo_v, hi_x, hi_v); veq_all: the equilibrium
 * with ghosts of every level, concatenated (nv_l + 4 each); *err != 0 and
 * NULL on a bad hierarchy */
void* vpo_hier_new(int L, int ncx, int ncv, double x_len, double v_lo, double v_hi, double qm, const int* ratios,
                   int nbox, const int* boxes, const double* veq_all, int* err);
void vpo_hier_free(void* h);
long vpo_hier_state_size(void* h);
long vpo_hier_patch_offset(void* h, int p);
void vpo_hier_fill_ghosts(void* h, const double* f, int p, double* out);
void vpo_hier_reduce_mask(void* h, const double* f, double* n);
void vpo_hier_constraints(void* h, const double* f, double* a, double* E_out);
void vpo_hier_rhs(void* h, const double* f, const double* a, double* k);
void vpo_hier_rk4_step(void* h, const double* f_in, double* f_out, double dt);
void vpo_hier_tag_values(void* h, const double* f, int l, double* values);
int vpo_hier_prolong_box(void* h, const double* f, int l, int x0, int v0, int x1, int v1, double* out);

/* two-level 2D+2V hierarchy (vp_oracle_amr4d.c): ncells[4] level-0 cells
 * (x, y, vx, vy), one ratio R in every direction, boxes: np x 8 (lo[4],
 * hi[4] in level-1 indices); a = [a_c (2 ncx ncy)][a_f (2 nfx nfy)] */
void* vpo_a4_new(const int* ncells, double x_len, double y_len, double v_lo, double v_hi, double qm, int R, int np,
                 const int* boxes, const double* gxc, const double* gyc, const double* gxf, const double* gyf);
void vpo_a4_free(void* h);
long vpo_a4_state_size(void* h);
long vpo_a4_patch_offset(void* h, int p);
void vpo_a4_fill_ghosts(void* h, const double* f, int p, double* out);
void vpo_a4_reduce_mask(void* h, const double* f, double* n);
void vpo_a4_constraints(void* h, const double* f, double* a, double* E_out);
void vpo_a4_rhs(void* h, const double* f, const double* a, double* k);
void vpo_a4_rk4_step(void* h, const double* f_in, double* f_out, double dt);

/* regridding (section 3): refinement criterion and conservative limited interpolation */
double vpo_tag_value(int nx, int nv, double dx, double dv, const double* vghost, const double* f, int i, int j);
void vpo_tag(int nx, int nv, double dx, double dv, const double* vghost, const double* f, double tol,
             unsigned char* tags);
void vpo_prolong1d(const double* u, int R, double* out);
void vpo_prolong_box(int ncx, int ncv, const double* fc, const double* vghost_c, int R, int fx0, int fv0, int fx1,
                     int fv1, double* out);

/* limited face averages (section 2, eq. limitedFace), 1D+1V single level */
double vpo_face_limited(double um1, double u0, double u1, double u2, int upwind_left);
void vpo_rhs_limited(int nx, int nv, double dx, double dv, double v_lo, const double* vghost, const double* f,
                     const double* a, double* k);
void vpo_rk4_step_limited(const vpo_ctx* c, const double* f_in, double* f_out, double dt);
void vpo_rk4_step_fixed_a_limited(const vpo_ctx* c, const double* f_in, double* f_out, const double* a, double dt);

/* 2D+2V single level, f[x][y][vx][vy]; a and E hold the x component, then y */
void* vpo4_ctx_new(int nx, int ny, int nvx, int nvy, double x_len, double y_len, double v_lo, double v_hi,
                   double qm, const double* veq_x, const double* veq_y);
void vpo4_ctx_free(void* h);
void vpo4_moment(void* h, double* f, double* n);
double vpo4_poisson(void* h, double* rho, double* phi);
void vpo4_field(void* h, double* phi, double* E);
void vpo4_constraints(void* h, double* f, double* a, double* phi_out, double* E_out);
void vpo4_rhs(void* h, double* f, double* a, double* k);
void vpo4_rk4_step(void* h, double* f_in, double* f_out, double dt);
void vpo4_rk4_step_fixed_a(void* h, double* f_in, double* f_out, double* a, double dt);
/* refinement criterion on a 2D+2V mesh (sums over x, y, vx, vy) */
double vpo4_tag_value(void* h, double* f, int i, int j, int k, int l);
void vpo4_tag(void* h, double* f, double tol, unsigned char* tags, double* values);
void vpo_amr_rk4_step(void* h, double* f_in, double* f_out, double dt);
/* subcycled two-level step: the coarse level takes dt with its own field,
 * the patches R substeps of dt/R (continuous extension of the coarse step
 * in time), then refluxing and the average-down */
void vpo_rk4_dense_weights(double theta, double* b);
void vpo_rk4_substage_weights(double theta0, double eta, int s, double* w);
void vpo_amr_subcycle_step(void* h, double* f_in, double* f_out, double dt);
/* several species, one two-level hierarchy each, the same finest
 * configuration mesh; rho = background + sum_s charge_s n_s */
void vpo_amr_species_constraints(int ns, void* const* hs, double* const* fs, const double* charge,
                                 double background, double* const* a);
void vpo_amr_species_rk4_step(int ns, void* const* hs, double* const* f_in, double* const* f_out,
                              const double* charge, double background, double dt);

#endif
