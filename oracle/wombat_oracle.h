/*
 * wombat_oracle.h -- serial FP64 CPU oracle for the WENO5 ideal-MHD stage.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path; it is
 * never called by the product path.  Only the tests, the smoke check and the
 * CPU baseline of the benchmark load it.  It shares no code, header, table or
 * helper with the HIP library.
 *
 * Method: Donnert et al., "Towards Exascale Simulations of the ICM Dynamo with
 * WENO-Wombat" (arXiv:1808.10633), Sec. 2.1: characteristic WENO5 finite
 * differences (eqs. 1-7), a Roe-type characteristic decomposition of the
 * eight MHD equations, Lax-Friedrichs flux splitting, a four-stage fourth-order
 * Runge-Kutta integrator and constrained transport of B.  The paper defers the
 * eigenvectors, the interface mean state, the CT averaging and the time-step
 * rule to unpublished papers; the readings adopted here are stated beside each
 * function.
 *
 * State layout (shared with the GPU library's contract, not its code):
 *   u[v][k][j][i], i fastest, v = (rho, mx, my, mz, Bx, By, Bz, E),
 *   dims (nx+2gx) x (ny+2gy) x (nz+2gz), g = 3 on an axis with n > 1, else 0.
 *   Point values at cell centres (finite differences, not cell averages).
 */
#ifndef WOMBAT_ORACLE_H
#define WOMBAT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, ny, nz;        /* interior cells; 1 marks an inactive axis        */
    double dx, dy, dz;     /* cell widths                                      */
    double gamma;          /* ratio of specific heats                          */
    double cfl;            /* Courant number for orc_cfl_dt                    */
    double eps;            /* WENO epsilon (the paper's value is 1e-6)         */
    int bc[6];             /* faces -x,+x,-y,+y,-z,+z: 0 periodic, 1 outflow   */
    int weights;           /* 0: weights of eq. (3); 1: WENO-Z (ablation)      */
    int lf_global;         /* 0: LF speed per stencil; 1: per sweep over the
                              whole box (ablation)                             */
    int b_face;            /* 0: B slots hold cell-centred B; 1: they hold the
                              staggered face-normal field, slot B_d of cell i
                              = b_d at its lower d-face i-1/2 (ablation;
                              periodic boxes)                                  */
} orc_grid;

/* ---- scalar WENO5 pieces (Sec. 2.1, eqs. 1-7) ---- */
void   orc_weno_weights(double a, double b, double c, double d, double eps,
                        double omega[3], double is[3]);
double orc_weno_phi(double a, double b, double c, double d, double eps);
/* WENO-Z weights (Borges et al. 2008, exponent 1): an ablation. */
void   orc_weno_weights_z(double a, double b, double c, double d, double eps,
                          double omega[3], double is[3]);
void   orc_interface_flux_z(const double Us[48], double gamma, double eps, double Fhat[8]);
/* The characteristic flux with given LF speeds alpha[0..6], one per field
 * (ablation: the global speeds of a sweep); z selects the WENO-Z weights. */
void   orc_interface_flux_alpha(const double Us[48], double gamma, double eps, int z,
                                const double alpha[7], double Fhat[8]);
/* Global LF speeds of the d-sweep: per field, the largest |lambda^s| over
 * every cell a stencil of that sweep reads (the 3-deep ghosts along d, one
 * transverse ghost layer on active transverse axes); zero on an inactive
 * axis. */
void   orc_lf_global(const orc_grid *g, const double *u, int d, double alpha[7]);
double orc_weno_field_flux(const double f[6], const double u[6],
                           double alpha, double eps);
/* eq. (1) for one field with the WENO-Z weights (ablation). */
double orc_weno_field_flux_z(const double f[6], const double u[6],
                             double alpha, double eps);

/* ---- ideal-MHD point functions (grid frame, 8 conserved variables) ---- */
void orc_prim_to_cons(const double W[8], double gamma, double U[8]);
void orc_cons_to_prim(const double U[8], double gamma, double W[8]);
void orc_flux(const double U[8], int dir, double gamma, double F[8]);
void orc_wave_speeds(const double U[8], int dir, double gamma,
                     double *cf, double *ca, double *cs);

/* ---- characteristic system in the sweep frame ---- */
/* Wn = (rho, vn, vt1, vt2, Bn, Bt1, Bt2, p); L, R row-major 8x8 over the
 * sweep-frame conserved vector (rho, mn, mt1, mt2, Bn, Bt1, Bt2, E). */
void orc_eigensystem(const double Wn[8], double gamma,
                     double lam[8], double L[64], double R[64]);
/* Us: 6 cells (i-2..i+3) of sweep-frame conserved variables, row-major 6x8.
 * Writes the sweep-frame interface flux at i+1/2. */
void orc_interface_flux(const double Us[48], double gamma, double eps,
                        double Fhat[8]);
/* As orc_interface_flux; common_alpha = 1 uses one LF speed
 * max(|v_n| + c_f) for every field; *dev (may be NULL) receives the largest
 * deviation of the weights of eq. (3) from (0.1, 0.6, 0.3) over all fields
 * and both sides. */
void orc_interface_flux_ex(const double Us[48], double gamma, double eps,
                           int common_alpha, double Fhat[8], double *dev);
/* Linear fifth-order component-wise flux with one LF speed (see the C file). */
void orc_linear_flux(const double Us[48], double gamma, double Fhat[8]);

/* ---- grid operations ---- */
long   orc_state_size(const orc_grid *g);          /* doubles in one state */
void   orc_fill_ghosts(const orc_grid *g, double *u);
int    orc_rhs(const orc_grid *g, const double *u, double *dudt);
int    orc_rhs_nofill(const orc_grid *g, const double *u, double *dudt);
int    orc_rhs_linear(const orc_grid *g, const double *u, double *dudt);
double orc_cfl_dt(const orc_grid *g, const double *u);
int    orc_rk4_step(const orc_grid *g, double *u, double dt);
/* Three-stage third-order strong-stability-preserving Runge-Kutta step
 * (Shu & Osher 1988): an ablation of the classical RK4 of Sec. 2.1.
 * Same contract as orc_rk4_step. */
int    orc_ssprk3_step(const orc_grid *g, double *u, double dt);
void   orc_sums(const orc_grid *g, const double *u, double out[8]);
int    orc_set_threads(int n);      /* OpenMP build: threads in use (serial build: 1) */
/* Staggered storage (b_face): the cell-centred state of a face-B state (its
 * ghosts filled), and the face divergence sum_d (b_d(i+1/2) - b_d(i-1/2))/dx_d
 * over the interior cells (max and mean of its magnitude). */
void   orc_face_to_cell(const orc_grid *g, const double *u, double *uc);
void   orc_divb_face(const orc_grid *g, const double *u, double *max_abs, double *l1);
void   orc_divb(const orc_grid *g, const double *u, double *max_abs,
                double *l1);

#ifdef __cplusplus
}
#endif
#endif
