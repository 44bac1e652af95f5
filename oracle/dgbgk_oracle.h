/*
 * dgbgk_oracle.h -- plain FP64 CPU oracle for the nodal discontinuous-Galerkin
 * discrete-Boltzmann BGK method (Ganeshan & Williams, "A finite element discrete
 * Boltzmann method for high Knudsen number flows", arXiv:2012.13487).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this library; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no source with the GPU library.
 *
 * Every routine is written from the paper's equations in the most direct form:
 * scalar loops, dense reference-element matrices, no blocking, fusion or
 * reordering.  Build with -O2 -ffp-contract=off so that each expression is
 * evaluated exactly as written.
 *
 * Conventions (shared *definitions*, not shared code):
 *   element  k = ex + nx*ey          (ex, ey: element column/row)
 *   node     n = i + (p+1)*j         (i along x, j along y; GLL points)
 *   velocity q = a + m*b for 2-D tensor sets (a indexes e_x, b indexes e_y)
 *   state    f[q][k][n], contiguous, FP64
 *   face     0 bottom (n=(0,-1)), 1 right (1,0), 2 top (0,1), 3 left (-1,0);
 *            a boundary face's side has the same number.
 */
#ifndef DGBGK_ORACLE_H
#define DGBGK_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_BC_PERIODIC 0
#define ORACLE_BC_DIFFUSE_WALL 1

typedef struct oracle_problem {
  int nx, ny;             /* elements per direction                         */
  double x0, y0, lx, ly;  /* domain [x0,x0+lx] x [y0,y0+ly]                  */
  int p;                  /* polynomial order, 1..8                          */
  int q;                  /* number of discrete velocities                  */
  const double *ex, *ey, *w; /* velocity set (copied at create)             */
  double theta;           /* RT in the second-order equilibrium             */
  double tau;             /* BGK relaxation time; +INF = collisionless      */
  int bc[4];              /* per side 0..3 (bottom,right,top,left)          */
  double wall_u[4][2];    /* wall velocity per side                         */
} oracle_problem;

typedef struct oracle oracle;

/* ---- velocity sets (1-D rules; the caller builds tensor products) ---- */
int oracle_gauss_hermite(int n, double *x, double *w);
int oracle_newton_cotes(int m, double vmax, double *x, double *w);
int oracle_tensor_set(int n, const double *x1, const double *w1,
                      double *ex, double *ey, double *w);
double oracle_second_moment(int q, const double *ex, const double *w);
double oracle_tau_from_kn(double kn, double L, int convention);

/* ---- reference element (1-D pieces, for pins) ---- */
int oracle_gll_nodes(int p, double *r);
int oracle_gauss_legendre(int n, double *x, double *w);

/* ---- solver ---- */
oracle *oracle_create(const oracle_problem *pb);
void oracle_destroy(oracle *o);
void oracle_set_threads(int nthreads);
int oracle_num_threads(void);
int oracle_sizes(const oracle *o, int *K, int *Np, int *Nfp, int *Q);
int oracle_operator(const oracle *o, int which, double *out);
int oracle_node_coords(const oracle *o, double *x, double *y);
int oracle_stable_dt(const oracle *o, double cfl, double *dt);
int oracle_set_state(oracle *o, const double *f);
int oracle_get_state(const oracle *o, double *f);
int oracle_init_equilibrium(oracle *o, double rho0, double ux0, double uy0);
int oracle_equilibrium(const oracle *o, double rho, double ux, double uy, double *feq);
int oracle_rhs(oracle *o, const double *f, double *k);
int oracle_rhs_parts(oracle *o, const double *f, double *vol, double *surf, double *coll);
int oracle_wall_density(oracle *o, const double *f, double *rho_w);
int oracle_rk4(oracle *o, long nsteps, double dt);
int oracle_moments(const oracle *o, double *rho, double *ux, double *uy);
int oracle_residual(oracle *o, double *r);
double oracle_total_mass(const oracle *o);
double oracle_couette_ux(double y, double L, double kn, double u_top, double u_bot);
double oracle_l2_error_couette(const oracle *o, double kn, double u_top, double u_bot);

#ifdef __cplusplus
}
#endif
#endif
