/*
 * dgbgk_oracle.c -- plain FP64 CPU oracle for the nodal DG discrete-Boltzmann
 * BGK method of Ganeshan & Williams (arXiv:2012.13487).
 *
 * TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg are the only users.  It shares no code with the GPU library.
 *
 * What it computes (paper references are to sections, equations and tables):
 *   - discrete velocity sets: Gauss-Hermite rules (Sec. II.A, "Choice of
 *     discrete velocities", Table I) and Newton-Cotes rules with Maxwellian
 *     weighting (Sec. III.B), 2-D sets as tensor products;
 *   - the second-order Hermite equilibrium, eq. (5), and the discrete moments
 *     rho = sum_i f_i, rho u = sum_i e_i f_i (Sec. II.A);
 *   - the nodal DG discretisation of the discrete Boltzmann equation, eq. (6),
 *     in the strong form that is algebraically equal to the weak form eq. (10)
 *     on affine elements (volume term, upwind face flux lifted into the element,
 *     BGK collision), on uniform Cartesian quadrilaterals with tensor
 *     Gauss-Lobatto-Legendre nodes;
 *   - the Maxwell diffuse-reflection wall, eq. (8), imposed through the exterior
 *     state (Sec. II.B, "Implementation of boundary conditions");
 *   - explicit classical RK4 time marching (the conclusion allows explicit RK of
 *     any order; the paper's own runs use SDIRK);
 *   - the Couette closed form eq. (11) (with the corrections listed beside
 *     oracle_couette_ux) and the L2 error of Sec. III.A.
 *
 * Plain on purpose: the reference-element operators are dense matrices built
 * from a 2-D orthonormal Vandermonde matrix, the RHS is evaluated element by
 * element and velocity by velocity with dense matrix-vector products, and the
 * RK4 stages are stored separately.  Compile with -O2 -ffp-contract=off.
 */
#include "dgbgk_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* small dense linear algebra                                                 */
/* ------------------------------------------------------------------------- */

/* C(n x l) = A(n x m) * B(m x l), row-major. */
static void matmul(int n, int m, int l, const double *A, const double *B, double *C) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < l; ++j) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += A[i * m + k] * B[k * l + j];
      C[i * l + j] = s;
    }
}

/* Ainv = A^{-1} by Gauss-Jordan elimination with partial pivoting.  Returns 0
 * on success, -1 if A is numerically singular. */
static int invert(int n, const double *A, double *Ainv) {
  double *a = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(2 * n));
  if (!a) return -1;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) a[i * 2 * n + j] = A[i * n + j];
    for (int j = 0; j < n; ++j) a[i * 2 * n + n + j] = (i == j) ? 1.0 : 0.0;
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(a[r * 2 * n + c]) > fabs(a[piv * 2 * n + c])) piv = r;
    if (fabs(a[piv * 2 * n + c]) < 1e-300) { free(a); return -1; }
    if (piv != c)
      for (int j = 0; j < 2 * n; ++j) {
        double t = a[c * 2 * n + j];
        a[c * 2 * n + j] = a[piv * 2 * n + j];
        a[piv * 2 * n + j] = t;
      }
    double d = a[c * 2 * n + c];
    for (int j = 0; j < 2 * n; ++j) a[c * 2 * n + j] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double fct = a[r * 2 * n + c];
      if (fct == 0.0) continue;
      for (int j = 0; j < 2 * n; ++j) a[r * 2 * n + j] -= fct * a[c * 2 * n + j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Ainv[i * n + j] = a[i * 2 * n + n + j];
  free(a);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* orthogonal polynomials                                                     */
/* ------------------------------------------------------------------------- */

/* Legendre P_n(x) and P_n'(x) by the three-term recurrence
 * (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1} and P'_{k+1} = P'_{k-1} + (2k+1) P_k. */
static void legendre(int n, double x, double *P, double *dP) {
  if (n == 0) { *P = 1.0; *dP = 0.0; return; }
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    double d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *P = p1;
  *dP = d1;
}

/* Orthonormal Legendre polynomial on [-1,1] (integral of its square is 1) and
 * its derivative. */
static void legendre_orthonormal(int n, double x, double *P, double *dP) {
  double p, dp;
  legendre(n, x, &p, &dp);
  double s = sqrt((2.0 * n + 1.0) / 2.0);
  *P = s * p;
  *dP = s * dp;
}

/* Probabilists' Hermite polynomial He_n(x): He_{k+1} = x He_k - k He_{k-1}. */
static double hermite_e(int n, double x) {
  if (n == 0) return 1.0;
  double h0 = 1.0, h1 = x;
  for (int k = 1; k < n; ++k) {
    double h2 = x * h1 - k * h0;
    h0 = h1;
    h1 = h2;
  }
  return h1;
}

/* ------------------------------------------------------------------------- */
/* velocity sets                                                              */
/* ------------------------------------------------------------------------- */

/* n-point Gauss-Hermite rule for the standard normal density
 * phi(x) = exp(-x^2/2)/sqrt(2 pi) (RT = 1), weights summing to one.  These are
 * the 1-D rules of Table I (D1Q4, D1Q5, D1Q6, ...) and of the D2Q9 set.
 * Nodes: the n roots of He_n, bracketed by sign changes on a fine grid,
 * bisected, then polished by Newton (He_n' = n He_{n-1}).
 * Weights: w_i = n! / (n^2 He_{n-1}(x_i)^2). */
int oracle_gauss_hermite(int n, double *x, double *w) {
  if (n < 1 || n > 40 || !x || !w) return -1;
  double L = sqrt(4.0 * n + 2.0) + 0.5; /* all roots lie in (-L, L) */
  int ngrid = 4000 * n + 1;             /* odd: x = 0 is never a grid point */
  int found = 0;
  double xa = -L, fa = hermite_e(n, xa);
  for (int g = 1; g <= ngrid && found < n; ++g) {
    double xb = -L + 2.0 * L * g / ngrid;
    double fb = hermite_e(n, xb);
    if ((fa < 0.0) != (fb < 0.0)) {
      double lo = xa, hi = xb, flo = fa;
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double fm = hermite_e(n, mid);
        if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
      }
      double r = 0.5 * (lo + hi);
      for (int it = 0; it < 3; ++it) {
        double d = n * hermite_e(n - 1, r);
        if (d == 0.0) break;
        double rn = r - hermite_e(n, r) / d;
        if (rn > lo && rn < hi) r = rn;
      }
      x[found++] = r;
    }
    xa = xb;
    fa = fb;
  }
  if (found != n) return -2;
  double nfact = 1.0;
  for (int k = 2; k <= n; ++k) nfact *= k;
  for (int i = 0; i < n; ++i) {
    double h = hermite_e(n - 1, x[i]);
    w[i] = nfact / ((double)n * (double)n * h * h);
  }
  return 0;
}

/* m-point composite Newton-Cotes (trapezoid) rule on [-vmax, vmax] with
 * Maxwellian weighting (Sec. III.B: equally spaced nodes; weights proportional
 * to the node's quadrature coefficient times the Maxwellian at the node),
 * normalised to sum to one.  vmax is in units of sqrt(RT). */
int oracle_newton_cotes(int m, double vmax, double *x, double *w) {
  if (m < 2 || !(vmax > 0.0) || !x || !w) return -1;
  double h = 2.0 * vmax / (m - 1);
  double sum = 0.0;
  for (int j = 0; j < m; ++j) {
    x[j] = vmax * (double)(2 * j - (m - 1)) / (double)(m - 1);
    double c = (j == 0 || j == m - 1) ? 0.5 : 1.0;
    w[j] = h * c * exp(-0.5 * x[j] * x[j]) / sqrt(2.0 * M_PI);
    sum += w[j];
  }
  for (int j = 0; j < m; ++j) w[j] /= sum;
  return 0;
}

/* 2-D tensor-product set (Sec. II.A: "2D quadratures ... as tensor products of
 * the 1D quadratures"): q = a + n b, e_q = (x_a, x_b), w_q = w_a w_b. */
int oracle_tensor_set(int n, const double *x1, const double *w1, double *ex, double *ey,
                      double *w) {
  if (n < 1) return -1;
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < n; ++a) {
      ex[a + n * b] = x1[a];
      ey[a + n * b] = x1[b];
      w[a + n * b] = w1[a] * w1[b];
    }
  return 0;
}

/* sum_q w_q e_qx^2: the discrete RT that makes eq. (5) conserve mass and
 * momentum exactly under the discrete moment sums. */
double oracle_second_moment(int q, const double *ex, const double *w) {
  double s = 0.0;
  for (int i = 0; i < q; ++i) s += w[i] * ex[i] * ex[i];
  return s;
}

/* Relaxation time from the Knudsen number, eq. (7) with c_s = 1:
 *   convention 0: tau = Kn L / sqrt(3);
 *   convention 1: the same with Kn multiplied by sqrt(pi/6) (the Kim-Pitsch
 *                 mean free path named after eq. (7)), i.e. tau = Kn L / sqrt(pi/2). */
double oracle_tau_from_kn(double kn, double L, int convention) {
  if (convention == 0) return kn * L / sqrt(3.0);
  if (convention == 1) return kn * L / sqrt(M_PI / 2.0);
  return NAN;
}

/* ------------------------------------------------------------------------- */
/* 1-D node sets                                                              */
/* ------------------------------------------------------------------------- */

/* Gauss-Lobatto-Legendre nodes on [-1,1]: the end points and the roots of
 * P_p'.  Newton on P_p' with P_p'' from Legendre's equation
 * (1-x^2) P'' = 2 x P' - p(p+1) P; start from Chebyshev-Gauss-Lobatto points. */
int oracle_gll_nodes(int p, double *r) {
  if (p < 1 || p > 32) return -1;
  r[0] = -1.0;
  r[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double x = -cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, x, &P, &dP);
      double d2P = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);
      double dx = dP / d2P;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    r[i] = x;
  }
  return 0;
}

/* n-point Gauss-Legendre rule on [-1,1] (for the L2 error quadrature). */
int oracle_gauss_legendre(int n, double *x, double *w) {
  if (n < 1 || n > 64) return -1;
  for (int i = 0; i < n; ++i) {
    double z = -cos(M_PI * (i + 0.75) / (n + 0.5));
    double P = 0.0, dP = 1.0;
    for (int it = 0; it < 100; ++it) {
      legendre(n, z, &P, &dP);
      double dz = P / dP;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    legendre(n, z, &P, &dP);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dP * dP);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* solver state                                                               */
/* ------------------------------------------------------------------------- */

struct oracle {
  oracle_problem pb;
  double *ex, *ey, *w;
  int K, Np, Nfp, Q, p;
  double hx, hy, rx, sy, J;
  double sJ[4], Fscale[4], nxf[4], nyf[4];
  int *Fmask; /* [4][Nfp]   element node on each face, increasing i or j */
  int *nbr;   /* [K][4]     neighbour element across each face, -1: wall */
  double *r;  /* [p+1]      GLL nodes */
  double *V1, *M1;            /* 1-D Vandermonde, 1-D mass matrix */
  double *Dr, *Ds, *M, *LIFT; /* 2-D reference operators */
  double *f;                  /* state [Q][K][Np] */
  double *k1, *k2, *k3, *k4, *tmp;
  double *rho, *ux, *uy; /* [K*Np] */
  double *rhow;          /* [K][4][Nfp] */
};

static int g_threads = 1;

void oracle_set_threads(int nthreads) {
  g_threads = nthreads > 0 ? nthreads : 1;
#ifdef _OPENMP
  omp_set_num_threads(g_threads);
#endif
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return g_threads;
#else
  return 1;
#endif
}

void oracle_destroy(oracle *o) {
  if (!o) return;
  free(o->ex); free(o->ey); free(o->w);
  free(o->Fmask); free(o->nbr); free(o->r);
  free(o->V1); free(o->M1); free(o->Dr); free(o->Ds); free(o->M); free(o->LIFT);
  free(o->f); free(o->k1); free(o->k2); free(o->k3); free(o->k4); free(o->tmp);
  free(o->rho); free(o->ux); free(o->uy); free(o->rhow);
  free(o);
}

static double *dalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

/* Build the 2-D reference-element operators from the orthonormal tensor
 * Legendre basis P_a(r) P_b(s) on the (p+1)^2 GLL nodes (Sec. II.B: nodal
 * Lagrange basis of degree p per direction):
 *   Dr = Vr V^{-1}, Ds = Vs V^{-1}, M = (V V^T)^{-1},
 *   E  = face mass matrices placed on each face's nodes, LIFT = M^{-1} E. */
static int build_reference_element(oracle *o) {
  int p = o->p, n1 = p + 1, Np = o->Np, Nfp = o->Nfp;
  o->r = dalloc(n1);
  if (oracle_gll_nodes(p, o->r)) return -1;

  /* 1-D Vandermonde and mass matrix (face mass). */
  o->V1 = dalloc((size_t)n1 * n1);
  o->M1 = dalloc((size_t)n1 * n1);
  double *VVt1 = dalloc((size_t)n1 * n1);
  for (int i = 0; i < n1; ++i)
    for (int a = 0; a < n1; ++a) {
      double P, dP;
      legendre_orthonormal(a, o->r[i], &P, &dP);
      o->V1[i * n1 + a] = P;
    }
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      double s = 0.0;
      for (int a = 0; a < n1; ++a) s += o->V1[i * n1 + a] * o->V1[j * n1 + a];
      VVt1[i * n1 + j] = s;
    }
  if (invert(n1, VVt1, o->M1)) { free(VVt1); return -1; }
  free(VVt1);

  /* 2-D Vandermonde: row = node n = i + n1 j, column = mode c = a + n1 b. */
  double *V = dalloc((size_t)Np * Np), *Vr = dalloc((size_t)Np * Np),
         *Vs = dalloc((size_t)Np * Np), *Vinv = dalloc((size_t)Np * Np),
         *VVt = dalloc((size_t)Np * Np);
  for (int j = 0; j < n1; ++j)
    for (int i = 0; i < n1; ++i)
      for (int b = 0; b < n1; ++b)
        for (int a = 0; a < n1; ++a) {
          double Pa, dPa, Pb, dPb;
          legendre_orthonormal(a, o->r[i], &Pa, &dPa);
          legendre_orthonormal(b, o->r[j], &Pb, &dPb);
          int n = i + n1 * j, c = a + n1 * b;
          V[n * Np + c] = Pa * Pb;
          Vr[n * Np + c] = dPa * Pb;
          Vs[n * Np + c] = Pa * dPb;
        }
  int rc = invert(Np, V, Vinv);
  o->Dr = dalloc((size_t)Np * Np);
  o->Ds = dalloc((size_t)Np * Np);
  o->M = dalloc((size_t)Np * Np);
  if (!rc) {
    matmul(Np, Np, Np, Vr, Vinv, o->Dr);
    matmul(Np, Np, Np, Vs, Vinv, o->Ds);
    for (int i = 0; i < Np; ++i)
      for (int j = 0; j < Np; ++j) {
        double s = 0.0;
        for (int c = 0; c < Np; ++c) s += V[i * Np + c] * V[j * Np + c];
        VVt[i * Np + j] = s;
      }
    rc = invert(Np, VVt, o->M);
  }

  /* Face node lists. */
  o->Fmask = (int *)calloc((size_t)4 * Nfp, sizeof(int));
  for (int m = 0; m < Nfp; ++m) {
    o->Fmask[0 * Nfp + m] = m;                /* bottom: j = 0  */
    o->Fmask[1 * Nfp + m] = p + n1 * m;       /* right:  i = p  */
    o->Fmask[2 * Nfp + m] = m + n1 * p;       /* top:    j = p  */
    o->Fmask[3 * Nfp + m] = n1 * m;           /* left:   i = 0  */
  }

  /* E (Np x 4Nfp) and LIFT = M^{-1} E = (V V^T) E. */
  double *E = dalloc((size_t)Np * 4 * Nfp);
  for (int fc = 0; fc < 4; ++fc)
    for (int m = 0; m < Nfp; ++m)
      for (int mm = 0; mm < Nfp; ++mm)
        E[o->Fmask[fc * Nfp + m] * (4 * Nfp) + fc * Nfp + mm] = o->M1[m * n1 + mm];
  o->LIFT = dalloc((size_t)Np * 4 * Nfp);
  if (!rc) matmul(Np, Np, 4 * Nfp, VVt, E, o->LIFT);

  free(V); free(Vr); free(Vs); free(Vinv); free(VVt); free(E);
  return rc;
}

/* Uniform Cartesian mesh: element k = ex + nx*ey, affine map
 * x = x0 + hx (ex + (1+r)/2), y = y0 + hy (ey + (1+s)/2). */
static void build_mesh(oracle *o) {
  const oracle_problem *pb = &o->pb;
  int nx = pb->nx, ny = pb->ny;
  o->hx = pb->lx / nx;
  o->hy = pb->ly / ny;
  o->rx = 2.0 / o->hx;
  o->sy = 2.0 / o->hy;
  o->J = o->hx * o->hy / 4.0;
  o->sJ[0] = o->hx / 2.0; o->sJ[2] = o->hx / 2.0;
  o->sJ[1] = o->hy / 2.0; o->sJ[3] = o->hy / 2.0;
  for (int fc = 0; fc < 4; ++fc) o->Fscale[fc] = o->sJ[fc] / o->J;
  o->nxf[0] = 0.0;  o->nyf[0] = -1.0;
  o->nxf[1] = 1.0;  o->nyf[1] = 0.0;
  o->nxf[2] = 0.0;  o->nyf[2] = 1.0;
  o->nxf[3] = -1.0; o->nyf[3] = 0.0;
  o->nbr = (int *)calloc((size_t)o->K * 4, sizeof(int));
  for (int ey = 0; ey < ny; ++ey)
    for (int exx = 0; exx < nx; ++exx) {
      int k = exx + nx * ey;
      int *nb = &o->nbr[4 * k];
      if (ey > 0) nb[0] = k - nx;
      else nb[0] = (pb->bc[0] == ORACLE_BC_PERIODIC) ? k + nx * (ny - 1) : -1;
      if (exx < nx - 1) nb[1] = k + 1;
      else nb[1] = (pb->bc[1] == ORACLE_BC_PERIODIC) ? k - (nx - 1) : -1;
      if (ey < ny - 1) nb[2] = k + nx;
      else nb[2] = (pb->bc[2] == ORACLE_BC_PERIODIC) ? k - nx * (ny - 1) : -1;
      if (exx > 0) nb[3] = k - 1;
      else nb[3] = (pb->bc[3] == ORACLE_BC_PERIODIC) ? k + (nx - 1) : -1;
    }
}

oracle *oracle_create(const oracle_problem *pb) {
  if (!pb || pb->nx < 1 || pb->ny < 1 || pb->p < 1 || pb->p > 8 || pb->q < 1) return NULL;
  if (!pb->ex || !pb->ey || !pb->w) return NULL;
  if (!(pb->lx > 0.0) || !(pb->ly > 0.0) || !(pb->theta > 0.0) || !(pb->tau > 0.0)) return NULL;
  for (int s = 0; s < 4; ++s)
    if (pb->bc[s] != ORACLE_BC_PERIODIC && pb->bc[s] != ORACLE_BC_DIFFUSE_WALL) return NULL;
  if ((pb->bc[0] == ORACLE_BC_PERIODIC) != (pb->bc[2] == ORACLE_BC_PERIODIC)) return NULL;
  if ((pb->bc[1] == ORACLE_BC_PERIODIC) != (pb->bc[3] == ORACLE_BC_PERIODIC)) return NULL;

  oracle *o = (oracle *)calloc(1, sizeof(oracle));
  if (!o) return NULL;
  o->pb = *pb;
  o->p = pb->p;
  o->Q = pb->q;
  o->Nfp = pb->p + 1;
  o->Np = o->Nfp * o->Nfp;
  o->K = pb->nx * pb->ny;
  o->ex = dalloc(o->Q);
  o->ey = dalloc(o->Q);
  o->w = dalloc(o->Q);
  memcpy(o->ex, pb->ex, sizeof(double) * o->Q);
  memcpy(o->ey, pb->ey, sizeof(double) * o->Q);
  memcpy(o->w, pb->w, sizeof(double) * o->Q);
  o->pb.ex = o->ex;
  o->pb.ey = o->ey;
  o->pb.w = o->w;
  if (build_reference_element(o)) { oracle_destroy(o); return NULL; }
  build_mesh(o);
  size_t ndof = (size_t)o->Q * o->K * o->Np, nnode = (size_t)o->K * o->Np;
  o->f = dalloc(ndof);
  o->k1 = dalloc(ndof); o->k2 = dalloc(ndof); o->k3 = dalloc(ndof); o->k4 = dalloc(ndof);
  o->tmp = dalloc(ndof);
  o->rho = dalloc(nnode); o->ux = dalloc(nnode); o->uy = dalloc(nnode);
  o->rhow = dalloc((size_t)o->K * 4 * o->Nfp);
  if (!o->f || !o->k1 || !o->k2 || !o->k3 || !o->k4 || !o->tmp || !o->rho || !o->rhow) {
    oracle_destroy(o);
    return NULL;
  }
  for (size_t i = 0; i < ndof; ++i) o->f[i] = 0.0;
  return o;
}

int oracle_sizes(const oracle *o, int *K, int *Np, int *Nfp, int *Q) {
  if (!o) return -1;
  if (K) *K = o->K;
  if (Np) *Np = o->Np;
  if (Nfp) *Nfp = o->Nfp;
  if (Q) *Q = o->Q;
  return 0;
}

/* which: 0 Dr, 1 Ds, 2 M, 3 LIFT, 4 r (1-D GLL nodes), 5 M1, 6 Fscale[4],
 *        7 neighbour table [K][4] (as doubles). */
int oracle_operator(const oracle *o, int which, double *out) {
  if (!o || !out) return -1;
  int Np = o->Np, Nfp = o->Nfp, n1 = o->p + 1;
  switch (which) {
    case 0: memcpy(out, o->Dr, sizeof(double) * Np * Np); return 0;
    case 1: memcpy(out, o->Ds, sizeof(double) * Np * Np); return 0;
    case 2: memcpy(out, o->M, sizeof(double) * Np * Np); return 0;
    case 3: memcpy(out, o->LIFT, sizeof(double) * Np * 4 * Nfp); return 0;
    case 4: memcpy(out, o->r, sizeof(double) * n1); return 0;
    case 5: memcpy(out, o->M1, sizeof(double) * n1 * n1); return 0;
    case 6: memcpy(out, o->Fscale, sizeof(double) * 4); return 0;
    case 7:
      for (int i = 0; i < 4 * o->K; ++i) out[i] = (double)o->nbr[i];
      return 0;
    default: return -1;
  }
}

int oracle_node_coords(const oracle *o, double *x, double *y) {
  if (!o || !x || !y) return -1;
  int n1 = o->p + 1;
  for (int k = 0; k < o->K; ++k) {
    int exx = k % o->pb.nx, ey = k / o->pb.nx;
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n1; ++i) {
        int n = i + n1 * j;
        x[k * o->Np + n] = o->pb.x0 + o->hx * (exx + 0.5 * (1.0 + o->r[i]));
        y[k * o->Np + n] = o->pb.y0 + o->hy * (ey + 0.5 * (1.0 + o->r[j]));
      }
  }
  return 0;
}

/* Explicit time step: dt = CFL * (min(hx,hy)/2) * min GLL spacing /
 * max_q (|e_qx| + |e_qy|). */
int oracle_stable_dt(const oracle *o, double cfl, double *dt) {
  if (!o || !dt || !(cfl > 0.0)) return -1;
  double dr = 2.0;
  for (int i = 0; i < o->p; ++i) {
    double d = o->r[i + 1] - o->r[i];
    if (d < dr) dr = d;
  }
  double vmax = 0.0;
  for (int q = 0; q < o->Q; ++q) {
    double v = fabs(o->ex[q]) + fabs(o->ey[q]);
    if (v > vmax) vmax = v;
  }
  if (!(vmax > 0.0)) return -1;
  double h = o->hx < o->hy ? o->hx : o->hy;
  *dt = cfl * (0.5 * h) * dr / vmax;
  return 0;
}

int oracle_set_state(oracle *o, const double *f) {
  if (!o || !f) return -1;
  memcpy(o->f, f, sizeof(double) * (size_t)o->Q * o->K * o->Np);
  return 0;
}

int oracle_get_state(const oracle *o, double *f) {
  if (!o || !f) return -1;
  memcpy(f, o->f, sizeof(double) * (size_t)o->Q * o->K * o->Np);
  return 0;
}

/* Second-order Hermite equilibrium, eq. (5), with RT = theta:
 * f_q^eq = w_q rho [1 + e.u/theta + (e.u)^2/(2 theta^2) - |u|^2/(2 theta)]. */
static double feq(const oracle *o, int q, double rho, double ux, double uy) {
  double th = o->pb.theta;
  double eu = o->ex[q] * ux + o->ey[q] * uy;
  double usq = ux * ux + uy * uy;
  return o->w[q] * rho * (1.0 + eu / th + (eu * eu) / (2.0 * th * th) - usq / (2.0 * th));
}

int oracle_equilibrium(const oracle *o, double rho, double ux, double uy, double *out) {
  if (!o || !out) return -1;
  for (int q = 0; q < o->Q; ++q) out[q] = feq(o, q, rho, ux, uy);
  return 0;
}

int oracle_init_equilibrium(oracle *o, double rho0, double ux0, double uy0) {
  if (!o) return -1;
  for (int q = 0; q < o->Q; ++q) {
    double v = feq(o, q, rho0, ux0, uy0);
    for (int i = 0; i < o->K * o->Np; ++i) o->f[(size_t)q * o->K * o->Np + i] = v;
  }
  return 0;
}

/* Discrete moments (Sec. II.A): rho = sum_q f_q, rho u = sum_q e_q f_q. */
static void compute_moments(const oracle *o, const double *f, double *rho, double *ux,
                            double *uy) {
  int KN = o->K * o->Np;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < KN; ++i) {
    double r = 0.0, mx = 0.0, my = 0.0;
    for (int q = 0; q < o->Q; ++q) {
      double v = f[(size_t)q * KN + i];
      r += v;
      mx += o->ex[q] * v;
      my += o->ey[q] * v;
    }
    rho[i] = r;
    ux[i] = mx / r;
    uy[i] = my / r;
  }
}

/* Maxwell diffuse-scattering wall, eq. (8), at every wall face node:
 * rho_w = sum_{(e_j-u_b).n > 0} |(e_j-u_b).n| f_j
 *       / sum_{(e_k-u_b).n < 0} |(e_k-u_b).n| f_k^eq(1, u_b),
 * so that the exterior state of an incoming velocity is rho_w f_i^eq(1, u_b).
 * The density of the equilibria cancels in the ratio; n is the outward normal
 * of the fluid element (pointing into the wall); f_j is the interior trace. */
static void compute_wall_density(const oracle *o, const double *f, double *rhow) {
  int Nfp = o->Nfp, Np = o->Np, KN = o->K * o->Np;
  for (int k = 0; k < o->K; ++k)
    for (int fc = 0; fc < 4; ++fc) {
      if (o->nbr[4 * k + fc] >= 0) continue;
      double ubx = o->pb.wall_u[fc][0], uby = o->pb.wall_u[fc][1];
      double den = 0.0;
      for (int q = 0; q < o->Q; ++q) {
        double cn = (o->ex[q] - ubx) * o->nxf[fc] + (o->ey[q] - uby) * o->nyf[fc];
        if (cn < 0.0) den += fabs(cn) * feq(o, q, 1.0, ubx, uby);
      }
      for (int m = 0; m < Nfp; ++m) {
        int node = o->Fmask[fc * Nfp + m];
        double num = 0.0;
        for (int q = 0; q < o->Q; ++q) {
          double cn = (o->ex[q] - ubx) * o->nxf[fc] + (o->ey[q] - uby) * o->nyf[fc];
          if (cn > 0.0) num += fabs(cn) * f[(size_t)q * KN + k * Np + node];
        }
        rhow[(k * 4 + fc) * Nfp + m] = num / den;
      }
    }
}

int oracle_wall_density(oracle *o, const double *f, double *rho_w) {
  if (!o || !rho_w) return -1;
  compute_wall_density(o, f ? f : o->f, rho_w);
  return 0;
}

/* Right-hand side L(f) of the semi-discrete system, split into its parts.
 * For each element and velocity (eq. (6) discretised by eq. (10)):
 *   volume     V = -(e_x rx Dr + e_y sy Ds) f_q                (strong form)
 *   surface    S = LIFT g,  g = Fscale (e.n)(f^- - f^+) on faces where
 *              e.n < 0 (upwind numerical flux; zero on outflow faces),
 *              f^+ = neighbour trace, or rho_w f_q^eq(1,u_b) at a wall;
 *   collision  C = -(f_q - f_q^eq(rho, u)) / tau.
 * Any of vol/surf/coll may be NULL. */
static void rhs_parts(oracle *o, const double *f, double *vol, double *surf, double *coll,
                      double *total) {
  int K = o->K, Np = o->Np, Nfp = o->Nfp, Q = o->Q, KN = K * Np;
  compute_moments(o, f, o->rho, o->ux, o->uy);
  compute_wall_density(o, f, o->rhow);
  double inv_tau_is_zero = isinf(o->pb.tau) ? 1.0 : 0.0;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < K; ++k) {
    double V[81], S[81], C[81], g[36];
    for (int q = 0; q < Q; ++q) {
      const double *fq = &f[(size_t)q * KN + (size_t)k * Np];
      double ex = o->ex[q], ey = o->ey[q];
      for (int n = 0; n < Np; ++n) {
        double dr = 0.0, ds = 0.0;
        for (int m = 0; m < Np; ++m) {
          dr += o->Dr[n * Np + m] * fq[m];
          ds += o->Ds[n * Np + m] * fq[m];
        }
        V[n] = -(ex * o->rx * dr + ey * o->sy * ds);
      }
      for (int fc = 0; fc < 4; ++fc) {
        double en = ex * o->nxf[fc] + ey * o->nyf[fc];
        int nb = o->nbr[4 * k + fc];
        for (int m = 0; m < Nfp; ++m) {
          double gv = 0.0;
          if (en < 0.0) {
            double fm = fq[o->Fmask[fc * Nfp + m]];
            double fp;
            if (nb >= 0) {
              int opp = (fc + 2) % 4;
              fp = f[(size_t)q * KN + (size_t)nb * Np + o->Fmask[opp * Nfp + m]];
            } else {
              fp = o->rhow[(k * 4 + fc) * Nfp + m] *
                   feq(o, q, 1.0, o->pb.wall_u[fc][0], o->pb.wall_u[fc][1]);
            }
            gv = o->Fscale[fc] * en * (fm - fp);
          }
          g[fc * Nfp + m] = gv;
        }
      }
      for (int n = 0; n < Np; ++n) {
        double s = 0.0;
        for (int j = 0; j < 4 * Nfp; ++j) s += o->LIFT[n * 4 * Nfp + j] * g[j];
        S[n] = s;
      }
      for (int n = 0; n < Np; ++n) {
        int i = k * Np + n;
        if (inv_tau_is_zero != 0.0) {
          C[n] = 0.0;
        } else {
          double fe = feq(o, q, o->rho[i], o->ux[i], o->uy[i]);
          C[n] = -(fq[n] - fe) / o->pb.tau;
        }
      }
      for (int n = 0; n < Np; ++n) {
        size_t idx = (size_t)q * KN + (size_t)k * Np + n;
        if (vol) vol[idx] = V[n];
        if (surf) surf[idx] = S[n];
        if (coll) coll[idx] = C[n];
        if (total) total[idx] = V[n] + S[n] + C[n];
      }
    }
  }
}

int oracle_rhs(oracle *o, const double *f, double *k) {
  if (!o || !k) return -1;
  rhs_parts(o, f ? f : o->f, NULL, NULL, NULL, k);
  return 0;
}

int oracle_rhs_parts(oracle *o, const double *f, double *vol, double *surf, double *coll) {
  if (!o) return -1;
  rhs_parts(o, f ? f : o->f, vol, surf, coll, NULL);
  return 0;
}

/* Classical four-stage RK4:
 *   k1 = L(f), k2 = L(f + dt/2 k1), k3 = L(f + dt/2 k2), k4 = L(f + dt k3),
 *   f <- f + dt/6 (k1 + 2 k2 + 2 k3 + k4). */
int oracle_rk4(oracle *o, long nsteps, double dt) {
  if (!o || nsteps < 0) return -1;
  size_t N = (size_t)o->Q * o->K * o->Np;
  for (long s = 0; s < nsteps; ++s) {
    rhs_parts(o, o->f, NULL, NULL, NULL, o->k1);
    for (size_t i = 0; i < N; ++i) o->tmp[i] = o->f[i] + 0.5 * dt * o->k1[i];
    rhs_parts(o, o->tmp, NULL, NULL, NULL, o->k2);
    for (size_t i = 0; i < N; ++i) o->tmp[i] = o->f[i] + 0.5 * dt * o->k2[i];
    rhs_parts(o, o->tmp, NULL, NULL, NULL, o->k3);
    for (size_t i = 0; i < N; ++i) o->tmp[i] = o->f[i] + dt * o->k3[i];
    rhs_parts(o, o->tmp, NULL, NULL, NULL, o->k4);
    for (size_t i = 0; i < N; ++i)
      o->f[i] = o->f[i] + dt / 6.0 * (o->k1[i] + 2.0 * o->k2[i] + 2.0 * o->k3[i] + o->k4[i]);
  }
  return 0;
}

int oracle_moments(const oracle *o, double *rho, double *ux, double *uy) {
  if (!o || !rho || !ux || !uy) return -1;
  compute_moments(o, o->f, rho, ux, uy);
  return 0;
}

/* Steady-state residual: the largest rate of change of the conserved moments,
 * R = max over nodes of max(|sum_q L_q|, |sum_q e_qx L_q|, |sum_q e_qy L_q|)
 * scaled by L_ref / (rho_ref U_ref), with rho_ref = 1, L_ref = min(lx, ly) and
 * U_ref the largest wall speed (1 if every wall is at rest).  Returns -4 (and
 * NaN) if the state or its RHS is not finite. */
int oracle_residual(oracle *o, double *r) {
  if (!o || !r) return -1;
  rhs_parts(o, o->f, NULL, NULL, NULL, o->k1);
  int KN = o->K * o->Np;
  double rmax = 0.0;
  int bad = 0;
  for (int i = 0; i < KN; ++i) {
    double a = 0.0, bx = 0.0, by = 0.0;
    for (int q = 0; q < o->Q; ++q) {
      double v = o->k1[(size_t)q * KN + i];
      a += v;
      bx += o->ex[q] * v;
      by += o->ey[q] * v;
    }
    if (!isfinite(a) || !isfinite(bx) || !isfinite(by)) bad = 1;
    double m = fabs(a);
    if (fabs(bx) > m) m = fabs(bx);
    if (fabs(by) > m) m = fabs(by);
    if (m > rmax) rmax = m;
  }
  double uref = 0.0;
  for (int s = 0; s < 4; ++s) {
    if (o->pb.bc[s] != ORACLE_BC_DIFFUSE_WALL) continue;
    double sp = sqrt(o->pb.wall_u[s][0] * o->pb.wall_u[s][0] +
                     o->pb.wall_u[s][1] * o->pb.wall_u[s][1]);
    if (sp > uref) uref = sp;
  }
  if (!(uref > 0.0)) uref = 1.0;
  double lref = o->pb.lx < o->pb.ly ? o->pb.lx : o->pb.ly;
  if (bad) { *r = NAN; return -4; }
  *r = rmax * lref / uref;
  return 0;
}

/* Total mass: sum over elements of J 1^T M rho. */
double oracle_total_mass(const oracle *o) {
  if (!o) return NAN;
  int Np = o->Np, KN = o->K * Np;
  double *rho = dalloc(KN), *ux = dalloc(KN), *uy = dalloc(KN);
  compute_moments(o, o->f, rho, ux, uy);
  double total = 0.0;
  for (int k = 0; k < o->K; ++k) {
    double s = 0.0;
    for (int n = 0; n < Np; ++n)
      for (int m = 0; m < Np; ++m) s += o->M[n * Np + m] * rho[k * Np + m];
    total += o->J * s;
  }
  free(rho); free(ux); free(uy);
  return total;
}

/* Couette closed form for D2Q16, eq. (11), with two corrections to the printed
 * form: the missing "+" between the cosh and sinh terms of Z16 is restored, and
 * the coordinate is measured from the channel centre, s = y - y_bottom - L/2,
 * so that the plates sit at s = -L/2 and s = +L/2.  kn is the Knudsen number
 * of eq. (7) (tau = kn L / sqrt(3)):
 *   u_x = U + dU [ sinh(s/(kn L)) / Z16 + s / (L Theta16) ],
 *   Theta16 = 1 + 2 kn (2 cosh(1/2kn) + mu sinh(1/2kn)) / (mu cosh(1/2kn) + 2 sqrt3 sinh(1/2kn)),
 *   Z16 = mu/(4 kn) [ (4 kn + mu) cosh(1/2kn) + 2 (mu kn + sqrt3) sinh(1/2kn) ],
 *   mu = sqrt(3 - sqrt6) + sqrt(3 + sqrt6),  dU = U_top - U_bot, U = (U_top + U_bot)/2.
 * Here y is measured from the bottom plate. */
double oracle_couette_ux(double y, double L, double kn, double u_top, double u_bot) {
  double mu = sqrt(3.0 - sqrt(6.0)) + sqrt(3.0 + sqrt(6.0));
  double a = 1.0 / (2.0 * kn);
  double ch = cosh(a), sh = sinh(a);
  double theta16 = 1.0 + 2.0 * kn * (2.0 * ch + mu * sh) / (mu * ch + 2.0 * sqrt(3.0) * sh);
  double z16 = mu / (4.0 * kn) * ((4.0 * kn + mu) * ch + 2.0 * (mu * kn + sqrt(3.0)) * sh);
  double dU = u_top - u_bot, U = 0.5 * (u_top + u_bot);
  double s = y - 0.5 * L;
  return U + dU * (sinh(s / (kn * L)) / z16 + s / (L * theta16));
}

/* L2 error of u_x against the Couette closed form (Sec. III.A):
 * E = sqrt( sum_k int_{D^k} (u_x^e - u_x^k)^2 dx ), with u_x^k the degree-p
 * interpolant of the nodal u_x, integrated by a (p+3)^2-point Gauss rule. */
double oracle_l2_error_couette(const oracle *o, double kn, double u_top, double u_bot) {
  if (!o) return NAN;
  int n1 = o->p + 1, Np = o->Np, ng = o->p + 3, KN = o->K * Np;
  double xg[64], wg[64];
  oracle_gauss_legendre(ng, xg, wg);
  double *rho = dalloc(KN), *ux = dalloc(KN), *uy = dalloc(KN);
  compute_moments(o, o->f, rho, ux, uy);
  /* Lagrange basis on the GLL nodes evaluated at the Gauss points. */
  double ell[64 * 9];
  for (int g = 0; g < ng; ++g)
    for (int i = 0; i < n1; ++i) {
      double v = 1.0;
      for (int m = 0; m < n1; ++m)
        if (m != i) v *= (xg[g] - o->r[m]) / (o->r[i] - o->r[m]);
      ell[g * n1 + i] = v;
    }
  double err2 = 0.0;
  for (int k = 0; k < o->K; ++k) {
    int ey = k / o->pb.nx;
    for (int gj = 0; gj < ng; ++gj)
      for (int gi = 0; gi < ng; ++gi) {
        double uh = 0.0;
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i)
            uh += ux[k * Np + i + n1 * j] * ell[gi * n1 + i] * ell[gj * n1 + j];
        double y = o->hy * (ey + 0.5 * (1.0 + xg[gj]));
        double ue = oracle_couette_ux(y, o->pb.ly, kn, u_top, u_bot);
        err2 += wg[gi] * wg[gj] * o->J * (ue - uh) * (ue - uh);
      }
  }
  free(rho); free(ux); free(uy);
  return sqrt(err2);
}
