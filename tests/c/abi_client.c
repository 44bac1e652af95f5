/*
 * A plain C99 client of the DG-BGK library, built by the tests against
 * include/dgbgk.h and libdgbgk.so: a lid-driven cavity on [0,1]^2 (6 x 5
 * quadrilaterals, p = 2, Newton-Cotes 8 x 8 velocities on [-4, 4], Kn = 1,
 * lid speed 0.1 on the top side; Sec. III.B).
 *
 *   abi_client cpu   host-only calls, and the error codes of device calls
 *                    on a machine without a GPU
 *   abi_client gpu   50 RK4 steps from rest; prints the residual and the
 *                    largest |u_x|
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dgbgk.h"

#define M1D 8
#define NQ (M1D * M1D)

static int check(int rc, int want, const char *what, const dgbgk_solver *s) {
  if (rc == want) return 0;
  fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, rc, want, s ? dgbgk_last_error(s) : "");
  return 1;
}

int main(int argc, char **argv) {
  const int gpu = argc > 1 && strcmp(argv[1], "gpu") == 0;
  double ex[NQ], ey[NQ], w[NQ], theta, tau, dt;
  dgbgk_problem pb;
  dgbgk_solver *s = NULL;
  size_t bytes = 0;
  int64_t K = 0;
  int32_t Np = 0, Nfp = 0, Q = 0;
  int side, bad = 0;

  if (check(dgbgk_velset_nc(M1D, 4.0, ex, ey, w, &theta), DGBGK_OK, "velset_nc", NULL)) return 1;
  if (check(dgbgk_tau_from_kn(1.0, 1.0, 1, &tau), DGBGK_OK, "tau_from_kn", NULL)) return 1;
  memset(&pb, 0, sizeof pb);
  pb.nx = 6;
  pb.ny = 5;
  pb.lx = 1.0;
  pb.ly = 1.0;
  pb.p = 2;
  pb.q = NQ;
  pb.ex = ex;
  pb.ey = ey;
  pb.w = w;
  pb.theta = theta;
  pb.tau = tau;
  for (side = 0; side < 4; ++side) pb.bc[side] = DGBGK_BC_DIFFUSE_WALL;
  pb.wall_u[2][0] = 0.1;

  if (check(dgbgk_required_bytes(&pb, DGBGK_FP64, &bytes), DGBGK_OK, "required_bytes", NULL)) return 1;
  if (check(dgbgk_create(&pb, DGBGK_FP64, NULL, &s), DGBGK_OK, "create", NULL)) return 1;
  bad |= check(dgbgk_sizes(s, &K, &Np, &Nfp, &Q), DGBGK_OK, "sizes", s);
  bad |= check(dgbgk_stable_dt(s, 0.2, &dt), DGBGK_OK, "stable_dt", s);
  bad |= check(dgbgk_step(NULL, 1, dt), DGBGK_EINVAL, "step(NULL)", NULL);
  bad |= check(dgbgk_stable_dt(s, -1.0, &dt), DGBGK_EINVAL, "stable_dt(-1)", s);
  bad |= check(dgbgk_stable_dt(s, 0.2, &dt), DGBGK_OK, "stable_dt", s);
  if (bad) return 1;
  printf("K %lld Np %d Nfp %d Q %d bytes %zu dt %.17g\n", (long long)K, Np, Nfp, Q, bytes, dt);

  if (!gpu) {
    bad |= check(dgbgk_init_equilibrium(s, 1.0, 0.0, 0.0), DGBGK_EDEVICE, "init_equilibrium", s);
    bad |= dgbgk_last_error(s)[0] == '\0';
    bad |= check(dgbgk_step(s, 1, dt), DGBGK_ESTATE, "step before a state", s);
  } else {
    const size_t n = (size_t)K * Np;
    double *rho = malloc(n * sizeof *rho), *ux = malloc(n * sizeof *ux), *uy = malloc(n * sizeof *uy);
    double r = 0.0, umax = 0.0;
    size_t i;
    if (!rho || !ux || !uy) return 1;
    bad |= check(dgbgk_init_equilibrium(s, 1.0, 0.0, 0.0), DGBGK_OK, "init_equilibrium", s);
    bad |= check(dgbgk_step(s, 50, dt), DGBGK_OK, "step", s);
    bad |= check(dgbgk_residual(s, &r), DGBGK_OK, "residual", s);
    bad |= check(dgbgk_moments(s, rho, ux, uy), DGBGK_OK, "moments", s);
    for (i = 0; i < n; ++i) umax = fabs(ux[i]) > umax ? fabs(ux[i]) : umax;
    printf("residual %.17g\numax %.17g\n", r, umax);
    free(rho);
    free(ux);
    free(uy);
  }
  dgbgk_destroy(s);
  if (!bad) printf("ok\n");
  return bad;
}
