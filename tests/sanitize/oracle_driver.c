/* Drives every entry point of the FP64 oracle on small random inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure: any out-of-bounds access, leak or undefined operation
 * aborts with a non-zero exit status).  Inputs come from a fixed-seed
 * linear congruential generator. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_oracle.h"

static unsigned long long rng_state = 12345u;
static double uniform(void) {
  rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(int nx, int ny, int nz, int n_spheres, int collision, int wall) {
  const int64_t ncell = (int64_t)nx * ny * nz;
  double* sp = malloc(sizeof(double) * 4 * (n_spheres > 0 ? n_spheres : 1));
  int emin = nx < ny ? (nx < nz ? nx : nz) : (ny < nz ? ny : nz);
  for (int s = 0; s < n_spheres; ++s) {
    sp[4 * s + 0] = uniform() * nx;
    sp[4 * s + 1] = uniform() * ny;
    sp[4 * s + 2] = uniform() * nz;
    sp[4 * s + 3] = 0.2 + uniform() * (0.45 * emin);
  }
  uint8_t* mask = malloc((size_t)ncell);
  double* Q = malloc(sizeof(double) * 19 * ncell);
  double* g = malloc(sizeof(double) * 19 * ncell);
  double* work = malloc(sizeof(double) * 19 * ncell);
  double* drho = malloc(sizeof(double) * ncell);
  double* u = malloc(sizeof(double) * 3 * ncell);
  int64_t n_solid = orc_voxelise(nx, ny, nz, sp, n_spheres, mask);
  if (n_solid == ncell) mask[0] = 0; /* keep one fluid cell */
  orc_wall_q(nx, ny, nz, mask, sp, n_spheres, Q);
  orc_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.tau = 0.55 + uniform();
  p.magic = 3.0 / 16.0;
  p.drho = 1e-4;
  p.collision = collision;
  p.wall = wall;
  for (int64_t c = 0; c < ncell; ++c) {
    drho[c] = 1e-4 * (uniform() - 0.5);
    for (int a = 0; a < 3; ++a) u[a * ncell + c] = 1e-3 * (uniform() - 0.5);
  }
  orc_init(&p, mask, drho, u, g);
  orc_run(&p, mask, Q, g, work, 3);
  orc_macroscopic(&p, mask, g, drho, u);
  double U[3], F[3];
  orc_mean_velocity(&p, mask, g, U);
  orc_drag(&p, mask, Q, g, F);
  double K = orc_permeability(&p, U[0]);
  int64_t done = 0;
  double res = 0.0;
  int32_t st = orc_run_to_residual(&p, mask, Q, g, work, 1e-30, 6, 2, &done, &res);
  int ok = isfinite(U[0]) && isfinite(F[0]) && isfinite(K) && done == 6 && st == 1;
  free(sp);
  free(mask);
  free(Q);
  free(g);
  free(work);
  free(drho);
  free(u);
  return ok;
}

int main(void) {
  int32_t e[57], opp[19];
  double w[19], M[361], Minv[361], n2[19], s[19], geq[19], gc[19];
  orc_lattice(e, w, opp);
  orc_mrt_matrix(M, Minv, n2);
  orc_mrt_rates(0.8, s);
  double uu[3] = {1e-3, -2e-3, 5e-4};
  orc_equilibrium(1e-3, uu, geq);
  memcpy(gc, geq, sizeof gc);
  orc_collide_mrt_rates(s, gc);
  const int shapes[][4] = {{1, 1, 1, 0}, {5, 1, 1, 0}, {1, 6, 3, 0}, {7, 5, 4, 2},
                           {6, 8, 5, 3}, {9, 4, 7, 4}, {8, 8, 8, 1}};
  int failures = 0, cases = 0;
  for (unsigned i = 0; i < sizeof shapes / sizeof shapes[0]; ++i)
    for (int coll = 0; coll < 3; ++coll)
      for (int wall = 0; wall < 6; ++wall) { /* tau < 2 here, so IEBB is defined */
        failures += !run_case(shapes[i][0], shapes[i][1], shapes[i][2], shapes[i][3], coll, wall);
        ++cases;
      }
  printf("oracle sanitizer driver: %d cases, %d failures\n", cases, failures);
  return failures ? 1 : 0;
}
