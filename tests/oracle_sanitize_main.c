/*
 * Driver for the sanitizer build of the FP64 oracle (test infrastructure):
 * exercises every entry point of oracle/lbm_oracle.h on small grids -- a
 * droplet with bubbles on a wetting wall under gravity and the Boussinesq
 * force with unequal phase properties, grids as narrow as 3x3, fields,
 * diagnostics, populations, checkpoint round trip and parameter validation
 * -- so that AddressSanitizer and UndefinedBehaviorSanitizer see every pass
 * of the step.  Exit status 0 when every call behaves as documented.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_oracle.h"

static oracle_params base_params(int nx, int ny) {
  oracle_params p;
  memset(&p, 0, sizeof(p));
  p.nx = nx;
  p.ny = ny;
  p.W = 4.0; p.M = 0.1; p.sigma = 0.005;
  p.rho_l = 1.0; p.rho_g = 1e-3; p.rho_s = 0.9;
  p.mu_l = 0.1; p.mu_g = 1e-3; p.mu_s = 0.1;
  p.cp_l = 1.0; p.cp_g = 0.9; p.cp_s = 0.5; p.cp_ref = 1.0;
  p.k_l = 0.1; p.k_g = 0.05; p.k_s = 0.38;
  p.latent = 10.0; p.T_melt = 1.0; p.T_bottom = 0.0;
  p.theta_bottom_deg = 70.0; p.theta_top_deg = 110.0;
  p.gx = 1e-6; p.gy = -2e-6;
  p.bq_beta = 0.05; p.bq_rho0 = 1.0; p.bq_Tref = 1.0;
  p.st_solid_mask = 1;
  return p;
}

static int run_case(int nx, int ny, int steps) {
  const size_t N = (size_t)nx * ny;
  double* phi0 = malloc(N * sizeof(double));
  double* T0 = malloc(N * sizeof(double));
  const double xc = 0.5 * nx, R = fmin(nx, ny) * 0.4;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const double r = hypot(x - xc, y + 0.5);
      const double rb = hypot(x - xc, y - 0.4 * R);  /* one bubble inside */
      double ph = 0.5 + 0.5 * tanh(2.0 * (R - r) / 4.0);
      ph *= 0.5 + 0.5 * tanh(2.0 * (rb - 0.25 * R) / 4.0);
      phi0[(size_t)y * nx + x] = ph;
      T0[(size_t)y * nx + x] = 1.0 + 1e-3 * sin(0.7 * x + 1.3 * y);
    }
  oracle_params p = base_params(nx, ny);
  oracle_ctx* c = NULL;
  int bad = 0;
  if (oracle_init(&p, phi0, T0, &c) != ORACLE_OK) return 1;
  if (oracle_step(c, steps) != ORACLE_OK) bad = 1;
  double* out[10];
  for (int j = 0; j < 10; ++j) out[j] = malloc(N * sizeof(double));
  if (oracle_fields(c, 0x3ffu, out) != ORACLE_OK) bad = 1;
  for (size_t k = 0; k < N; ++k)
    if (!isfinite(out[0][k]) || !isfinite(out[1][k])) bad = 1;
  oracle_diag_t d;
  if (oracle_diag(c, &d) != ORACLE_OK || d.step != steps) bad = 1;
  double* pops = malloc(9 * N * sizeof(double));
  for (int lat = 0; lat < 3; ++lat)
    if (oracle_pops(c, lat, pops) != ORACLE_OK) bad = 1;
  if (oracle_pops(c, 3, pops) == ORACLE_OK) bad = 1;
  const size_t nb = oracle_state_bytes(c);
  void* blob = malloc(nb);
  if (oracle_save(c, blob, nb) != ORACLE_OK) bad = 1;
  if (oracle_step(c, 2) != ORACLE_OK) bad = 1;
  if (oracle_load(c, blob, nb) != ORACLE_OK || oracle_step_count(c) != steps) bad = 1;
  if (oracle_save(c, blob, nb - 1) == ORACLE_OK) bad = 1;  /* too small */
  oracle_destroy(c);
  free(blob);
  free(pops);
  for (int j = 0; j < 10; ++j) free(out[j]);
  free(phi0);
  free(T0);
  return bad;
}

int main(void) {
  int bad = 0;
  oracle_set_threads(2);
  bad |= run_case(3, 3, 7);
  bad |= run_case(17, 9, 40);
  bad |= run_case(40, 24, 60);
  /* validation refuses bad parameters without touching memory */
  oracle_params p = base_params(2, 8);
  if (oracle_validate(&p) == ORACLE_OK) bad = 1;
  p = base_params(8, 8);
  p.M = 0.0;
  if (oracle_validate(&p) == ORACLE_OK) bad = 1;
  p = base_params(8, 8);
  p.theta_bottom_deg = 180.0;
  if (oracle_validate(&p) == ORACLE_OK) bad = 1;
  /* per-node blocks */
  double o9[9], f9[9] = {0};
  oracle_geq(0.7, 1e-3, -2e-3, o9);
  oracle_gsrc(0.7, 1e-5, 2e-5, 0.1, -0.1, 1e-4, o9);
  oracle_feq(1e-3, 1.0, 1e-3, 0.0, o9);
  oracle_fforce(1e-4, 1e-5, 0.0, 0.0, 0.0, 1e-3, 0.0, 1e-5, 0.0, o9);
  oracle_heq(11.0, 1.0, 1.0, 1.0, 0.0, 0.0, o9);
  double pr, fl, T;
  oracle_pressure(f9, 0.0, 0.0, 0.8, 1.0, 0.0, 0.0, &pr);
  oracle_enthalpy(5.0, 1.0, 1.0, 10.0, &fl, &T);
  double ext[5 * 4], gx[3 * 4], gy[3 * 4], lap[3 * 4], r0[4] = {1, 0.5, 0, 0.5}, r1[4] = {1, 1, 0, 0}, gh[4];
  for (int i = 0; i < 20; ++i) ext[i] = 0.1 * i;
  oracle_stencil(4, 3, ext, gx, gy, lap);
  oracle_wetting_ghost(4, 60.0, r0, r1, gh);
  printf(bad ? "sanitizer driver: FAILED\n" : "sanitizer driver: ok\n");
  return bad;
}
