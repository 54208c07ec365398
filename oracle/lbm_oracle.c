/*
 * FP64 CPU oracle for one time step of the three coupled D2Q9 lattices of
 * Huang, Wang, Chai & Shi, "Phase-field based lattice Boltzmann method for
 * containerless freezing" (arXiv:2403.16122).
 *
 * TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
 * baseline load this library; nothing on the product path may.  It shares
 * no code with the GPU library.
 *
 * The step is written as full-field passes in the order the method needs
 * them (macroscopic quantities at time t, then the isotropic stencils of
 * Sec. 3.4 at time t, then forces, then the three BGK collisions).  Every
 * pass cites the equation it follows.  Equation numbers count the paper's
 * numbered displays in order: Eq. (1) property mixing, (2)-(3) Allen-Cahn,
 * (7)-(9) enthalpy, (10)-(13) Navier-Stokes and surface tension, (19) mass
 * source, (20) fluid-solid force, (21)-(26) phase-field LBE, (27)-(29)
 * enthalpy LBE, (30)-(36) flow LBE, (37) time derivative, (38a,b) stencils,
 * (39)-(41) wetting boundary.  Where the paper is silent or garbled the
 * reading taken is named inline; the full list lives with the design notes.
 *
 * Every term is pinned by a CPU test against a closed form; the c_s^2 grad S
 * term of F~ (Eq. (33)) by the exact one-step response of the pressure of
 * Eq. (36) to a prescribed lagged S under uniform flow.
 *
 * Plain loops; OpenMP splits rows of each pass (results do not depend on the
 * thread count: no reduction runs in parallel).
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 lattice, Sec. 3.1 (Eq. (22)-(23)): rest, 4 axis, 4 diagonal. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0;

struct oracle_ctx {
  oracle_params P;
  int nx, ny;
  size_t N;
  int64_t step;
  /* persistent state: post-collision populations and lagged fields */
  double *g, *f, *h;                 /* [9][N] */
  double *phiu_x, *phiu_y;           /* (phi u)^{n-1}, Eq. (37) */
  double *fsH_prev;                  /* f_s^H at the previous step */
  double *p_prev, *S_prev;           /* p^{n-1}, S^{n-1} */
  /* per-step work arrays */
  double *gs, *fs, *hs;              /* streamed populations [9][N] */
  double *G0, *phi, *phic, *rho, *mu, *cp, *kk, *H, *T, *fl, *fsH, *fsol, *mdot;
  double *phi_ext, *rho_ext, *p_ext, *S_ext;   /* (ny+2) x nx with ghost rows */
  double *gphx, *gphy, *lphi, *grx, *gry, *lrho, *gpx, *gpy, *lp, *gSx, *gSy, *lS;
  double *ux, *uy, *p, *S, *lamnx, *lamny;
  double *Fi;                        /* flow forcing term [9][N] */
};

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* Eq. (1): zeta = f_s zeta_s + (1-f_s) phi zeta_l + (1-f_s)(1-phi) zeta_g,
 * with phi clamped to [0,1] (reading: mixing uses the clamped order parameter). */
static double mix(double fsol, double phic, double zs, double zl, double zg) {
  return fsol * zs + (1.0 - fsol) * phic * zl + (1.0 - fsol) * (1.0 - phic) * zg;
}

/* ------------------------------------------------------------------ */
/* Per-node building blocks                                            */
/* ------------------------------------------------------------------ */

/* Eq. (24): g_i^eq = w_i phi (1 + c_i.u / cs^2). */
void oracle_geq(double phi, double ux, double uy, double* out) {
  for (int i = 0; i < 9; ++i) {
    double cu = CX[i] * ux + CY[i] * uy;
    out[i] = WT[i] * phi * (1.0 + cu / CS2);
  }
}

/* Eq. (25): G_i = w_i c_i.[d_t(phi u) + cs^2 lambda n]/cs^2 + w_i phi div(u),
 * with div(u) = mdot (Eq. (19)).  lnx, lny hold lambda*n. */
void oracle_gsrc(double phi, double dphiux, double dphiuy, double lnx, double lny, double mdot,
                 double* out) {
  for (int i = 0; i < 9; ++i) {
    double a = CX[i] * (dphiux + CS2 * lnx) + CY[i] * (dphiuy + CS2 * lny);
    out[i] = WT[i] * a / CS2 + WT[i] * phi * mdot;
  }
}

/* Eq. (31)-(32): f_i^eq = p/cs^2 (w_i - delta_i0) + rho s_i(u),
 * s_i(u) = w_i [c.u/cs^2 + (c.u)^2/(2 cs^4) - u.u/(2 cs^2)]. */
void oracle_feq(double p, double rho, double ux, double uy, double* out) {
  double usq = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    double cu = CX[i] * ux + CY[i] * uy;
    double s = WT[i] * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - usq / (2.0 * CS2));
    double d = (i == 0) ? 1.0 : 0.0;
    out[i] = p / CS2 * (WT[i] - d) + rho * s;
  }
}

/* Eq. (33): F_i = w_i [ S + c_i.(F + rho f)/cs^2
 *                       + (u Ft + Ft u):(c_i c_i - cs^2 I)/(2 cs^4) ],
 * reading the printed "(u Ft + u Ft)" as the symmetric product u Ft + Ft u. */
void oracle_fforce(double S, double Fx, double Fy, double rfx, double rfy, double ux, double uy,
                   double Ftx, double Fty, double* out) {
  for (int i = 0; i < 9; ++i) {
    double cx = CX[i], cy = CY[i];
    /* (u Ft + Ft u):(c c - cs^2 I) written out component by component */
    double Axx = 2.0 * ux * Ftx, Ayy = 2.0 * uy * Fty, Axy = ux * Fty + Ftx * uy;
    double contr = Axx * (cx * cx - CS2) + Ayy * (cy * cy - CS2) + 2.0 * Axy * cx * cy;
    out[i] = WT[i] * (S + (cx * (Fx + rfx) + cy * (Fy + rfy)) / CS2 + contr / (2.0 * CS2 * CS2));
  }
}

/* Eq. (28): total-enthalpy equilibrium (rest population carries H - cp_ref T). */
void oracle_heq(double H, double T, double cp, double cp_ref, double ux, double uy, double* out) {
  double usq = ux * ux + uy * uy;
  out[0] = H - cp_ref * T + WT[0] * cp * T * (cp_ref / cp - usq / (2.0 * CS2));
  for (int i = 1; i < 9; ++i) {
    double cu = CX[i] * ux + CY[i] * uy;
    /* (e e - cs^2 I):uu = (e.u)^2 - cs^2 u.u */
    double q = (cu * cu - CS2 * usq) / (2.0 * CS2 * CS2);
    out[i] = WT[i] * cp * T * (cp_ref / cp + cu / CS2 + q);
  }
}

/* Eq. (36): p = cs^2/(1-w_0) [ sum_{i!=0} f_i + dt/2 S + tau dt F_0 + rho s_0(u) ],
 * tau read as the local flow relaxation time. */
void oracle_pressure(const double* f9, double S, double F0, double tau_f, double rho, double ux,
                     double uy, double* p_out) {
  double sum = 0.0;
  for (int i = 1; i < 9; ++i) sum += f9[i];
  double usq = ux * ux + uy * uy;
  double s0 = WT[0] * (-usq / (2.0 * CS2));
  *p_out = CS2 / (1.0 - WT[0]) * (sum + 0.5 * S + tau_f * F0 + rho * s0);
}

/* Eq. (9a,b) for a pure substance (T_s = T_l = T_m), with H_s = cp T_m and
 * H_l = cp T_m + L (the second printed "H_s" read as H_l). */
void oracle_enthalpy(double H, double cp, double T_melt, double latent, double* fl, double* T) {
  double Hs = cp * T_melt;
  double Hl = cp * T_melt + latent;
  if (H <= Hs)
    *fl = 0.0;
  else if (H >= Hl)
    *fl = 1.0;
  else
    *fl = (H - Hs) / (Hl - Hs);
  if (H < Hs)
    *T = H / cp;
  else if (H > Hl)
    *T = T_melt + (H - Hl) / cp;
  else
    *T = T_melt;
}

/* Eq. (38a,b): grad z = sum_{i!=0} w_i c_i z(x+c_i)/cs^2,
 *              lap z  = sum_{i!=0} 2 w_i [z(x+c_i) - z(x)]/cs^2. */
void oracle_stencil(int32_t nx, int32_t ny, const double* ext, double* gx, double* gy,
                    double* lap) {
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      double zc = ext[(size_t)(y + 1) * nx + x];
      double sx = 0.0, sy = 0.0, sl = 0.0;
      for (int i = 1; i < 9; ++i) {
        int xn = ((x + CX[i]) % nx + nx) % nx;
        int yn = y + CY[i];
        double z = ext[(size_t)(yn + 1) * nx + xn];
        sx += WT[i] * CX[i] * z;
        sy += WT[i] * CY[i] * z;
        sl += 2.0 * WT[i] * (z - zc);
      }
      size_t k = (size_t)y * nx + x;
      if (gx) gx[k] = sx / CS2;
      if (gy) gy[k] = sy / CS2;
      if (lap) lap[k] = sl / CS2;
    }
  }
}

/* Eq. (39)-(41): n_w.grad(phi) = -tan(pi/2 - theta) |n_t.grad(phi)|, with the
 * normal derivative (phi_fluid - phi_ghost)/dx and the tangential derivative
 * extrapolated to the wall, 1.5 d_x phi(row0) - 0.5 d_x phi(row1), each by
 * central differences.  Solved for the ghost value. */
void oracle_wetting_ghost(int32_t nx, double theta_deg, const double* r0, const double* r1,
                          double* ghost) {
  double t = tan((90.0 - theta_deg) * M_PI / 180.0);
  for (int x = 0; x < nx; ++x) {
    int xp = (x + 1) % nx, xm = (x - 1 + nx) % nx;
    double d0 = 0.5 * (r0[xp] - r0[xm]);
    double d1 = 0.5 * (r1[xp] - r1[xm]);
    double tang = 1.5 * d0 - 0.5 * d1;
    ghost[x] = r0[x] + t * fabs(tang);
  }
}

/* ------------------------------------------------------------------ */
/* Validation and set-up                                               */
/* ------------------------------------------------------------------ */

static int finite_all(const oracle_params* p) {
  const double v[] = {p->W,     p->M,      p->sigma,  p->rho_l,  p->rho_g,  p->rho_s,
                      p->mu_l,  p->mu_g,   p->mu_s,   p->cp_l,   p->cp_g,   p->cp_s,
                      p->cp_ref, p->k_l,   p->k_g,    p->k_s,    p->latent, p->T_melt,
                      p->T_bottom, p->theta_bottom_deg, p->theta_top_deg, p->gx, p->gy,
                      p->bq_beta, p->bq_rho0, p->bq_Tref};
  for (size_t i = 0; i < sizeof(v) / sizeof(v[0]); ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

int oracle_validate(const oracle_params* p) {
  if (!p) return ORACLE_EINVAL;
  if (p->nx < 3 || p->ny < 3) return ORACLE_EINVAL;
  if (!finite_all(p)) return ORACLE_EINVAL;
  if (!(p->W > 0.0) || !(p->M > 0.0) || p->sigma < 0.0) return ORACLE_EINVAL;
  if (!(p->rho_l > 0 && p->rho_g > 0 && p->rho_s > 0)) return ORACLE_EINVAL;
  /* tau_f = mu/(rho cs^2) + 1/2 > 1/2 for every phase and mixture */
  if (!(p->mu_l > 0 && p->mu_g > 0 && p->mu_s > 0)) return ORACLE_EINVAL;
  if (!(p->cp_l > 0 && p->cp_g > 0 && p->cp_s > 0 && p->cp_ref > 0)) return ORACLE_EINVAL;
  /* tau_h = k/(cp_ref cs^2) + 1/2 > 1/2 */
  if (!(p->k_l > 0 && p->k_g > 0 && p->k_s > 0)) return ORACLE_EINVAL;
  if (!(p->latent > 0)) return ORACLE_EINVAL;
  if (!(p->theta_bottom_deg > 0 && p->theta_bottom_deg < 180)) return ORACLE_EINVAL;
  if (!(p->theta_top_deg > 0 && p->theta_top_deg < 180)) return ORACLE_EINVAL;
  if (p->st_solid_mask != 0 && p->st_solid_mask != 1) return ORACLE_EINVAL;
  return ORACLE_OK;
}

static double* dalloc(size_t n) { return (double*)calloc(n ? n : 1, sizeof(double)); }

void oracle_destroy(oracle_ctx* c) {
  if (!c) return;
  double** arrs[] = {&c->g,    &c->f,    &c->h,     &c->phiu_x, &c->phiu_y, &c->fsH_prev,
                     &c->p_prev, &c->S_prev, &c->gs, &c->fs,   &c->hs,     &c->G0,
                     &c->phi,  &c->phic, &c->rho,   &c->mu,     &c->cp,     &c->kk,
                     &c->H,    &c->T,    &c->fl,    &c->fsH,    &c->fsol,   &c->mdot,
                     &c->phi_ext, &c->rho_ext, &c->p_ext, &c->S_ext, &c->gphx, &c->gphy,
                     &c->lphi, &c->grx,  &c->gry,   &c->lrho,   &c->gpx,    &c->gpy,
                     &c->lp,   &c->gSx,  &c->gSy,   &c->lS,     &c->ux,     &c->uy,
                     &c->p,    &c->S,    &c->lamnx, &c->lamny,  &c->Fi};
  for (size_t i = 0; i < sizeof(arrs) / sizeof(arrs[0]); ++i) free(*arrs[i]);
  free(c);
}

int oracle_init(const oracle_params* p, const double* phi0, const double* T0, oracle_ctx** out) {
  if (!out) return ORACLE_EINVAL;
  *out = NULL;
  int rc = oracle_validate(p);
  if (rc) return rc;
  if (!phi0 || !T0) return ORACLE_EINVAL;
  oracle_ctx* c = (oracle_ctx*)calloc(1, sizeof(*c));
  if (!c) return ORACLE_ENOMEM;
  c->P = *p;
  c->nx = p->nx;
  c->ny = p->ny;
  size_t N = (size_t)p->nx * p->ny, NE = (size_t)p->nx * (p->ny + 2);
  c->N = N;
  c->g = dalloc(9 * N); c->f = dalloc(9 * N); c->h = dalloc(9 * N);
  c->gs = dalloc(9 * N); c->fs = dalloc(9 * N); c->hs = dalloc(9 * N); c->Fi = dalloc(9 * N);
  double** singles[] = {&c->phiu_x, &c->phiu_y, &c->fsH_prev, &c->p_prev, &c->S_prev, &c->G0,
                        &c->phi,    &c->phic,   &c->rho,      &c->mu,     &c->cp,     &c->kk,
                        &c->H,      &c->T,      &c->fl,       &c->fsH,    &c->fsol,   &c->mdot,
                        &c->gphx,   &c->gphy,   &c->lphi,     &c->grx,    &c->gry,    &c->lrho,
                        &c->gpx,    &c->gpy,    &c->lp,       &c->gSx,    &c->gSy,    &c->lS,
                        &c->ux,     &c->uy,     &c->p,        &c->S,      &c->lamnx,  &c->lamny};
  for (size_t i = 0; i < sizeof(singles) / sizeof(singles[0]); ++i) *singles[i] = dalloc(N);
  c->phi_ext = dalloc(NE); c->rho_ext = dalloc(NE); c->p_ext = dalloc(NE); c->S_ext = dalloc(NE);
  if (!c->g || !c->f || !c->h || !c->gs || !c->fs || !c->hs || !c->Fi || !c->phi_ext ||
      !c->rho_ext || !c->p_ext || !c->S_ext) {
    oracle_destroy(c);
    return ORACLE_ENOMEM;
  }
  for (size_t i = 0; i < sizeof(singles) / sizeof(singles[0]); ++i)
    if (!*singles[i]) { oracle_destroy(c); return ORACLE_ENOMEM; }

  /* Initial state (the paper does not spell it out): u = 0, p = 0, the
   * liquid fraction is 1 everywhere so H0 = cp T0 + L, every lattice starts
   * at its equilibrium, and the lagged fields start from that state so the
   * first mass source is zero. */
  for (size_t k = 0; k < N; ++k) {
    if (!isfinite(phi0[k]) || !isfinite(T0[k])) { oracle_destroy(c); return ORACLE_EINVAL; }
    double phc = clamp01(phi0[k]);
    double cp = mix(0.0, phc, p->cp_s, p->cp_l, p->cp_g);
    double H0 = cp * T0[k] + p->latent;
    double fl, T;
    oracle_enthalpy(H0, cp, p->T_melt, p->latent, &fl, &T);
    double e[9];
    oracle_geq(phi0[k], 0.0, 0.0, e);
    for (int i = 0; i < 9; ++i) c->g[i * N + k] = e[i];
    oracle_feq(0.0, mix(0.0, phc, p->rho_s, p->rho_l, p->rho_g), 0.0, 0.0, e);
    for (int i = 0; i < 9; ++i) c->f[i * N + k] = e[i];
    oracle_heq(H0, T, cp, p->cp_ref, 0.0, 0.0, e);
    for (int i = 0; i < 9; ++i) c->h[i * N + k] = e[i];
    c->fsH_prev[k] = 1.0 - fl;
    c->phiu_x[k] = c->phiu_y[k] = 0.0;
    c->p_prev[k] = c->S_prev[k] = 0.0;
  }
  c->step = 0;
  *out = c;
  return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* The step, pass by pass                                              */
/* ------------------------------------------------------------------ */

/* Pass 1: pull streaming of all three lattices (left-hand sides of Eq. (21),
 * (27), (30)).  x is periodic.  At the walls (half a spacing beyond the
 * first/last row) the half-way bounce-back gives no flux for g and no slip
 * for f; h uses the anti-bounce-back ("general bounce-back") Dirichlet rule
 * h_i = -h_opp + 2 w_i cp_ref T_w at the bottom and plain bounce-back
 * (adiabatic) at the top (Sec. 4.1). */
static void pass_stream(oracle_ctx* c) {
  const int nx = c->nx, ny = c->ny;
  const size_t N = c->N;
  const double cpr = c->P.cp_ref, Tw = c->P.T_bottom;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      size_t k = (size_t)y * nx + x;
      for (int i = 0; i < 9; ++i) {
        int sy = y - CY[i];
        int sx = ((x - CX[i]) % nx + nx) % nx;
        size_t d = (size_t)i * N + k;
        if (sy < 0) {
          size_t o = (size_t)OPP[i] * N + k;
          c->gs[d] = c->g[o];
          c->fs[d] = c->f[o];
          c->hs[d] = -c->h[o] + 2.0 * WT[i] * cpr * Tw;
        } else if (sy >= ny) {
          size_t o = (size_t)OPP[i] * N + k;
          c->gs[d] = c->g[o];
          c->fs[d] = c->f[o];
          c->hs[d] = c->h[o];
        } else {
          size_t s = (size_t)i * N + (size_t)sy * nx + sx;
          c->gs[d] = c->g[s];
          c->fs[d] = c->f[s];
          c->hs[d] = c->h[s];
        }
      }
    }
  }
}

/* Pass 2: node-local macroscopic quantities.
 *  - H = sum h_i (Eq. (29)); f_l and T from Eq. (9), with the mixture heat
 *    capacity of Eq. (1) built from the previous step's solid fraction
 *    (reading: cp and k depend on f_s which depends on T, so they are lagged);
 *  - solid fraction of the enthalpy rule f_s^H = 1 - f_l;
 *  - mass source mdot = (1 - rho_s/rho_l) d f_s/dt (Eq. (19)), backward
 *    Euler like Eq. (37), masked by clamp(sum g) so gas never acts as source;
 *  - phi from Eq. (26) with div(u) = mdot, solved for phi;
 *  - f_s = clamp(phi) f_s^H, then rho and mu from Eq. (1). */
static void pass_macro(oracle_ctx* c) {
  const oracle_params* P = &c->P;
  const size_t N = c->N;
  const double gam = P->rho_s / P->rho_l;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < c->ny; ++y) {
    for (int x = 0; x < c->nx; ++x) {
      size_t k = (size_t)y * c->nx + x;
      double G0 = 0.0, H = 0.0;
      for (int i = 0; i < 9; ++i) {
        G0 += c->gs[(size_t)i * N + k];
        H += c->hs[(size_t)i * N + k];
      }
      double phc0 = clamp01(G0);
      double fs_lag = phc0 * c->fsH_prev[k];
      double cp = mix(fs_lag, phc0, P->cp_s, P->cp_l, P->cp_g);
      double kk = mix(fs_lag, phc0, P->k_s, P->k_l, P->k_g);
      double fl, T;
      oracle_enthalpy(H, cp, P->T_melt, P->latent, &fl, &T);
      double fsH = 1.0 - fl;
      double mdot = (1.0 - gam) * phc0 * (fsH - c->fsH_prev[k]);
      double phi = G0 / (1.0 - 0.5 * mdot);
      double phc = clamp01(phi);
      double fsol = phc * fsH;
      c->G0[k] = G0;
      c->H[k] = H;
      c->cp[k] = cp;
      c->kk[k] = kk;
      c->fl[k] = fl;
      c->T[k] = T;
      c->fsH[k] = fsH;
      c->mdot[k] = mdot;
      c->phi[k] = phi;
      c->phic[k] = phc;
      c->fsol[k] = fsol;
      c->rho[k] = mix(fsol, phc, P->rho_s, P->rho_l, P->rho_g);
      c->mu[k] = mix(fsol, phc, P->mu_s, P->mu_l, P->mu_g);
    }
  }
}

/* Pass 3: ghost rows below row 0 and above row ny-1.
 *  - phi from the wetting condition Eq. (39)-(41);
 *  - rho from Eq. (1) with the ghost phi and the adjacent row's f_s^H;
 *  - the lagged p and S copy the adjacent row (zero normal gradient). */
static void pass_ghost(oracle_ctx* c) {
  const oracle_params* P = &c->P;
  const int nx = c->nx, ny = c->ny;
  memcpy(c->phi_ext + nx, c->phi, c->N * sizeof(double));
  memcpy(c->rho_ext + nx, c->rho, c->N * sizeof(double));
  memcpy(c->p_ext + nx, c->p_prev, c->N * sizeof(double));
  memcpy(c->S_ext + nx, c->S_prev, c->N * sizeof(double));
  double* gb = c->phi_ext;                            /* row y = -1 */
  double* gt = c->phi_ext + (size_t)(ny + 1) * nx;    /* row y = ny */
  oracle_wetting_ghost(nx, P->theta_bottom_deg, c->phi, c->phi + nx, gb);
  oracle_wetting_ghost(nx, P->theta_top_deg, c->phi + (size_t)(ny - 1) * nx,
                       c->phi + (size_t)(ny - 2) * nx, gt);
  for (int x = 0; x < nx; ++x) {
    double pcb = clamp01(gb[x]), pct = clamp01(gt[x]);
    double fsb = pcb * c->fsH[x];
    double fst = pct * c->fsH[(size_t)(ny - 1) * nx + x];
    c->rho_ext[x] = mix(fsb, pcb, P->rho_s, P->rho_l, P->rho_g);
    c->rho_ext[(size_t)(ny + 1) * nx + x] = mix(fst, pct, P->rho_s, P->rho_l, P->rho_g);
    c->p_ext[x] = c->p_prev[x];
    c->S_ext[x] = c->S_prev[x];
    c->p_ext[(size_t)(ny + 1) * nx + x] = c->p_prev[(size_t)(ny - 1) * nx + x];
    c->S_ext[(size_t)(ny + 1) * nx + x] = c->S_prev[(size_t)(ny - 1) * nx + x];
  }
}

/* Pass 4: isotropic stencils, Eq. (38).  phi and rho are taken at the
 * current time (as the stencil definition states); p and S come from the
 * previous step, because p at this step needs F_0 which needs grad p. */
static void pass_gradients(oracle_ctx* c) {
  oracle_stencil(c->nx, c->ny, c->phi_ext, c->gphx, c->gphy, c->lphi);
  oracle_stencil(c->nx, c->ny, c->rho_ext, c->grx, c->gry, c->lrho);
  oracle_stencil(c->nx, c->ny, c->p_ext, c->gpx, c->gpy, c->lp);
  oracle_stencil(c->nx, c->ny, c->S_ext, c->gSx, c->gSy, c->lS);
}

/* Pass 5: interface terms, forces, velocity, source and pressure.
 *  - lambda = 4 phi (1-phi)/W and n = grad phi/|grad phi| (Eq. (3));
 *  - mu_phi = 4 beta phi (phi-1)(phi-1/2) - kappa lap(phi) with
 *    kappa = 3 sigma W / 2 and beta = 12 sigma / W (Eq. (12)-(13));
 *  - F_s = mu_phi grad(phi) (Eq. (11)); for bubble cases the force is kept
 *    only outside the solid, (1 - chi f_s) mu_phi grad(phi) (Sec. 4.3);
 *  - G = rho g plus an optional Boussinesq term -rho0 beta (T-Tref) g;
 *  - rho u* = sum c_i f_i + F/2 (Eq. (34)); f = f_s (u_s - u*) with u_s = 0
 *    and u = u* + f/2 (Eq. (35) and the fluid-solid force of Sec. 3.3);
 *  - S = rho mdot + u.grad(rho), Ft = F - grad p + cs^2 grad rho
 *    + cs^2 grad S (the printed "div S" of a scalar read as its gradient);
 *  - forcing F_i (Eq. (33)) and pressure (Eq. (36)) with tau_f = 3 mu/rho + 1/2. */
static void pass_flow(oracle_ctx* c) {
  const oracle_params* P = &c->P;
  const size_t N = c->N;
  const double beta = 12.0 * P->sigma / P->W;
  const double kappa = 1.5 * P->sigma * P->W;
  const double chi = (double)P->st_solid_mask;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < c->ny; ++y) {
    for (int x = 0; x < c->nx; ++x) {
      size_t k = (size_t)y * c->nx + x;
      double phi = c->phi[k], rho = c->rho[k];
      double lam = 4.0 * phi * (1.0 - phi) / P->W;
      double gpx = c->gphx[k], gpy = c->gphy[k];
      double gn = sqrt(gpx * gpx + gpy * gpy);
      double nxv = 0.0, nyv = 0.0;
      if (gn > 1e-12) { nxv = gpx / gn; nyv = gpy / gn; }
      c->lamnx[k] = lam * nxv;
      c->lamny[k] = lam * nyv;
      double muphi = 4.0 * beta * phi * (phi - 1.0) * (phi - 0.5) - kappa * c->lphi[k];
      double mask = 1.0 - chi * c->fsol[k];
      double Fx = mask * muphi * gpx, Fy = mask * muphi * gpy;
      double bq = -P->bq_rho0 * P->bq_beta * (c->T[k] - P->bq_Tref);
      Fx += rho * P->gx + bq * P->gx;
      Fy += rho * P->gy + bq * P->gy;
      double mx = 0.0, my = 0.0, f9[9];
      for (int i = 0; i < 9; ++i) {
        f9[i] = c->fs[(size_t)i * N + k];
        mx += CX[i] * f9[i];
        my += CY[i] * f9[i];
      }
      double usx = (mx + 0.5 * Fx) / rho, usy = (my + 0.5 * Fy) / rho;
      double fbx = c->fsol[k] * (0.0 - usx), fby = c->fsol[k] * (0.0 - usy);
      double ux = usx + 0.5 * fbx, uy = usy + 0.5 * fby;
      double S = rho * c->mdot[k] + ux * c->grx[k] + uy * c->gry[k];
      double Ftx = Fx - c->gpx[k] + CS2 * c->grx[k] + CS2 * c->gSx[k];
      double Fty = Fy - c->gpy[k] + CS2 * c->gry[k] + CS2 * c->gSy[k];
      double Fi[9];
      oracle_fforce(S, Fx, Fy, rho * fbx, rho * fby, ux, uy, Ftx, Fty, Fi);
      for (int i = 0; i < 9; ++i) c->Fi[(size_t)i * N + k] = Fi[i];
      double tauf = c->mu[k] / (rho * CS2) + 0.5;
      double p;
      oracle_pressure(f9, S, Fi[0], tauf, rho, ux, uy, &p);
      c->ux[k] = ux;
      c->uy[k] = uy;
      c->S[k] = S;
      c->p[k] = p;
    }
  }
}

/* Pass 6: the three BGK collisions and the stored history.
 *  - flow, Eq. (30): f+ = f - (f - f^eq)/tau_f + (1 - 1/(2 tau_f)) F_i;
 *  - phase field, Eq. (21): g+ = g - (g - g^eq)/tau_g + (1 - 1/(2 tau_g)) G_i,
 *    with d_t(phi u) by Eq. (37) and tau_g from M = cs^2 (tau_g - 1/2)
 *    (the printed tau_f read as tau_g);
 *  - enthalpy, Eq. (27): h+ = h - (h - h^eq)/tau_h, with
 *    k = cp_ref cs^2 (tau_h - 1/2) (the paper does not relate tau_h to k). */
static void pass_collide(oracle_ctx* c) {
  const oracle_params* P = &c->P;
  const size_t N = c->N;
  const double taug = P->M / CS2 + 0.5;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < c->ny; ++y) {
    for (int x = 0; x < c->nx; ++x) {
      size_t k = (size_t)y * c->nx + x;
      double rho = c->rho[k], ux = c->ux[k], uy = c->uy[k], phi = c->phi[k];
      double tauf = c->mu[k] / (rho * CS2) + 0.5;
      double e[9], src[9];
      oracle_feq(c->p[k], rho, ux, uy, e);
      for (int i = 0; i < 9; ++i) {
        size_t d = (size_t)i * N + k;
        c->f[d] = c->fs[d] - (c->fs[d] - e[i]) / tauf + (1.0 - 0.5 / tauf) * c->Fi[d];
      }
      double dphiux = phi * ux - c->phiu_x[k], dphiuy = phi * uy - c->phiu_y[k];
      oracle_geq(phi, ux, uy, e);
      oracle_gsrc(phi, dphiux, dphiuy, c->lamnx[k], c->lamny[k], c->mdot[k], src);
      for (int i = 0; i < 9; ++i) {
        size_t d = (size_t)i * N + k;
        c->g[d] = c->gs[d] - (c->gs[d] - e[i]) / taug + (1.0 - 0.5 / taug) * src[i];
      }
      double tauh = c->kk[k] / (P->cp_ref * CS2) + 0.5;
      oracle_heq(c->H[k], c->T[k], c->cp[k], P->cp_ref, ux, uy, e);
      for (int i = 0; i < 9; ++i) {
        size_t d = (size_t)i * N + k;
        c->h[d] = c->hs[d] - (c->hs[d] - e[i]) / tauh;
      }
      c->phiu_x[k] = phi * ux;
      c->phiu_y[k] = phi * uy;
      c->fsH_prev[k] = c->fsH[k];
      c->p_prev[k] = c->p[k];
      c->S_prev[k] = c->S[k];
    }
  }
}

static void macro_passes(oracle_ctx* c) {
  pass_stream(c);
  pass_macro(c);
  pass_ghost(c);
  pass_gradients(c);
  pass_flow(c);
}

int oracle_step(oracle_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return ORACLE_EINVAL;
  for (int32_t s = 0; s < nsteps; ++s) {
    macro_passes(c);
    pass_collide(c);
    c->step++;
  }
  return ORACLE_OK;
}

int oracle_fields(oracle_ctx* c, uint32_t mask, double* const* out) {
  if (!c || !out) return ORACLE_EINVAL;
  macro_passes(c);
  const double* src[10] = {c->phi, c->T, c->ux, c->uy, c->p, c->fsol, c->fl, c->rho, c->H, c->mdot};
  int j = 0;
  for (int b = 0; b < 10; ++b) {
    if (mask & (1u << b)) {
      if (!out[j]) return ORACLE_EINVAL;
      memcpy(out[j], src[b], c->N * sizeof(double));
      ++j;
    }
  }
  return ORACLE_OK;
}

int oracle_diag(oracle_ctx* c, oracle_diag_t* d) {
  if (!c || !d) return ORACLE_EINVAL;
  macro_passes(c);
  memset(d, 0, sizeof(*d));
  d->step = c->step;
  int bad = 0;
  for (size_t k = 0; k < c->N; ++k) {
    double ph = c->phi[k], pc = clamp01(ph);
    double um = sqrt(c->ux[k] * c->ux[k] + c->uy[k] * c->uy[k]);
    d->sum_phi += ph;
    d->sum_phic += pc;
    d->sum_solid += pc * c->fsH[k];
    d->sum_liquid += pc * c->fl[k];
    d->sum_H += c->H[k];
    if (um > d->max_u) d->max_u = um;
    if (!isfinite(ph) || !isfinite(c->T[k]) || !isfinite(um) || !isfinite(c->p[k])) bad = 1;
  }
  int xc = c->nx / 2;
  for (int y = 0; y < c->ny; ++y) {
    size_t k = (size_t)y * c->nx + xc;
    d->h_c += clamp01(c->phi[k]) * c->fsH[k];
  }
  d->nonfinite = bad;
  return bad ? ORACLE_ENONFINITE : ORACLE_OK;
}

int oracle_pops(oracle_ctx* c, int32_t lattice, double* out) {
  if (!c || !out || lattice < 0 || lattice > 2) return ORACLE_EINVAL;
  const double* src = lattice == 0 ? c->g : (lattice == 1 ? c->f : c->h);
  memcpy(out, src, 9 * c->N * sizeof(double));
  return ORACLE_OK;
}

/* checkpoint: header (4 x int64: magic, nx, ny, step) + 32 N doubles */
#define ORACLE_MAGIC 0x4f52434c4250484cLL
size_t oracle_state_bytes(const oracle_ctx* c) {
  return c ? 4 * sizeof(int64_t) + 32 * c->N * sizeof(double) : 0;
}

int oracle_save(const oracle_ctx* c, void* buf, size_t bytes) {
  if (!c || !buf || bytes < oracle_state_bytes(c)) return ORACLE_EINVAL;
  int64_t hdr[4] = {ORACLE_MAGIC, c->nx, c->ny, c->step};
  char* o = (char*)buf;
  memcpy(o, hdr, sizeof(hdr));
  o += sizeof(hdr);
  size_t n9 = 9 * c->N * sizeof(double), n1 = c->N * sizeof(double);
  memcpy(o, c->g, n9); o += n9;
  memcpy(o, c->f, n9); o += n9;
  memcpy(o, c->h, n9); o += n9;
  memcpy(o, c->phiu_x, n1); o += n1;
  memcpy(o, c->phiu_y, n1); o += n1;
  memcpy(o, c->fsH_prev, n1); o += n1;
  memcpy(o, c->p_prev, n1); o += n1;
  memcpy(o, c->S_prev, n1);
  return ORACLE_OK;
}

int oracle_load(oracle_ctx* c, const void* buf, size_t bytes) {
  if (!c || !buf || bytes < oracle_state_bytes(c)) return ORACLE_EINVAL;
  int64_t hdr[4];
  const char* o = (const char*)buf;
  memcpy(hdr, o, sizeof(hdr));
  if (hdr[0] != ORACLE_MAGIC || hdr[1] != c->nx || hdr[2] != c->ny) return ORACLE_ESTATE;
  o += sizeof(hdr);
  size_t n9 = 9 * c->N * sizeof(double), n1 = c->N * sizeof(double);
  memcpy(c->g, o, n9); o += n9;
  memcpy(c->f, o, n9); o += n9;
  memcpy(c->h, o, n9); o += n9;
  memcpy(c->phiu_x, o, n1); o += n1;
  memcpy(c->phiu_y, o, n1); o += n1;
  memcpy(c->fsH_prev, o, n1); o += n1;
  memcpy(c->p_prev, o, n1); o += n1;
  memcpy(c->S_prev, o, n1);
  c->step = hdr[3];
  return ORACLE_OK;
}

int64_t oracle_step_count(const oracle_ctx* c) { return c ? c->step : -1; }

void oracle_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
