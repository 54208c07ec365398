/*
 * FP64 CPU oracle for the phase-field lattice Boltzmann freezing step
 * (Huang, Wang, Chai & Shi, "Phase-field based lattice Boltzmann method for
 * containerless freezing", arXiv:2403.16122).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a plain, slow, obviously correct implementation.  Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header or table with the GPU library.
 *
 * Units are lattice units (dx = dt = 1, cs^2 = 1/3).  Node (x, y) has index
 * k = y*nx + x; x is periodic; walls sit at y = -1/2 and y = ny - 1/2.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nx, ny;
  double W, M, sigma;
  double rho_l, rho_g, rho_s, mu_l, mu_g, mu_s;
  double cp_l, cp_g, cp_s, cp_ref, k_l, k_g, k_s;
  double latent, T_melt, T_bottom;
  double theta_bottom_deg, theta_top_deg;
  double gx, gy;
  double bq_beta, bq_rho0, bq_Tref;
  int32_t st_solid_mask;
  int32_t storage; /* ignored by the oracle (always FP64) */
} oracle_params;

typedef struct {
  int64_t step;
  double sum_phi;        /* sum of phi                                  */
  double sum_phic;       /* sum of clamp(phi,0,1)                       */
  double sum_solid;      /* sum of clamp(phi) * f_s^H                   */
  double sum_liquid;     /* sum of clamp(phi) * f_l                     */
  double sum_H;          /* sum of total enthalpy H                     */
  double max_u;          /* max |u|                                     */
  double h_c;            /* solid height on the centre column           */
  int32_t nonfinite;     /* 1 if any field is NaN/Inf                   */
} oracle_diag_t;

typedef struct oracle_ctx oracle_ctx;

enum {
  ORACLE_OK = 0,
  ORACLE_EINVAL = -1,
  ORACLE_ENOMEM = -2,
  ORACLE_ENONFINITE = -4,
  ORACLE_ESTATE = -5
};

/* field selection bits for oracle_fields */
enum {
  ORF_PHI = 1u << 0, ORF_T = 1u << 1, ORF_UX = 1u << 2, ORF_UY = 1u << 3,
  ORF_P = 1u << 4, ORF_FS = 1u << 5, ORF_FL = 1u << 6, ORF_RHO = 1u << 7,
  ORF_H = 1u << 8, ORF_MDOT = 1u << 9
};

int oracle_validate(const oracle_params* p);
int oracle_init(const oracle_params* p, const double* phi0, const double* T0, oracle_ctx** out);
int oracle_step(oracle_ctx* c, int32_t nsteps);
/* Macroscopic fields at the current time level (the macro part of a step,
 * without collision); out[j] receives the j-th set bit's field (nx*ny). */
int oracle_fields(oracle_ctx* c, uint32_t mask, double* const* out);
int oracle_diag(oracle_ctx* c, oracle_diag_t* d);
/* Post-collision populations of lattice 0=g,1=f,2=h: out[i*N + k]. */
int oracle_pops(oracle_ctx* c, int32_t lattice, double* out);
size_t oracle_state_bytes(const oracle_ctx* c);
int oracle_save(const oracle_ctx* c, void* buf, size_t bytes);
int oracle_load(oracle_ctx* c, const void* buf, size_t bytes);
int64_t oracle_step_count(const oracle_ctx* c);
void oracle_set_threads(int32_t n);
void oracle_destroy(oracle_ctx* c);

/* ---- per-node building blocks, exported for the algebraic pins ---- */
void oracle_geq(double phi, double ux, double uy, double* out9);
void oracle_gsrc(double phi, double dphiux, double dphiuy, double lnx, double lny,
                 double mdot, double* out9);
void oracle_feq(double p, double rho, double ux, double uy, double* out9);
void oracle_fforce(double S, double Fx, double Fy, double rfx, double rfy,
                   double ux, double uy, double Ftx, double Fty, double* out9);
void oracle_heq(double H, double T, double cp, double cp_ref, double ux, double uy, double* out9);
void oracle_pressure(const double* f9, double S, double F0, double tau_f, double rho,
                     double ux, double uy, double* p_out);
void oracle_enthalpy(double H, double cp, double T_melt, double latent, double* fl, double* T);
/* Isotropic gradient/Laplacian on an (ny+2) x nx array whose first and last
 * rows are ghost rows; outputs are ny x nx. */
void oracle_stencil(int32_t nx, int32_t ny, const double* ext, double* gx, double* gy, double* lap);
/* Wetting ghost value below row 0 (or above row ny-1): rows r0 = adjacent
 * fluid row, r1 = next row, each nx long. */
void oracle_wetting_ghost(int32_t nx, double theta_deg, const double* r0, const double* r1, double* ghost);

#ifdef __cplusplus
}
#endif
#endif
