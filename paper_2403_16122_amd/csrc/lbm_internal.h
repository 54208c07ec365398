// Internal definitions shared by the host side (lbm_api.hip) and the
// kernels (lbm_kernels.hip) of the gfx950 solver.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbmk {

// Precomputed lattice-unit constants handed to every kernel by value.
struct KParams {
  int nx, ny;
  unsigned plane;  // floats per population/field plane (padded to 64); every index fits 32 bits
  // phase field (Sec. 3.1)
  float inv_tau_g, src_g;          // 1/tau_g and 1 - 1/(2 tau_g)
  float four_over_W, beta4, kappa; // 4/W, 4 beta, kappa
  // Eq. (1) property values
  float rho_s, rho_l, rho_g, mu_s, mu_l, mu_g, cp_s, cp_l, cp_g, k_s, k_l, k_g;
  // enthalpy model (Sec. 3.2); h is stored as the deviation from the
  // equilibrium of liquid at rest at T_melt (shift is exact algebra)
  float cp_ref, T_melt, latent, inv_latent, three_over_cpref;
  float hwall[9];                  // anti-bounce-back constant 2 w_i cp_ref (T_w - T_m)
  float mdot_coef;                 // 1 - rho_s/rho_l (Eq. (19))
  float tan_b, tan_t;              // tan(pi/2 - theta) at the bottom / top wall
  float gx, gy, bq_coef, bq_Tref;  // body force
  float chi;                       // surface-tension solid mask
  int storage;                     // STORE_FP32 / STORE_FP16 / STORE_BF16
  float sc_st[3], sc_ld[3];        // FP16 only: per-lattice power-of-two scale on store / load
};

enum { STORE_FP32 = 0, STORE_FP16 = 1, STORE_BF16 = 2 };

struct State {
  void* pops[2];   // 27 planes each: g0..g8, f0..f8, h0..h8 (FP32, FP16 or BF16)
  float* phiu[2];  // 2 planes each: (phi u)^{n-1}
  void* ref[2];    // node references of the stored populations: FP32 phi_ref, or
                   // (16-bit storage) FP16 pairs (phi_ref, T - T_m)
  float* fsH[2];   // f_s^H of the previous step (read n-1, write n)
  float* p[2];     // pressure of the previous step
  float* S[2];     // mass-source term S of the previous step
  float* fields;   // 10 planes of output fields
  double* part;    // reduction scratch
};

enum { NFIELD = 10 };
enum { NTILE_VARIANTS = 8 };  // tiles 64x4, 32x8, 64x8, 64x16, 128x4; strips 60x32, 60x64, 60x128
enum { RED_NVAL = 8 };
constexpr int RED_BLOCKS = 512;

// FP64 constants for building the initial state.
struct IParams {
  double cp_l, cp_g, cp_ref, T_melt, latent;
};

int launch_init(const KParams& P, const IParams& I, const State& S, int cur, const double* d_phi0,
                const double* d_T0, hipStream_t st);
int launch_step(const KParams& P, const State& S, int cur, bool fields_only, int tile_variant,
                int xcd_remap, hipStream_t st);
// The 9 populations of `lattice` as FP32 (shifted variables) into the first
// nine field planes.
int launch_expand(const KParams& P, const State& S, int cur, int lattice, hipStream_t st);
// Reduces the field planes into RED_NVAL doubles at part[RED_BLOCKS * RED_NVAL].
int launch_reduce(const KParams& P, const State& S, double Href, hipStream_t st);

}  // namespace lbmk
