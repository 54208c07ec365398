// Internal definitions shared by the host side (lbm_api.hip) and the
// kernels (lbm_kernels.hip) of the gfx950 solver.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lbm.h"

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
  unsigned seed;                   // 16-bit storage: step number, seeds the stochastic rounding
  int stream_stores;               // host-side launch choice: streaming (non-temporal) stores
};

// Resident state beyond this (MI355X's Infinity Cache) cannot stay cached from
// one step's stores to the next step's loads: the step then streams its stores.
constexpr size_t kInfinityCacheBytes = size_t(256) << 20;

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

// Buffers one step reads (time n) and writes (time n+1).  The step is a
// pure function of the *_in buffers, so it can be replayed for timing.
struct StepIO {
  const void* A;  // populations of time n (storage type of the instantiation)
  void* B;        // populations of time n+1
  const float* phiu_in;
  float* phiu_out;
  const void* ref_in;  // node references (FP32 phi_ref, or FP16 pairs (phi_ref, th))
  void* ref_out;
  const float* fsH_in;
  float* fsH_out;
  const float* p_in;
  float* p_out;
  const float* S_in;
  float* S_out;
  float* fields;
};


__host__ __device__ inline StepIO make_io(const State& S, int cur) {
  const int nxt = cur ^ 1;
  return StepIO{S.pops[cur], S.pops[nxt], S.phiu[cur], S.phiu[nxt], S.ref[cur], S.ref[nxt],
                S.fsH[cur], S.fsH[nxt], S.p[cur], S.p[nxt], S.S[cur], S.S[nxt], S.fields};
}

// The buffer set of one grid of a batch as byte offsets from the batch's
// workspace base.  The kernels rebuild the pointers from the base they get
// as an argument, so the compiler knows every access is to global memory.
struct StepOff {
  unsigned long long A, B, phiu_in, phiu_out, ref_in, ref_out, fsH_in, fsH_out, p_in, p_out, S_in, S_out, fields;
};

enum { NFIELD = 10 };
// tiles 64x4, 32x8, 64x8, 64x16, 128x4; 5: unfused two-kernel 64x8; 6, 7, 8:
// two steps per launch on 64x8, 32x8, 32x16 tiles; 9, 10: the same on 32x16
// and 32x8 tiles with two and three lanes per tile node (these two in every
// storage format; 6-8 FP32 only)
enum { NTILE_VARIANTS = 11, TWO_STEP_VARIANT = 6, NTWO_STEP_VARIANTS = 5 };
inline bool is_two_step(int tile_variant) {
  return tile_variant >= TWO_STEP_VARIANT && tile_variant < TWO_STEP_VARIANT + NTWO_STEP_VARIANTS;
}
// Two-step variants with more lanes than tile nodes (32x16 / 1024 lanes and
// 32x8 / 768 lanes): built for every storage format and for batches.
inline bool is_two_step_any_storage(int tile_variant) {
  return tile_variant == TWO_STEP_VARIANT + 3 || tile_variant == TWO_STEP_VARIANT + 4;
}
enum { NTUNED_VARIANTS = 5 };  // single-step shapes the autotuner times (plus the two-step ones)
enum { NXCD_MODES = 3 };      // workgroup -> tile orders (map_tile)
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
// Two steps n -> n+2 in one launch (variants 6-8 FP32 storage only, 9-10
// every format; steps P.seed and P.seed + 1): reads buffer cur, writes
// buffer cur^1, like one step.
int launch_step2(const KParams& P, const State& S, int cur, int tile_variant, int xcd_remap, hipStream_t st);
// nsteps single steps n -> n + nsteps (steps P.seed, P.seed + 1, ...) in one
// cooperative launch on 64x8 tiles, with a grid-wide barrier between steps:
// every workgroup writes its XCD's L2 back (per_xcd 0), or the last
// workgroup to arrive on each XCD does it for all (per_xcd 1).  bar:
// NPERSIST_WORDS 64-bit words of device memory (zeroed here on the stream):
// [0] flat-barrier arrivals, [1] nonzero if a wait exceeded limit_ticks of
// the device's wall clock, [2] XCD arrivals, [3..10] workgroup arrivals per
// XCD, [11..18] workgroups per XCD.  *grid_out receives the number of
// workgroups.  Returns the runtime's error, hipErrorNotSupported without
// cooperative launches, or hipErrorCooperativeLaunchTooLarge if no grid fits.
enum { NPERSIST_WORDS = 19 };
hipError_t launch_persist(const KParams& P, const State& S, int cur, int nsteps, int xcd_remap, int per_xcd,
                          unsigned long long* bar, unsigned long long limit_ticks, int* grid_out, hipStream_t st);
// The 9 populations of `lattice` as FP32 (shifted variables) into the first
// nine field planes.
int launch_expand(const KParams& P, const State& S, int cur, int lattice, hipStream_t st);
// Reduces the field planes into RED_NVAL doubles at part[RED_BLOCKS * RED_NVAL].
int launch_reduce(const KParams& P, const State& S, double Href, hipStream_t st);

// ---- host-side set-up shared by the single-grid and batch contexts --------
int validate_params(const lbm_params* p);
size_t pop_bytes(int storage);
long long plane_floats(long long nodes);
// Bytes of one grid's state (both population buffers, history planes and
// the NFIELD output planes) at the given plane stride; carve_state lays it
// out from `base` (S.part is left alone).
size_t state_bytes(long long plane, int storage);
void carve_state(State& S, char* base, long long plane, int storage);
// Kernel constants of p (K.plane = nx*ny rounded up to 64).
void fill_constants(const lbm_params& p, KParams& K, IParams& I, double& Href);
// Storage-dependent constants from the initial temperature; LBM_EINVAL if
// the temperature span does not fit the FP16 references of 16-bit storage.
int storage_setup(const lbm_params& p, const double* T0, long long N, KParams& K);

// ---- batches of grids ------------------------------------------------------
enum { NBATCH_VARIANTS = 5 };  // the tile shapes of variants 0..4
void tile_shape(int tile_variant, int* tx, int* ty);
// Step s (0-based, even at a sample) of a sampling interval, or the fields
// pass (s = 0), for every tile listed in d_tmap (nblocks entries:
// slot << 16 | tile, ~0u = none), with the per-slot constants d_ptab[slot],
// buffer sets d_otab[2 slot + (s & 1)] (offsets from d_base) and step
// numbers d_steps[slot] + s (seeds of the stochastic rounding).  Tile
// variants 0-4 (single steps), and 9-10 (steps s and s + 1 in one launch,
// s even, buffer set (s / 2) & 1; their fields pass runs single-step tiles
// of the same shape).
int launch_batch(int storage, int tile_variant, bool fields_only, bool stream_stores, char* d_base,
                 const KParams* d_ptab,
                 const StepOff* d_otab, const unsigned* d_tmap, const unsigned* d_steps, int nblocks, int s,
                 hipStream_t st);
// Steps 0 .. nsteps-1 of a sampling interval (as nsteps launch_batch calls
// of tile variant 2, 64x8) in one cooperative launch, with the grid barrier
// of launch_persist between steps (per_xcd 0 flat, 1 per XCD) and the same
// barrier words; d_tmap must be the map of 64x8 tiles.
hipError_t launch_batch_persist(int storage, bool stream_stores, int per_xcd, char* d_base, const KParams* d_ptab,
                                const StepOff* d_otab, const unsigned* d_tmap, const unsigned* d_steps, int nblocks,
                                int nsteps, unsigned long long* bar, unsigned long long limit_ticks, int* grid_out,
                                hipStream_t st);
// Per listed slot (d_slots, nslots entries), from its field planes:
// out[2 slot] = sum clamp(phi) f_l (liquid volume), out[2 slot + 1] = number
// of non-finite phi, T, u values.
int launch_batch_liquid(const char* d_base, const KParams* d_ptab, const StepOff* d_otab, const int* d_slots,
                        int nslots, double* d_out, hipStream_t st);
// Per listed slot, shape of the phi = 1/2 contour from its field planes:
// out[4 slot + 0..3] = height above the wall, base half-width on row 0,
// tip angle in degrees, number of contour points in the tip fit.
int launch_batch_shape(const char* d_base, const KParams* d_ptab, const StepOff* d_otab, const int* d_slots,
                       int nslots, double* d_out, hipStream_t st);

}  // namespace lbmk
