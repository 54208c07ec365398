/*
 * lbm.h -- C ABI of the MI355X (gfx950) solver for the phase-field lattice
 * Boltzmann method for containerless freezing of Huang, Wang, Chai & Shi
 * (arXiv:2403.16122).
 *
 * One time step updates three coupled D2Q9 lattices:
 *   g  conservative Allen-Cahn phase field with the dilatation term phi div(u)
 *      (Sec. 3.1, Eq. (21)-(26)),
 *   f  pressure/velocity flow model with surface tension mu_phi grad(phi),
 *      body force, the fluid-solid force rho f and the freezing mass source
 *      (Sec. 3.3, Eq. (30)-(36), mass source Eq. (19)),
 *   h  total-enthalpy model with the liquid-fraction rule (Sec. 3.2,
 *      Eq. (27)-(29), enthalpy rule Eq. (9)),
 * on a rectangular domain that is periodic in x, with walls half a spacing
 * below row 0 and above row ny-1: half-way bounce-back for g and f,
 * anti-bounce-back Dirichlet temperature at the bottom, adiabatic top, and
 * the geometric wetting condition of Eq. (39)-(41) at both walls (Sec. 4.1).
 * All quantities are in lattice units (dx = dt = 1, cs^2 = 1/3).
 *
 * Layout.  Node (x, y) has index k = y*nx + x; host arrays are row-major
 * with nx*ny doubles.  Device state lives in one caller-provided workspace.
 *
 * Errors.  Every call returns LBM_OK (0) or a negative code; no exception
 * crosses this boundary.  Kernel faults surface at the next call that
 * synchronises (lbm_fields, lbm_diag, lbm_save, lbm_sync).
 *
 * Threading.  A context is bound to one device and one stream; calls on
 * one context must not overlap.
 */
#ifndef LBM_H
#define LBM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* bad argument: sizes, a relaxation time <= 1/2, angle, workspace */
  LBM_ENOMEM = -2,     /* library-side allocation failed */
  LBM_EDEVICE = -3,    /* HIP runtime error; text from lbm_last_error() */
  LBM_ENONFINITE = -4, /* diagnostics found NaN/Inf in the fields */
  LBM_ESTATE = -5      /* checkpoint does not match this context */
};

enum {
  LBM_STORE_FP32 = 0,        /* populations stored as FP32 */
  LBM_STORE_FP16_SHIFT = 1,  /* shifted populations rounded to FP16 (per-lattice power-of-two scale) */
  LBM_STORE_BF16_SHIFT = 2   /* shifted populations rounded to BF16 */
};

/* Physical parameters in lattice units.  Mixture properties follow Eq. (1)
 * with subscripts s (solid), l (liquid), g (gas). */
typedef struct {
  int32_t nx, ny;                 /* >= 3 each; nx*ny below 39.77M nodes (FP32 storage) or
                                     79.5M (16-bit), so that one buffer spans < 4 GiB */
  double W, M, sigma;             /* interface width, mobility (tau_g = M/cs^2 + 1/2, Sec. 3.1),
                                     surface tension (beta = 12 sigma/W, kappa = 3 sigma W/2, Eq. (13)) */
  double rho_l, rho_g, rho_s;     /* densities (> 0); rho_s/rho_l sets the mass source, Eq. (19) */
  double mu_l, mu_g, mu_s;        /* dynamic viscosities (> 0); tau_f = mu/(rho cs^2) + 1/2 */
  double cp_l, cp_g, cp_s, cp_ref;/* heat capacities; cp_ref of the enthalpy equilibrium, Eq. (28) */
  double k_l, k_g, k_s;           /* conductivities (> 0); tau_h = k/(cp_ref cs^2) + 1/2 */
  double latent, T_melt, T_bottom;/* latent heat (> 0), melting temperature, bottom wall temperature */
  double theta_bottom_deg, theta_top_deg; /* contact angles in (0, 180), Eq. (39) */
  double gx, gy;                  /* gravity: body force rho*g */
  double bq_beta, bq_rho0, bq_Tref; /* optional Boussinesq force -rho0 beta (T - Tref) g (Sec. 4.3) */
  int32_t st_solid_mask;          /* 0: F_s = mu grad(phi) (Eq. (11)); 1: (1 - f_s) mu grad(phi) */
  int32_t storage;                /* LBM_STORE_FP32, LBM_STORE_FP16_SHIFT or LBM_STORE_BF16_SHIFT:
                                     the format of the stored populations; compute is FP32 */
} lbm_params;

typedef struct {
  int64_t step;
  double sum_phi, sum_phic, sum_solid, sum_liquid, sum_H, max_u;
  double h_c;  /* solid height on the centre column (the front height H_c of Sec. 4.2.1) */
  int32_t nonfinite;
} lbm_diag_t;

/* Field selection bits for lbm_fields / lbm_fields_device. */
enum {
  LBM_F_PHI = 1u << 0, LBM_F_T = 1u << 1, LBM_F_UX = 1u << 2, LBM_F_UY = 1u << 3,
  LBM_F_P = 1u << 4, LBM_F_FS = 1u << 5, LBM_F_FL = 1u << 6, LBM_F_RHO = 1u << 7,
  LBM_F_H = 1u << 8, LBM_F_MDOT = 1u << 9
};

typedef struct lbm_ctx lbm_ctx;

/* Bytes of device workspace lbm_init needs for these parameters. */
int lbm_workspace_bytes(const lbm_params* p, size_t* bytes);

/* Validate p, lay out the state in d_workspace (device memory, 256-byte
 * aligned, at least lbm_workspace_bytes; NULL lets the library allocate
 * and own it), copy phi0/T0 (host, nx*ny doubles each, read before return)
 * and build the initial state: u = 0, p = 0, liquid fraction 1, every
 * lattice at equilibrium.  hip_stream is a hipStream_t (NULL = default
 * stream).  On success *out owns the context; the caller's workspace must
 * outlive it. */
int lbm_init(const lbm_params* p, const double* phi0, const double* T0, void* d_workspace,
             size_t ws_bytes, void* hip_stream, lbm_ctx** out);

/* Enqueue nsteps >= 0 time steps on the context's stream (asynchronous).
 * One step is the update of Sec. 3 in this order: pull-streaming with the
 * wall rules of Sec. 4.1, the enthalpy rule Eq. (9) on H = sum h_i
 * (Eq. (29)), the mass source Eq. (19), the order parameter Eq. (26), the
 * mixture properties Eq. (1), the wetting ghost rows Eq. (39)-(41), the
 * stencils Eq. (38), the chemical potential and interface terms
 * Eq. (3), (12)-(13), the forces Eq. (11) (with the Boussinesq term and
 * solid mask of Sec. 4.3), the velocity and fluid-solid force Eq. (34)-(35),
 * the forcing Eq. (33), the pressure Eq. (36), and the collisions Eq. (21)
 * with (24)-(25), (37), Eq. (30)-(32) and Eq. (27)-(28).  LBM_EINVAL for a
 * negative count; launch failures give LBM_EDEVICE. */
int lbm_step(lbm_ctx* c, int32_t nsteps);

/* The same nsteps time steps (Sec. 3, as lbm_step) in ONE persistent launch:
 * a cooperative grid of co-resident workgroups on 64x8 tiles (the context's
 * xcd_remap order; its tile variant is not used) loops over the steps with a
 * grid-wide barrier between them, since every step pulls the halo its
 * neighbours wrote in the step before.  barrier LBM_BARRIER_FLAT: every
 * workgroup writes its XCD's L2 back before it arrives (the agent-scope
 * release of the HIP memory model); LBM_BARRIER_PER_XCD: the last workgroup
 * to arrive on each XCD (read from the XCC_ID hardware register) writes that
 * L2 back once for all of them.  Results are bitwise those of lbm_step in
 * both.  Kept to measure a persistent launch against one launch per step;
 * lbm_step is the faster path on MI355X.  wait_limit_us bounds one barrier
 * wait in microseconds of the device's wall clock (0: 2 s).  nsteps in
 * 0..LBM_PERSIST_MAX_STEPS, barrier 0 or 1 and wait_limit_us >= 0, else
 * LBM_EINVAL.  *workgroups (optional) receives the grid size.  Uses the
 * context's reduction scratch for the barrier words.  Synchronises.
 * LBM_EDEVICE if the device has no cooperative launch, no grid fits, or a
 * barrier wait exceeded its bound: then no workgroup waits again, every wave
 * leaves the kernel, and the context's state is invalid (load a checkpoint
 * or destroy it). */
#define LBM_PERSIST_MAX_STEPS 1000000
enum { LBM_BARRIER_FLAT = 0, LBM_BARRIER_PER_XCD = 1 };
int lbm_step_persistent(lbm_ctx* c, int32_t nsteps, int32_t barrier, int32_t wait_limit_us, int32_t* workgroups);

/* Macroscopic fields at the current time level as the next step would
 * compute them: phi (Eq. (26)), T and f_l (Eq. (9)), u (Eq. (34)-(35), with
 * the fluid-solid force), p (Eq. (36)), f_s = clamp(phi) (1 - f_l), rho
 * (Eq. (1)), H (Eq. (29)) and mdot (Eq. (19)) -- the quantities of the
 * paper's Figs. 4-11.  host_out[j] receives the j-th set bit of field_mask
 * (caller-owned, nx*ny doubles each, row-major).  LBM_EINVAL for an unknown
 * bit or a NULL output.  Synchronises. */
int lbm_fields(lbm_ctx* c, uint32_t field_mask, double* const* host_out);

/* Same fields as FP32 into device buffers (nx*ny floats each), enqueued on
 * the context's stream; no synchronisation.  H is given relative to
 * H_ref = cp_ref*T_melt + latent, as the step keeps it (lbm_fields adds H_ref
 * back in FP64; in FP32 the sum would lose the resolution of the relative
 * value). */
int lbm_fields_device(lbm_ctx* c, uint32_t field_mask, float* const* d_out);

/* FP64 sums over the grid (wave reductions in FP64 of the FP32 fields, in
 * a fixed order): sum phi (conserved exactly without freezing, Sec. 3.1),
 * sum clamp(phi), solid volume sum f_s and liquid volume sum clamp(phi) f_l
 * (the volume change of Eq. (44)), sum H (Eq. (29)), max |u|, and the solid
 * height on the centre column, sum of f_s over the column x = nx/2 (the
 * front height H_c of Sec. 4.2.1).  Returns LBM_ENONFINITE if a field is
 * NaN/Inf (the sums are still written).  Synchronises. */
int lbm_diag(lbm_ctx* c, lbm_diag_t* out);

/* Post-collision populations of lattice 0 = g, 1 = f, 2 = h (9*nx*ny
 * doubles, [i][k]) as stored after the last step.  Synchronises. */
int lbm_pops(lbm_ctx* c, int32_t lattice, double* host_out);

/* Checkpoint of the whole state (populations, history fields, step count)
 * as raw bytes; lbm_load accepts only a blob from an identical grid. */
size_t lbm_state_bytes(const lbm_ctx* c);
int lbm_save(lbm_ctx* c, void* host_buf, size_t bytes);
int lbm_load(lbm_ctx* c, const void* host_buf, size_t bytes);

int64_t lbm_step_count(const lbm_ctx* c);
int lbm_sync(lbm_ctx* c);
void lbm_destroy(lbm_ctx* c);
const char* lbm_strerror(int code);
const char* lbm_last_error(void);

/* Launch shape of the fused step.  tile_variant 0..4: 2-D tiles of 64x4
 * (default), 32x8, 64x8, 64x16, 128x4 nodes per workgroup, halo macros
 * recomputed per tile.  5: the unfused two-kernel step on 64x8 tiles (a
 * macro pass writes phi, rho and f_s^H of every node, then the collide pass
 * reads its halo from there), bitwise equal to the fused step and kept to
 * measure what fusion saves; lbm_autotune does not consider it.  6-10:
 * two steps per launch on 64x8, 32x8, 32x16 tiles (6-8: FP32 storage only,
 * else LBM_EINVAL), then on 32x16 tiles with two lanes per tile node (9: one
 * cell of each step per lane, four waves per SIMD) and on 32x8 tiles with
 * three (10: two workgroups per CU, six waves per SIMD; 9 and 10 in every
 * storage format, the first step's 16-bit populations kept in LDS exactly
 * as a single step stores them) -- each workgroup
 * runs the first step on its tile plus 3 columns and 2 rows
 * of halo from global memory, keeps those results in LDS and runs the
 * second step on the tile from there, so the state crosses HBM once per two
 * steps at ~1.3-1.5x the arithmetic; lbm_step issues pairs and a single
 * 64x8 step for an odd remainder; bitwise equal to single steps.
 * xcd_remap, the order in which the workgroups, dealt round-robin to the
 * 8 XCDs, take tiles: 0 row-major (the XCDs sweep the grid together); 1 one
 * contiguous row-major band of tiles per XCD; 2 one band of tile columns
 * per XCD, swept row by row (the XCDs still sweep the rows together, and
 * a tile's halo neighbours are mostly in its own XCD's L2).  Results are
 * bitwise identical for every choice; anything else is LBM_EINVAL. */
int lbm_set_launch(lbm_ctx* c, int32_t tile_variant, int32_t xcd_remap);

/* How the step kernel stores its outputs: 0 (default) streaming stores when
 * the state exceeds MI355X's 256 MiB Infinity Cache, so that it cannot stay
 * cached from one step's stores to the next step's loads, else cached
 * stores; 1 always cached; 2 always streaming.  Results are bitwise
 * identical; anything else is LBM_EINVAL. */
int lbm_set_store_mode(lbm_ctx* c, int32_t mode);

/* Time every launch shape for `reps` launches and keep the fastest per step
 * (written to the optional out-pointers): tile variants 0-4 and the
 * two-step variants the storage format admits (6-10 under FP32, 9-10
 * otherwise) at half their time per launch.  The
 * state is not advanced: each timed launch recomputes the next step(s) from
 * the same buffers.  Synchronises. */
int lbm_autotune(lbm_ctx* c, int32_t reps, int32_t* tile_variant, int32_t* xcd_remap);

/* ---- Batched sweep -----------------------------------------------------
 * Many droplets (each its own grid and parameters, as in the parametric
 * study of Sec. 4.2.2) run as one queue: up to `slots` are resident at a
 * time and every step of all of them is one launch.  A droplet is frozen once its liquid
 * volume sum clamp(phi) f_l has fallen to freeze_frac (default 0.01) of its
 * initial value; t_freeze is interpolated linearly between the samples taken
 * every sample_every steps.  At that sample its shape is measured from the
 * phi = 1/2 contour: height above the wall (topmost crossing over the
 * columns + 1/2), base half-width (crossings on row 0) and tip angle (angle
 * between least-squares lines x(y) through the left and right crossings of
 * the rows at heights in [0.75, 0.95] of the height).  The freed slot takes
 * the next queued droplet. */

enum {
  LBM_DROP_QUEUED = 0,   /* not started */
  LBM_DROP_RUNNING = 1,  /* resident */
  LBM_DROP_FROZEN = 2,   /* reached t_freeze and retired */
  LBM_DROP_LIMIT = 3,    /* retired at max_steps without freezing */
  LBM_DROP_NONFINITE = 4 /* retired: NaN/Inf in its fields */
};

typedef struct {
  int32_t status;       /* LBM_DROP_* */
  int32_t slot;         /* resident slot, -1 if none */
  int64_t steps;        /* steps run */
  double t_freeze;      /* steps (NaN until frozen) */
  double t_star;        /* Fourier number of t_freeze, k_l t/(rho_l cp_l R^2) (Eq. (42)); NaN without R */
  double liquid0;       /* liquid volume at the start */
  double liquid;        /* liquid volume at the last sample */
  double height;        /* shape at retirement (NaN before) */
  double base_radius;
  double tip_angle_deg; /* NaN if fewer than two rows fall in the fit band */
} lbm_drop_result;

typedef struct lbm_batch lbm_batch;

/* Workspace for n droplets with up to `slots` resident (p: n parameter sets,
 * all with the same storage; every grid within the single-grid limits). */
int lbm_batch_workspace_bytes(const lbm_params* p, int32_t n, int32_t slots, size_t* bytes);

/* Set up the queue.  phi0[i], T0[i]: host arrays of p[i].nx*p[i].ny doubles,
 * read when droplet i enters a slot (the first `slots` here, the rest during
 * lbm_batch_step): they must stay valid until then.  radius: n initial radii
 * for t_star, or NULL.  Workspace and stream as for lbm_init. */
int lbm_batch_init(const lbm_params* p, int32_t n, const double* const* phi0, const double* const* T0,
                   const double* radius, int32_t slots, void* d_workspace, size_t ws_bytes, void* hip_stream,
                   lbm_batch** out);

/* Sampling interval (even, >= 2; default 100), per-droplet step limit
 * (0 = none), freezing threshold (default 0.01), and how the steps of an
 * interval are launched: LBM_INTERVAL_LAUNCHES one launch per step (or per
 * two), LBM_INTERVAL_GRAPH the same launches captured once as a hipGraph
 * and replayed (default), or LBM_INTERVAL_PERSIST_FLAT / _PER_XCD all steps
 * of the interval in ONE persistent cooperative launch over the resident
 * droplets' tiles, with the flat or per-XCD grid barrier of
 * lbm_step_persistent between steps (64x8 tiles only: the tile variant is
 * set to 2, and lbm_batch_set_launch and lbm_batch_autotune keep it there;
 * wait_limit_us bounds one barrier wait as in lbm_step_persistent, 0: 2 s;
 * LBM_EDEVICE from lbm_batch_step if a wait runs out, and the resident
 * droplets' states are then invalid).  Results are bitwise the same in
 * every mode; anything else (or wait_limit_us < 0) is LBM_EINVAL. */
enum {
  LBM_INTERVAL_LAUNCHES = 0,
  LBM_INTERVAL_GRAPH = 1,
  LBM_INTERVAL_PERSIST_FLAT = 2,
  LBM_INTERVAL_PERSIST_PER_XCD = 3
};
int lbm_batch_configure(lbm_batch* b, int32_t sample_every, int64_t max_steps, double freeze_frac,
                        int32_t interval_launch, int32_t wait_limit_us);

/* Tile shape (tile_variant 0..4 of lbm_set_launch, or the two-step variants
 * 9 and 10 when the sampling interval is a multiple of 4; LBM_EINVAL
 * otherwise) and how tiles are dealt to the 8 XCDs: each droplet's tiles
 * kept on one XCD (xcd_group 1, default), laid out droplet after droplet
 * (0), or the tiles of all droplets cut into 8 contiguous equal lists, one
 * per XCD (2: balanced however few droplets remain); results are bitwise
 * identical either way.  lbm_batch_autotune times the same set (per step)
 * and keeps the fastest; after it, lbm_batch_step repeats the tuning each
 * time the resident set has halved (the last droplets of a sweep favour
 * other launches).  With a two-step variant set, lbm_batch_configure
 * refuses a sampling interval that is not a multiple of 4. */
int lbm_batch_set_launch(lbm_batch* b, int32_t tile_variant, int32_t xcd_group);
int lbm_batch_autotune(lbm_batch* b, int32_t reps, int32_t* tile_variant, int32_t* xcd_group);
/* Store mode of the batched step, as lbm_set_store_mode, except that mode 0
 * keeps cached stores: the sweep's many small grids run 7 % faster with
 * them even when the whole batch exceeds the Infinity Cache. */
int lbm_batch_set_store_mode(lbm_batch* b, int32_t mode);

/* Advance the resident droplets by nsteps (whole sampling intervals).  With
 * until_frozen, finished droplets retire and queued ones take their slots,
 * and the call returns early once the queue is empty.  Synchronises. */
int lbm_batch_step(lbm_batch* b, int64_t nsteps, int32_t until_frozen);

/* Per-droplet results, n entries. */
int lbm_batch_results(lbm_batch* b, lbm_drop_result* out);

/* Current fields of a resident droplet (as lbm_fields; LBM_ESTATE if it is
 * not resident).  Synchronises. */
int lbm_batch_fields(lbm_batch* b, int32_t drop, uint32_t field_mask, double* const* host_out);

const char* lbm_batch_last_error(void);
void lbm_batch_destroy(lbm_batch* b);

/* The batch's shape measurement on any phi field (host, ny rows of nx
 * doubles, row 0 half a spacing above the wall), rounded to FP32 as the
 * fields are: out[0..3] = height, base radius, tip angle in degrees, number
 * of rows in the tip fit.  Allocates and synchronises (a utility, not for
 * hot loops). */
int lbm_shape_of(const double* phi, int32_t nx, int32_t ny, double* out);

/* ---- Surrogate network ---------------------------------------------------
 * An ensemble of `ensemble` networks maps the 5 parameters of a sweep
 * droplet (normalised by the caller) to 3 outputs (t*, height/R, tip
 * angle, normalised): two hidden layers of 128 units with the exact GELU,
 * BF16 weights on the matrix cores with FP32 accumulation, FP32 master
 * weights trained with Adam on the loss
 *     L = sum_j w_j sum_s mask_sj (y_sj - t_sj)^2 / n.
 * Its spread over the ensemble tells when to fall back to the solver.
 * Parameters per member (lbm_mlp_param_count floats): W1 (128x5,
 * row-major), b1 (128), W2 (128x128), b2 (128), W3 (3x128), b3 (3).
 * Device arrays are row-major: x [n][5], targets and mask [n][3],
 * outputs [ensemble][n][3]. */
typedef struct lbm_mlp lbm_mlp;

size_t lbm_mlp_param_count(void);

/* He-uniform initial weights (seeded per member), zero biases; buffers
 * for batches of up to max_batch samples.  The library allocates. */
int lbm_mlp_create(int32_t ensemble, uint64_t seed, int32_t max_batch, void* hip_stream, lbm_mlp** out);

/* All members' FP32 parameters (ensemble x param_count floats, host);
 * setting them also resets the Adam state.  Synchronise. */
int lbm_mlp_set_params(lbm_mlp* m, const float* host, size_t count);
int lbm_mlp_get_params(lbm_mlp* m, float* host, size_t count);

/* Outputs of every member for n device samples (asynchronous). */
int lbm_mlp_forward(lbm_mlp* m, const float* d_x, int32_t n, float* d_y);

/* Loss (per member) and its gradient (ensemble x param_count floats) for
 * one batch, without updating.  w3: the 3 output weights (NULL = 1).
 * Synchronises. */
int lbm_mlp_gradient(lbm_mlp* m, const float* d_x, const float* d_t, const float* d_mask, int32_t n,
                     const float* w3, float* host_grad, double* host_loss);

/* `steps` Adam steps (beta 0.9/0.999, eps 1e-8, rate lr) on one batch of
 * n <= max_batch samples; host_loss receives each member's loss before the
 * last update.  Synchronises. */
int lbm_mlp_train(lbm_mlp* m, const float* d_x, const float* d_t, const float* d_mask, int32_t n, const float* w3,
                  float lr, int32_t steps, double* host_loss);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward pass of lbm_mlp_forward without a handle and without any
 * allocation.  d_params: device FP32 parameters of `ensemble` members in the
 * layout of lbm_mlp_set_params (ensemble x lbm_mlp_param_count floats);
 * d_x [n][5], d_y [ensemble][n][3] as for lbm_mlp_forward, all device
 * memory the caller owns.  The BF16 copies the kernels read are packed into
 * a static device buffer of the library (about 1.4 MB, held by every GPU it
 * runs on until the process ends), so ensemble is limited to
 * 1..LBM_MLP_NOALLOC_MAX_ENSEMBLE and n to 1..2^26 (else LBM_EINVAL).
 * Asynchronous on hip_stream (NULL = default stream); outputs equal
 * lbm_mlp_forward's with the same parameters bit for bit.  All calls on one
 * GPU share the buffer: calls that overlap in time on one GPU (other
 * streams, other threads) race and must be serialised by the caller. */
#define LBM_MLP_NOALLOC_MAX_ENSEMBLE 16
int lbm_mlp_forward_noalloc(const float* d_params, int32_t ensemble, const float* d_x, int32_t n, float* d_y,
                            void* hip_stream);

const char* lbm_mlp_last_error(void);
void lbm_mlp_destroy(lbm_mlp* m);

#ifdef __cplusplus
}
#endif
#endif
