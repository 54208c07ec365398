// Host side of the C ABI declared in include/lbm.h: parameter validation,
// workspace layout, launches on the caller's stream, read-back and
// checkpointing.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

namespace {

thread_local std::string g_last_error;

int dev_error(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return LBM_EDEVICE;
}

#define LBM_CK(expr)                                  \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return dev_error(e_, #expr); \
  } while (0)

constexpr double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
constexpr int kPops = 27;
constexpr int kAuxPlanes = 4 + 8;  // (phi u) x/y, node references, f_s^H, p, S, all double-buffered
constexpr int kStatePlanes = kPops + 6;  // checkpointed planes
constexpr int64_t kMagic = 0x4c424d4750555331LL;

}  // namespace

namespace lbmk {

bool all_finite(const lbm_params* p) {
  const double v[] = {p->W,       p->M,      p->sigma,  p->rho_l,  p->rho_g,  p->rho_s,
                      p->mu_l,    p->mu_g,   p->mu_s,   p->cp_l,   p->cp_g,   p->cp_s,
                      p->cp_ref,  p->k_l,    p->k_g,    p->k_s,    p->latent, p->T_melt,
                      p->T_bottom, p->theta_bottom_deg, p->theta_top_deg, p->gx, p->gy,
                      p->bq_beta, p->bq_rho0, p->bq_Tref};
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

// Every relaxation time must exceed 1/2: tau_g = M/cs^2 + 1/2 needs M > 0,
// tau_f = mu/(rho cs^2) + 1/2 needs mu, rho > 0 in every phase (mixtures
// stay positive), tau_h = k/(cp_ref cs^2) + 1/2 needs k, cp_ref > 0.
int validate_params(const lbm_params* p) {
  if (!p) return LBM_EINVAL;
  if (p->nx < 3 || p->ny < 3) return LBM_EINVAL;
  {
    // The kernels address a buffer by a 32-bit byte offset from its base:
    // the 27 population planes of one buffer and the 10 output-field planes
    // must each span less than 4 GiB.
    const long long nodes = (long long)p->nx * p->ny;
    const long long plane = (nodes + 63) / 64 * 64;
    const long long pb = p->storage == LBM_STORE_FP32 ? 4 : 2;
    if (27 * plane * pb >= (1LL << 32) || 10 * plane * 4 >= (1LL << 32)) return LBM_EINVAL;
  }
  if (!all_finite(p)) return LBM_EINVAL;
  if (!(p->W > 0) || !(p->M > 0) || p->sigma < 0) return LBM_EINVAL;
  if (!(p->rho_l > 0 && p->rho_g > 0 && p->rho_s > 0)) return LBM_EINVAL;
  if (!(p->mu_l > 0 && p->mu_g > 0 && p->mu_s > 0)) return LBM_EINVAL;
  if (!(p->cp_l > 0 && p->cp_g > 0 && p->cp_s > 0 && p->cp_ref > 0)) return LBM_EINVAL;
  if (!(p->k_l > 0 && p->k_g > 0 && p->k_s > 0)) return LBM_EINVAL;
  if (!(p->latent > 0)) return LBM_EINVAL;
  if (!(p->theta_bottom_deg > 0 && p->theta_bottom_deg < 180)) return LBM_EINVAL;
  if (!(p->theta_top_deg > 0 && p->theta_top_deg < 180)) return LBM_EINVAL;
  if (p->st_solid_mask != 0 && p->st_solid_mask != 1) return LBM_EINVAL;
  if (p->storage != LBM_STORE_FP32 && p->storage != LBM_STORE_FP16_SHIFT && p->storage != LBM_STORE_BF16_SHIFT)
    return LBM_EINVAL;
  return LBM_OK;
}

size_t pop_bytes(int storage) { return storage == LBM_STORE_FP32 ? 4 : 2; }

long long plane_floats(long long nodes) { return (nodes + 63) / 64 * 64; }  // 256-byte aligned planes

size_t state_bytes(long long plane, int storage) {
  return (size_t)2 * kPops * plane * pop_bytes(storage) + (size_t)(kAuxPlanes + NFIELD) * plane * sizeof(float);
}

void carve_state(State& S, char* base, long long pl, int storage) {
  const size_t popbuf = (size_t)kPops * pl * pop_bytes(storage);  // multiple of 256 bytes
  S.pops[0] = base;
  S.pops[1] = base + popbuf;
  float* aux = (float*)(base + 2 * popbuf);
  S.phiu[0] = aux;
  S.phiu[1] = aux + 2 * pl;
  S.fsH[0] = aux + 4 * pl;
  S.fsH[1] = aux + 5 * pl;
  S.p[0] = aux + 6 * pl;
  S.p[1] = aux + 7 * pl;
  S.S[0] = aux + 8 * pl;
  S.S[1] = aux + 9 * pl;
  S.ref[0] = aux + 10 * pl;
  S.ref[1] = aux + 11 * pl;
  S.fields = aux + kAuxPlanes * pl;
}

// FP16 scales (powers of two).  g and the shifted h stay O(1) and f is
// O(pressure + rho u); the scales lift their small values out of the FP16
// subnormals while leaving a wide margin below its maximum 65504: |g| < 256,
// |f| < 64, and h within 16x of the largest enthalpy excess the parameters
// and the initial temperature imply.
void fp16_scales(const lbm_params& p, double tspan, KParams& K) {
  const double cpmax = std::max(std::max(p.cp_l, p.cp_g), std::max(p.cp_s, p.cp_ref));
  const double hmax = cpmax * std::max(tspan, 1.0) + p.latent;
  double sh = 16.0;
  while (sh > 1.0 / 1024 && sh * hmax * 16.0 > 65504.0) sh *= 0.5;
  const double sc[3] = {256.0, 1024.0, sh};
  for (int j = 0; j < 3; ++j) {
    K.sc_st[j] = (float)sc[j];
    K.sc_ld[j] = (float)(1.0 / sc[j]);
  }
}


void fill_constants(const lbm_params& p, KParams& K, IParams& I, double& Href) {
  K.nx = p.nx;
  K.ny = p.ny;
  K.plane = (unsigned)plane_floats((long long)p.nx * p.ny);
  const double tau_g = 3.0 * p.M + 0.5;
  K.inv_tau_g = (float)(1.0 / tau_g);
  K.src_g = (float)(1.0 - 0.5 / tau_g);
  K.four_over_W = (float)(4.0 / p.W);
  K.beta4 = (float)(4.0 * 12.0 * p.sigma / p.W);
  K.kappa = (float)(1.5 * p.sigma * p.W);
  K.rho_s = (float)p.rho_s; K.rho_l = (float)p.rho_l; K.rho_g = (float)p.rho_g;
  K.mu_s = (float)p.mu_s; K.mu_l = (float)p.mu_l; K.mu_g = (float)p.mu_g;
  K.cp_s = (float)p.cp_s; K.cp_l = (float)p.cp_l; K.cp_g = (float)p.cp_g;
  K.k_s = (float)p.k_s; K.k_l = (float)p.k_l; K.k_g = (float)p.k_g;
  K.cp_ref = (float)p.cp_ref;
  K.T_melt = (float)p.T_melt;
  K.latent = (float)p.latent;
  K.inv_latent = (float)(1.0 / p.latent);
  K.three_over_cpref = (float)(3.0 / p.cp_ref);
  for (int i = 0; i < 9; ++i) K.hwall[i] = 0.0f;
  for (int i : {2, 5, 6}) K.hwall[i] = (float)(2.0 * kW[i] * p.cp_ref * (p.T_bottom - p.T_melt));
  K.mdot_coef = (float)(1.0 - p.rho_s / p.rho_l);
  K.tan_b = (float)std::tan((90.0 - p.theta_bottom_deg) * M_PI / 180.0);
  K.tan_t = (float)std::tan((90.0 - p.theta_top_deg) * M_PI / 180.0);
  K.gx = (float)p.gx;
  K.gy = (float)p.gy;
  K.bq_coef = (float)(p.bq_rho0 * p.bq_beta);
  K.bq_Tref = (float)p.bq_Tref;
  K.chi = (float)p.st_solid_mask;
  K.seed = 0;
  K.stream_stores = 0;
  K.storage = p.storage;
  for (int j = 0; j < 3; ++j) K.sc_st[j] = K.sc_ld[j] = 1.0f;
  I.cp_l = p.cp_l;
  I.cp_g = p.cp_g;
  I.cp_ref = p.cp_ref;
  I.T_melt = p.T_melt;
  I.latent = p.latent;
  Href = p.cp_ref * p.T_melt + p.latent;
}

// Temperatures stay within the initial and wall values (maximum
// principle); 16-bit storage keeps T - T_m of every node as an FP16
// reference, which needs that span well inside FP16's range.
int storage_setup(const lbm_params& p, const double* T0, long long N, KParams& K) {
  double tspan = std::fabs(p.T_bottom - p.T_melt);
  for (long long k = 0; k < N; ++k) tspan = std::max(tspan, std::fabs(T0[k] - p.T_melt));
  if (p.storage != LBM_STORE_FP32 && !(tspan < 3.0e4)) return LBM_EINVAL;
  if (p.storage == LBM_STORE_FP16_SHIFT) fp16_scales(p, tspan, K);
  return LBM_OK;
}


}  // namespace lbmk

struct lbm_ctx {
  lbm_params P;
  lbmk::KParams K;
  lbmk::IParams I;
  lbmk::State S;
  hipStream_t stream;
  int device;
  void* ws;
  bool own_ws;
  int cur;
  int64_t step;
  int tile_variant;
  int xcd;
  int store_mode;  // 0 by resident size, 1 cached, 2 streaming stores
  double Href;
  std::vector<float> stage;
};

namespace {

// Two steps per launch on one lane per node (variants 6-8) are built for FP32
// storage only; every other variant for every format.
bool variant_allowed(int v, int storage) {
  return !lbmk::is_two_step(v) || storage == LBM_STORE_FP32 || lbmk::is_two_step_any_storage(v);
}

size_t part_bytes() { return (size_t)(lbmk::RED_BLOCKS + 1) * lbmk::RED_NVAL * sizeof(double); }

size_t ws_size(const lbm_params* p) {
  return lbmk::state_bytes(lbmk::plane_floats((long long)p->nx * p->ny), p->storage) + part_bytes();
}


void carve(lbm_ctx* c) {
  const long long pl = c->K.plane;
  lbmk::carve_state(c->S, (char*)c->ws, pl, c->P.storage);
  c->S.part = (double*)(c->S.fields + lbmk::NFIELD * pl);
}

int run_fields(lbm_ctx* c) {
  if (lbmk::launch_step(c->K, c->S, c->cur, true, c->tile_variant, c->xcd, c->stream))
    return dev_error(hipGetLastError(), "fields kernel launch");
  return LBM_OK;
}

// Host <-> device copy of the checkpointed planes of the current buffer:
// the populations in their storage format, then the FP32 history planes.
int copy_state(lbm_ctx* c, char* host, bool save) {
  const size_t N = (size_t)c->P.nx * c->P.ny;
  const size_t pb = lbmk::pop_bytes(c->P.storage);
  void* dev[kStatePlanes];
  for (int i = 0; i < kPops; ++i) dev[i] = (char*)c->S.pops[c->cur] + (size_t)i * c->K.plane * pb;
  dev[kPops + 0] = c->S.phiu[c->cur];
  dev[kPops + 1] = c->S.phiu[c->cur] + c->K.plane;
  dev[kPops + 2] = c->S.fsH[c->cur];
  dev[kPops + 3] = c->S.p[c->cur];
  dev[kPops + 4] = c->S.S[c->cur];
  dev[kPops + 5] = c->S.ref[c->cur];
  for (int i = 0; i < kStatePlanes; ++i) {
    const size_t nb = N * (i < kPops ? pb : sizeof(float));
    if (save)
      LBM_CK(hipMemcpyAsync(host, dev[i], nb, hipMemcpyDeviceToHost, c->stream));
    else
      LBM_CK(hipMemcpyAsync(dev[i], host, nb, hipMemcpyHostToDevice, c->stream));
    host += nb;
  }
  LBM_CK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_workspace_bytes(const lbm_params* p, size_t* bytes) {
  if (!bytes) return LBM_EINVAL;
  int rc = lbmk::validate_params(p);
  if (rc) return rc;
  *bytes = ws_size(p);
  return LBM_OK;
}

int lbm_init(const lbm_params* p, const double* phi0, const double* T0, void* d_workspace,
             size_t ws_bytes, void* hip_stream, lbm_ctx** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  int rc = lbmk::validate_params(p);
  if (rc) {
    g_last_error = "invalid parameters";
    return rc;
  }
  if (!phi0 || !T0) return LBM_EINVAL;
  const size_t need = ws_size(p);
  if (d_workspace && (ws_bytes < need || ((uintptr_t)d_workspace & 255))) {
    g_last_error = "workspace too small or not 256-byte aligned";
    return LBM_EINVAL;
  }
  const long long N = (long long)p->nx * p->ny;
  for (long long k = 0; k < N; ++k)
    if (!std::isfinite(phi0[k]) || !std::isfinite(T0[k])) {
      g_last_error = "non-finite initial field";
      return LBM_EINVAL;
    }
  lbmk::KParams K;
  lbmk::IParams I;
  double Href;
  lbmk::fill_constants(*p, K, I, Href);
  if (lbmk::storage_setup(*p, T0, N, K)) {
    g_last_error = "temperature span too wide for the FP16 node references of 16-bit storage";
    return LBM_EINVAL;
  }
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ENOMEM;
  c->P = *p;
  c->stream = (hipStream_t)hip_stream;
  c->cur = 0;
  c->step = 0;
  c->tile_variant = 0;
  c->xcd = 1;
  c->store_mode = 0;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return dev_error(e, "hipGetDevice");
  }
  c->K = K;
  c->K.stream_stores = need > lbmk::kInfinityCacheBytes;
  c->I = I;
  c->Href = Href;
  if (d_workspace) {
    c->ws = d_workspace;
    c->own_ws = false;
  } else {
    e = hipMalloc(&c->ws, need);
    if (e != hipSuccess) {
      delete c;
      g_last_error = "hipMalloc of the workspace failed";
      return LBM_ENOMEM;
    }
    c->own_ws = true;
  }
  carve(c);
  // stage phi0 and T0 (FP64) in the output-field planes (10 planes >= 4)
  double* d_phi0 = (double*)c->S.fields;
  double* d_T0 = d_phi0 + N;
  e = hipMemcpyAsync(d_phi0, phi0, N * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_T0, T0, N * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && lbmk::launch_init(c->K, c->I, c->S, 0, d_phi0, d_T0, c->stream))
    e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    int r = dev_error(e, "lbm_init");
    lbm_destroy(c);
    return r;
  }
  *out = c;
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return LBM_EINVAL;
  for (int32_t s = 0; s < nsteps;) {
    if (lbmk::is_two_step(c->tile_variant) && nsteps - s >= 2) {
      c->K.seed = (unsigned)c->step;  // steps n and n + 1 seed 16-bit stochastic rounding
      if (lbmk::launch_step2(c->K, c->S, c->cur, c->tile_variant, c->xcd, c->stream))
        return dev_error(hipGetLastError(), "two-step kernel launch");
      c->cur ^= 1;
      c->step += 2;
      s += 2;
      continue;
    }
    c->K.seed = (unsigned)c->step;  // the step number seeds 16-bit stochastic rounding
    if (lbmk::launch_step(c->K, c->S, c->cur, false, c->tile_variant, c->xcd, c->stream))
      return dev_error(hipGetLastError(), "step kernel launch");
    c->cur ^= 1;
    c->step++;
    ++s;
  }
  return LBM_OK;
}

int lbm_step_persistent(lbm_ctx* c, int32_t nsteps, int32_t barrier, int32_t wait_limit_us, int32_t* workgroups) {
  if (!c || nsteps < 0 || nsteps > LBM_PERSIST_MAX_STEPS) return LBM_EINVAL;
  if (barrier != LBM_BARRIER_FLAT && barrier != LBM_BARRIER_PER_XCD) return LBM_EINVAL;
  if (wait_limit_us < 0) return LBM_EINVAL;
  if (nsteps == 0) return LBM_OK;
  int rate_khz = 0;
  LBM_CK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device));
  if (rate_khz <= 0) {
    g_last_error = "device reports no wall-clock rate";
    return LBM_EDEVICE;
  }
  // by default a barrier wait of 2 s is a failure: a step of the largest grid takes ~1 ms
  const unsigned long long us = wait_limit_us ? (unsigned long long)wait_limit_us : 2000000ull;
  const unsigned long long limit = us * (unsigned long long)rate_khz / 1000ull;
  // the barrier words sit in the reduction scratch, which no step reads
  static_assert(lbmk::NPERSIST_WORDS <= (lbmk::RED_BLOCKS + 1) * lbmk::RED_NVAL, "barrier words");
  unsigned long long* bar = (unsigned long long*)c->S.part;
  c->K.seed = (unsigned)c->step;
  int grid = 0;
  hipError_t e = lbmk::launch_persist(c->K, c->S, c->cur, nsteps, c->xcd, barrier, bar, limit, &grid, c->stream);
  if (e != hipSuccess) return dev_error(e, "persistent step launch");
  unsigned long long w[lbmk::NPERSIST_WORDS];
  LBM_CK(hipMemcpyAsync(w, bar, sizeof(w), hipMemcpyDeviceToHost, c->stream));
  LBM_CK(hipStreamSynchronize(c->stream));
  if (w[1]) {
    g_last_error = "grid barrier of the persistent step timed out; the state is invalid";
    return LBM_EDEVICE;
  }
  // every workgroup arrives once per barrier: the counts must add up
  const unsigned long long g = (unsigned long long)grid, nb = (unsigned long long)(nsteps - 1);
  unsigned long long arrivals = 0, placed = 0;
  for (int x = 0; x < 8; ++x) {
    arrivals += w[3 + x];
    placed += w[11 + x];
  }
  const bool census = barrier == LBM_BARRIER_PER_XCD && nsteps > 1;
  const bool ok = census ? (w[0] == g && arrivals == nb * g && placed == g) : (w[0] == nb * g && arrivals == 0);
  if (!ok) {
    g_last_error = "grid barrier arrivals of the persistent step do not add up; the state is invalid";
    return LBM_EDEVICE;
  }
  if ((nsteps & 1) != 0) c->cur ^= 1;
  c->step += nsteps;
  if (workgroups) *workgroups = grid;
  return LBM_OK;
}

int lbm_fields_device(lbm_ctx* c, uint32_t mask, float* const* d_out) {
  if (!c || !d_out || (mask >> lbmk::NFIELD)) return LBM_EINVAL;
  int rc = run_fields(c);
  if (rc) return rc;
  const long long N = (long long)c->P.nx * c->P.ny;
  int j = 0;
  for (int b = 0; b < lbmk::NFIELD; ++b) {
    if (!(mask & (1u << b))) continue;
    if (!d_out[j]) return LBM_EINVAL;
    LBM_CK(hipMemcpyAsync(d_out[j], c->S.fields + b * c->K.plane, N * sizeof(float),
                          hipMemcpyDeviceToDevice, c->stream));
    ++j;
  }
  return LBM_OK;
}

int lbm_fields(lbm_ctx* c, uint32_t mask, double* const* host_out) {
  if (!c || !host_out || (mask >> lbmk::NFIELD)) return LBM_EINVAL;
  int rc = run_fields(c);
  if (rc) return rc;
  const long long N = (long long)c->P.nx * c->P.ny;
  c->stage.resize(N);
  int j = 0;
  for (int b = 0; b < lbmk::NFIELD; ++b) {
    if (!(mask & (1u << b))) continue;
    if (!host_out[j]) return LBM_EINVAL;
    LBM_CK(hipMemcpyAsync(c->stage.data(), c->S.fields + b * c->K.plane, N * sizeof(float),
                          hipMemcpyDeviceToHost, c->stream));
    LBM_CK(hipStreamSynchronize(c->stream));
    const double add = (b == 8) ? c->Href : 0.0;  // H is kept relative to H_ref on the device
    for (long long k = 0; k < N; ++k) host_out[j][k] = (double)c->stage[k] + add;
    ++j;
  }
  LBM_CK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int lbm_diag(lbm_ctx* c, lbm_diag_t* out) {
  if (!c || !out) return LBM_EINVAL;
  int rc = run_fields(c);
  if (rc) return rc;
  if (lbmk::launch_reduce(c->K, c->S, c->Href, c->stream))
    return dev_error(hipGetLastError(), "reduce launch");
  double v[lbmk::RED_NVAL];
  LBM_CK(hipMemcpyAsync(v, c->S.part + lbmk::RED_BLOCKS * lbmk::RED_NVAL, sizeof(v),
                        hipMemcpyDeviceToHost, c->stream));
  LBM_CK(hipStreamSynchronize(c->stream));
  out->step = c->step;
  out->sum_phi = v[0];
  out->sum_phic = v[1];
  out->sum_solid = v[2];
  out->sum_liquid = v[3];
  out->sum_H = v[4];
  out->max_u = v[5];
  out->nonfinite = v[6] > 0 ? 1 : 0;
  out->h_c = v[7];
  return out->nonfinite ? LBM_ENONFINITE : LBM_OK;
}

int lbm_pops(lbm_ctx* c, int32_t lattice, double* host_out) {
  if (!c || !host_out || lattice < 0 || lattice > 2) return LBM_EINVAL;
  const long long N = (long long)c->P.nx * c->P.ny;
  const bool noderef = c->P.storage != LBM_STORE_FP32;
  c->stage.resize(N);
  const double cpr = c->P.cp_ref, Tm = c->P.T_melt;
  // Undo the storage shifts: g is kept relative to w_i phi_ref and the rest h
  // population relative to L f_s^H (under 16-bit storage the expand kernel
  // has already added the node references back).
  std::vector<float> ref1;
  auto fetch = [&](std::vector<float>& v, const float* d) -> int {
    v.resize(N);
    LBM_CK(hipMemcpyAsync(v.data(), d, N * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    return LBM_OK;
  };
  int rc = LBM_OK;
  if (lattice == 0 && !noderef) rc = fetch(ref1, (const float*)c->S.ref[c->cur]);
  if (lattice == 2) rc = fetch(ref1, c->S.fsH[c->cur]);
  if (rc) return rc;
  if (lbmk::launch_expand(c->K, c->S, c->cur, lattice, c->stream))
    return dev_error(hipGetLastError(), "expand launch");
  for (int i = 0; i < 9; ++i) {
    LBM_CK(hipMemcpyAsync(c->stage.data(), c->S.fields + i * c->K.plane, N * sizeof(float),
                          hipMemcpyDeviceToHost, c->stream));
    LBM_CK(hipStreamSynchronize(c->stream));
    double add = 0.0;
    if (lattice == 2) add = i == 0 ? c->Href - cpr * Tm + kW[0] * cpr * Tm : kW[i] * cpr * Tm;
    for (long long k = 0; k < N; ++k) {
      double v = (double)c->stage[k] + add;
      if (lattice == 0 && !noderef) v += kW[i] * (double)ref1[k];
      if (lattice == 2 && i == 0) v -= c->P.latent * (double)ref1[k];
      host_out[i * N + k] = v;
    }
  }
  return LBM_OK;
}

size_t lbm_state_bytes(const lbm_ctx* c) {
  if (!c) return 0;
  const size_t N = (size_t)c->P.nx * c->P.ny;
  return 4 * sizeof(int64_t) + (size_t)kPops * N * lbmk::pop_bytes(c->P.storage) +
         (size_t)(kStatePlanes - kPops) * N * sizeof(float);
}

int lbm_save(lbm_ctx* c, void* buf, size_t bytes) {
  if (!c || !buf || bytes < lbm_state_bytes(c)) return LBM_EINVAL;
  int64_t hdr[4] = {kMagic + c->P.storage, c->P.nx, c->P.ny, c->step};
  char* o = (char*)buf;
  std::memcpy(o, hdr, sizeof(hdr));
  return copy_state(c, o + sizeof(hdr), true);
}

int lbm_load(lbm_ctx* c, const void* buf, size_t bytes) {
  if (!c || !buf || bytes < lbm_state_bytes(c)) return LBM_EINVAL;
  int64_t hdr[4];
  std::memcpy(hdr, buf, sizeof(hdr));
  if (hdr[0] != kMagic + c->P.storage || hdr[1] != c->P.nx || hdr[2] != c->P.ny) return LBM_ESTATE;
  int rc = copy_state(c, (char*)buf + sizeof(hdr), false);
  if (rc) return rc;
  c->step = hdr[3];
  return LBM_OK;
}

int64_t lbm_step_count(const lbm_ctx* c) { return c ? c->step : -1; }

int lbm_sync(lbm_ctx* c) {
  if (!c) return LBM_EINVAL;
  LBM_CK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int lbm_set_launch(lbm_ctx* c, int32_t tile_variant, int32_t xcd_remap) {
  if (!c || tile_variant < 0 || tile_variant >= lbmk::NTILE_VARIANTS || xcd_remap < 0 ||
      xcd_remap >= lbmk::NXCD_MODES)
    return LBM_EINVAL;
  if (!variant_allowed(tile_variant, c->P.storage)) return LBM_EINVAL;
  c->tile_variant = tile_variant;
  c->xcd = xcd_remap;
  return LBM_OK;
}

int lbm_set_store_mode(lbm_ctx* c, int32_t mode) {
  if (!c || mode < 0 || mode > 2) return LBM_EINVAL;
  c->store_mode = mode;
  c->K.stream_stores = mode == 2 || (mode == 0 && ws_size(&c->P) > lbmk::kInfinityCacheBytes);
  return LBM_OK;
}

int lbm_autotune(lbm_ctx* c, int32_t reps, int32_t* tile_variant, int32_t* xcd_remap) {
  if (!c || reps < 1) return LBM_EINVAL;
  // The step kernel reads buffer cur and writes buffer cur^1 only, so
  // replaying it without flipping leaves the state where it was.
  struct Events {  // destroyed on every return path
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  LBM_CK(hipEventCreate(&ev.a));
  LBM_CK(hipEventCreate(&ev.b));
  hipEvent_t e0 = ev.a, e1 = ev.b;
  float best = 1e30f;
  int bv = c->tile_variant, bx = c->xcd;
  c->K.seed = (unsigned)c->step;
  for (int v = 0; v < lbmk::NTILE_VARIANTS; ++v) {
    const bool two = lbmk::is_two_step(v);
    if (v >= lbmk::NTUNED_VARIANTS && !two) continue;  // the unfused reference step
    if (!variant_allowed(v, c->P.storage)) continue;
    for (int x = 0; x < lbmk::NXCD_MODES; ++x) {
      auto launch = [&]() {
        return two ? lbmk::launch_step2(c->K, c->S, c->cur, v, x, c->stream)
                   : lbmk::launch_step(c->K, c->S, c->cur, false, v, x, c->stream);
      };
      if (launch()) return dev_error(hipGetLastError(), "autotune launch");  // warm-up
      LBM_CK(hipEventRecord(e0, c->stream));
      for (int r = 0; r < reps; ++r)
        if (launch()) return dev_error(hipGetLastError(), "autotune launch");
      LBM_CK(hipEventRecord(e1, c->stream));
      LBM_CK(hipEventSynchronize(e1));
      float ms = 0.0f;
      LBM_CK(hipEventElapsedTime(&ms, e0, e1));
      if (two) ms *= 0.5f;  // two steps per launch: compare time per step
      if (ms < best) {
        best = ms;
        bv = v;
        bx = x;
      }
    }
  }
  c->tile_variant = bv;
  c->xcd = bx;
  if (tile_variant) *tile_variant = bv;
  if (xcd_remap) *xcd_remap = bx;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  if (c->own_ws && c->ws) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->ws);
  }
  delete c;
}

const char* lbm_strerror(int code) {
  switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of memory";
    case LBM_EDEVICE: return "HIP device error";
    case LBM_ENONFINITE: return "non-finite field";
    case LBM_ESTATE: return "state mismatch";
    default: return "unknown error";
  }
}

const char* lbm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
