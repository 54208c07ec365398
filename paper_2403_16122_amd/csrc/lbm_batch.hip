// Batched sweep: many droplets of different grid sizes advanced together.
//
// Up to `slots` droplets are resident at a time, each in a slot of the
// workspace holding the same state a single context keeps (plane stride
// sized for the largest grid of the queue).  One launch of the fused step
// updates every tile of every resident droplet: workgroups read their
// (slot, tile) from a tile map and the slot's constants and buffer offsets
// from device tables.  K steps (the sampling interval), a fields pass and a
// per-droplet reduction of the liquid volume run as one captured hipGraph.
// After each replay the host checks every resident droplet: a droplet whose
// liquid volume sum clamp(phi) f_l has fallen to `freeze_frac` of its initial
// value is frozen (t_freeze interpolated linearly between the last two
// samples), its shape is measured on the device and its slot is refilled
// from the queue; the tile map and the graph are then rebuilt.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

namespace {

thread_local std::string g_batch_error;

int bdev_error(hipError_t e, const char* what) {
  g_batch_error = std::string(what) + ": " + hipGetErrorString(e);
  return LBM_EDEVICE;
}

#define LBMB_CK(expr)                                  \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return bdev_error(e_, #expr); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kPersistVariant = 2;  // 64x8: the tiles of the persistent interval launch
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  long long plane;     // floats per plane in every slot
  size_t slot_bytes;   // one slot's state
  size_t tmap_cap;     // tile-map entries
  size_t off_ptab, off_otab, off_tmap, off_slots, off_steps, off_liq, off_shape, off_bar, off_slots_ws, total;
};

int max_tiles(int nx, int ny) {
  int m = 0;
  for (int v = 0; v < lbmk::NBATCH_VARIANTS; ++v) {
    int tx, ty;
    lbmk::tile_shape(v, &tx, &ty);
    m = std::max(m, ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty));
  }
  return m;
}

Layout layout(const lbm_params* p, int n, int slots) {
  Layout L{};
  long long maxn = 0;
  int mt = 0;
  for (int i = 0; i < n; ++i) {
    maxn = std::max(maxn, (long long)p[i].nx * p[i].ny);
    mt = std::max(mt, max_tiles(p[i].nx, p[i].ny));
  }
  L.plane = lbmk::plane_floats(maxn);
  L.slot_bytes = align_up(lbmk::state_bytes(L.plane, p[0].storage));
  // every resident tile once, plus padding of the 8 per-XCD lists to equal length
  L.tmap_cap = (size_t)slots * mt + 8 * (size_t)mt + 64;
  size_t o = 0;
  L.off_ptab = o;
  o = align_up(o + sizeof(lbmk::KParams) * slots);
  L.off_otab = o;
  o = align_up(o + sizeof(lbmk::StepOff) * 2 * slots);
  L.off_tmap = o;
  o = align_up(o + sizeof(unsigned) * L.tmap_cap);
  L.off_slots = o;
  o = align_up(o + sizeof(int) * slots);
  L.off_steps = o;
  o = align_up(o + sizeof(unsigned) * slots);
  L.off_liq = o;
  o = align_up(o + sizeof(double) * 2 * slots);
  L.off_shape = o;
  o = align_up(o + sizeof(double) * 4 * slots);
  L.off_bar = o;  // grid-barrier words of the persistent interval launch
  o = align_up(o + sizeof(unsigned long long) * lbmk::NPERSIST_WORDS);
  L.off_slots_ws = o;
  L.total = o + L.slot_bytes * slots;
  return L;
}

struct Drop {
  lbm_params P;
  const double* phi0;
  const double* T0;
  double radius;
  lbm_drop_result r;
  double prev_liq;     // liquid volume at the previous sample
  int64_t prev_step;
};

}  // namespace

struct lbm_batch {
  int n, slots, storage;
  Layout L;
  char* ws;
  bool own_ws;
  hipStream_t stream;      // the caller's stream: every launch and replay
  hipStream_t cap_stream;  // private stream used only to capture the graph
  int device;
  std::vector<Drop> drops;
  std::vector<int> slot_drop;  // drop index per slot or -1
  int next;                    // next queued drop
  std::vector<lbmk::KParams> ptab;
  std::vector<lbmk::StepOff> otab;
  std::vector<int> active;     // resident slots (device list order)
  int nblocks;
  int sample_every;
  int64_t max_steps;
  double freeze_frac;
  int tile_variant, xcd_group;
  int tune_reps;     // repetitions of the last lbm_batch_autotune (0: never tuned)
  int tuned_active;  // resident droplets at that tuning
  int store_mode;  // 0 and 1 cached, 2 streaming stores
  bool nt;         // the step kernels stream their stores
  bool use_graph;
  int persist;                   // -1: launches per step; 0 / 1: one persistent launch per interval
                                 // with the flat / per-XCD grid barrier
  unsigned long long bar_limit;  // wall-clock ticks a barrier wait may take (default 2 s)
  unsigned long long clock_khz;  // the device's wall-clock rate
  int persist_grid;              // workgroups of the last persistent launch
  hipGraphExec_t exec;
  bool graph_valid;
  double* h_liq;      // pinned: 2 doubles per slot
  unsigned* h_steps;  // pinned: step count of each slot's droplet at the start of an interval
  unsigned long long* h_bar;  // pinned: the barrier words after the last persistent launch
  std::vector<double> shape;
  char* d(size_t off) const { return ws + off; }
  lbmk::KParams* d_ptab() const { return (lbmk::KParams*)d(L.off_ptab); }
  lbmk::StepOff* d_otab() const { return (lbmk::StepOff*)d(L.off_otab); }
  unsigned* d_tmap() const { return (unsigned*)d(L.off_tmap); }
  int* d_slots() const { return (int*)d(L.off_slots); }
  unsigned* d_steps() const { return (unsigned*)d(L.off_steps); }
  double* d_liq() const { return (double*)d(L.off_liq); }
  double* d_shape() const { return (double*)d(L.off_shape); }
  unsigned long long* d_bar() const { return (unsigned long long*)d(L.off_bar); }
  char* slot_base(int s) const { return d(L.off_slots_ws) + (size_t)s * L.slot_bytes; }
};

namespace {

lbmk::StepOff offsets(const lbm_batch* b, const lbmk::State& S, int par) {
  const lbmk::StepIO io = lbmk::make_io(S, par);
  auto off = [&](const void* ptr) { return (unsigned long long)((const char*)ptr - b->ws); };
  return lbmk::StepOff{off(io.A),      off(io.B),     off(io.phiu_in), off(io.phiu_out), off(io.ref_in),
                       off(io.ref_out), off(io.fsH_in), off(io.fsH_out), off(io.p_in),     off(io.p_out),
                       off(io.S_in),    off(io.S_out),  off(io.fields)};
}

// Tile map of the resident droplets.  xcd_group 0: droplet after droplet.
// xcd_group 1: droplets are dealt to the 8 XCDs by node count (largest
// first to the least loaded), and workgroup b, which the hardware places on
// XCD b mod 8, takes the (b / 8)-th tile of XCD (b mod 8)'s list, so all
// tiles of a droplet share one L2.  xcd_group 2: the tiles of all resident
// droplets, droplet after droplet and row by row, cut into 8 contiguous
// lists of equal length, one per XCD: every XCD gets the same work however
// few droplets are left (with group 1 a lone droplet runs on one XCD), and
// a tile's halo neighbours are still mostly in its own XCD's list.
std::vector<unsigned> build_tmap(const lbm_batch* b) {
  int tx, ty;
  lbmk::tile_shape(b->tile_variant, &tx, &ty);
  std::vector<unsigned> out;
  auto tiles_of = [&](int s) {
    const lbm_params& P = b->drops[b->slot_drop[s]].P;
    return ((P.nx + tx - 1) / tx) * ((P.ny + ty - 1) / ty);
  };
  if (b->xcd_group == 0 || b->xcd_group == 2) {
    for (int s : b->active)
      for (int t = 0, nt = tiles_of(s); t < nt; ++t) out.push_back(((unsigned)s << 16) | (unsigned)t);
    if (b->xcd_group == 0) return out;
    const size_t len = (out.size() + 7) / 8;  // list length per XCD
    std::vector<unsigned> dealt(8 * len, ~0u);
    for (size_t i = 0; i < out.size(); ++i) dealt[8 * (i % len) + i / len] = out[i];
    return dealt;
  }
  std::vector<int> order(b->active);
  std::sort(order.begin(), order.end(), [&](int a, int c) { return tiles_of(a) > tiles_of(c); });
  std::vector<std::vector<unsigned>> lists(8);
  for (int s : order) {
    size_t j = 0;
    for (size_t q = 1; q < 8; ++q)
      if (lists[q].size() < lists[j].size()) j = q;
    for (int t = 0, nt = tiles_of(s); t < nt; ++t) lists[j].push_back(((unsigned)s << 16) | (unsigned)t);
  }
  size_t len = 0;
  for (auto& l : lists) len = std::max(len, l.size());
  out.assign(8 * len, ~0u);
  for (size_t j = 0; j < 8; ++j)
    for (size_t i = 0; i < lists[j].size(); ++i) out[8 * i + j] = lists[j][i];
  return out;
}

void drop_graph(lbm_batch* b) {
  if (b->graph_valid) (void)hipGraphExecDestroy(b->exec);
  b->graph_valid = false;
}

// Upload the tile map and the resident-slot list (stream-ordered).
int upload_map(lbm_batch* b) {
  const std::vector<unsigned> tm = build_tmap(b);
  if (tm.size() > b->L.tmap_cap) {
    g_batch_error = "tile map exceeds its capacity";
    return LBM_EINVAL;
  }
  b->nblocks = (int)tm.size();
  if (!tm.empty())
    LBMB_CK(hipMemcpyAsync(b->d_tmap(), tm.data(), tm.size() * sizeof(unsigned), hipMemcpyHostToDevice, b->stream));
  if (!b->active.empty())
    LBMB_CK(hipMemcpyAsync(b->d_slots(), b->active.data(), b->active.size() * sizeof(int), hipMemcpyHostToDevice,
                           b->stream));
  // the host vectors die here: the copies must have read them
  LBMB_CK(hipStreamSynchronize(b->stream));
  drop_graph(b);
  return LBM_OK;
}

// K steps, the fields pass, the liquid reduction and its copy to the host,
// on stream `st` (the capture stream or the caller's).
int enqueue_chunk(lbm_batch* b, hipStream_t st) {
  // step numbers at the start of the interval (read from pinned memory when the copy runs)
  LBMB_CK(hipMemcpyAsync(b->d_steps(), b->h_steps, sizeof(unsigned) * b->slots, hipMemcpyHostToDevice, st));
  if (b->persist >= 0) {
    // the whole interval in one cooperative launch; its barrier words are
    // read back with the liquid volumes and checked after the interval
    hipError_t e = lbmk::launch_batch_persist(b->storage, b->nt, b->persist, b->ws, b->d_ptab(), b->d_otab(),
                                              b->d_tmap(), b->d_steps(), b->nblocks, b->sample_every, b->d_bar(),
                                              b->bar_limit, &b->persist_grid, st);
    if (e != hipSuccess) return bdev_error(e, "persistent batch launch");
    LBMB_CK(hipMemcpyAsync(b->h_bar, b->d_bar(), sizeof(unsigned long long) * lbmk::NPERSIST_WORDS,
                           hipMemcpyDeviceToHost, st));
  } else {
    const int per = lbmk::is_two_step_any_storage(b->tile_variant) ? 2 : 1;  // steps per launch
    for (int s = 0; s < b->sample_every; s += per)
      if (lbmk::launch_batch(b->storage, b->tile_variant, false, b->nt, b->ws, b->d_ptab(), b->d_otab(),
                             b->d_tmap(), b->d_steps(), b->nblocks, s, st))
        return bdev_error(hipGetLastError(), "batch step launch");
  }
  if (lbmk::launch_batch(b->storage, b->tile_variant, true, false, b->ws, b->d_ptab(), b->d_otab(), b->d_tmap(),
                         b->d_steps(), b->nblocks, 0, st))
    return bdev_error(hipGetLastError(), "batch fields launch");
  const int na = (int)b->active.size();
  if (lbmk::launch_batch_liquid(b->ws, b->d_ptab(), b->d_otab(), b->d_slots(), na, b->d_liq(), st))
    return bdev_error(hipGetLastError(), "batch liquid launch");
  LBMB_CK(hipMemcpyAsync(b->h_liq, b->d_liq(), sizeof(double) * 2 * b->slots, hipMemcpyDeviceToHost, st));
  return LBM_OK;
}

// After a persistent interval: no barrier wait timed out, and every
// workgroup arrived once per barrier.
int check_barrier(lbm_batch* b) {
  const unsigned long long* w = b->h_bar;
  if (w[1]) {
    g_batch_error = "grid barrier of the persistent interval timed out; the states are invalid";
    return LBM_EDEVICE;
  }
  const unsigned long long g = (unsigned long long)b->persist_grid, nb = (unsigned long long)(b->sample_every - 1);
  unsigned long long arrivals = 0, placed = 0;
  for (int x = 0; x < 8; ++x) {
    arrivals += w[3 + x];
    placed += w[11 + x];
  }
  const bool ok = b->persist ? (w[0] == g && arrivals == nb * g && placed == g) : (w[0] == nb * g && arrivals == 0);
  if (!ok) {
    g_batch_error = "grid barrier arrivals of the persistent interval do not add up; the states are invalid";
    return LBM_EDEVICE;
  }
  return LBM_OK;
}

int run_chunk(lbm_batch* b) {
  for (int s : b->active) b->h_steps[s] = (unsigned)b->drops[b->slot_drop[s]].r.steps;
  if (!b->use_graph || b->persist >= 0) return enqueue_chunk(b, b->stream);
  if (!b->graph_valid) {
    hipGraph_t g;
    LBMB_CK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_chunk(b, b->cap_stream);
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc) {
      if (e == hipSuccess) (void)hipGraphDestroy(g);
      return rc;
    }
    LBMB_CK(e);
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    LBMB_CK(e);
    b->graph_valid = true;
  }
  LBMB_CK(hipGraphLaunch(b->exec, b->stream));
  return LBM_OK;
}

// Liquid volumes of the listed slots at their current state (fields pass +
// reduction over a temporary map of just those slots), into h_liq.
int sample_now(lbm_batch* b, const std::vector<int>& slots) {
  if (slots.empty()) return LBM_OK;
  std::vector<int> keep_active = b->active;
  b->active = slots;
  int rc = upload_map(b);
  if (!rc && lbmk::launch_batch(b->storage, b->tile_variant, true, false, b->ws, b->d_ptab(), b->d_otab(), b->d_tmap(),
                                b->d_steps(), b->nblocks, 0, b->stream))
    rc = bdev_error(hipGetLastError(), "batch fields launch");
  if (!rc && lbmk::launch_batch_liquid(b->ws, b->d_ptab(), b->d_otab(), b->d_slots(), (int)slots.size(), b->d_liq(),
                                       b->stream))
    rc = bdev_error(hipGetLastError(), "batch liquid launch");
  if (!rc) {
    hipError_t e = hipMemcpyAsync(b->h_liq, b->d_liq(), sizeof(double) * 2 * b->slots, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) rc = bdev_error(e, "liquid read-back");
  }
  b->active = keep_active;
  int rc2 = upload_map(b);
  return rc ? rc : rc2;
}

// Shapes of the listed slots from their field planes (the last fields pass).
int measure_shapes(lbm_batch* b, const std::vector<int>& slots) {
  if (slots.empty()) return LBM_OK;
  LBMB_CK(hipMemcpyAsync(b->d_slots(), slots.data(), slots.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
  if (lbmk::launch_batch_shape(b->ws, b->d_ptab(), b->d_otab(), b->d_slots(), (int)slots.size(), b->d_shape(),
                               b->stream))
    return bdev_error(hipGetLastError(), "batch shape launch");
  LBMB_CK(hipMemcpyAsync(b->shape.data(), b->d_shape(), sizeof(double) * 4 * b->slots, hipMemcpyDeviceToHost,
                         b->stream));
  LBMB_CK(hipStreamSynchronize(b->stream));
  for (int s : slots) {
    lbm_drop_result& r = b->drops[b->slot_drop[s]].r;
    r.height = b->shape[4 * s + 0];
    r.base_radius = b->shape[4 * s + 1];
    r.tip_angle_deg = b->shape[4 * s + 2];
  }
  // the resident list on the device is restored by the caller's next upload
  return LBM_OK;
}

// Place queued droplets into the free slots and build their initial state.
int refill(lbm_batch* b, std::vector<int>& fresh) {
  fresh.clear();
  for (int s = 0; s < b->slots && b->next < b->n; ++s) {
    if (b->slot_drop[s] >= 0) continue;
    const int i = b->next++;
    Drop& D = b->drops[i];
    lbmk::State S{};
    lbmk::carve_state(S, b->slot_base(s), b->L.plane, b->storage);
    lbmk::KParams K;
    lbmk::IParams I;
    double Href;
    lbmk::fill_constants(D.P, K, I, Href);
    const long long N = (long long)D.P.nx * D.P.ny;
    if (lbmk::storage_setup(D.P, D.T0, N, K)) {
      g_batch_error = "temperature span too wide for the FP16 node references of 16-bit storage";
      return LBM_EINVAL;
    }
    K.plane = (unsigned)b->L.plane;
    b->ptab[s] = K;
    b->otab[2 * s] = offsets(b, S, 0);
    b->otab[2 * s + 1] = offsets(b, S, 1);
    LBMB_CK(hipMemcpyAsync(b->d_ptab() + s, &b->ptab[s], sizeof(lbmk::KParams), hipMemcpyHostToDevice, b->stream));
    LBMB_CK(hipMemcpyAsync(b->d_otab() + 2 * s, &b->otab[2 * s], 2 * sizeof(lbmk::StepOff), hipMemcpyHostToDevice,
                           b->stream));
    // stage phi0 and T0 (FP64) in the slot's output-field planes (10 planes >= 4)
    double* d_phi0 = (double*)S.fields;
    double* d_T0 = d_phi0 + N;
    LBMB_CK(hipMemcpyAsync(d_phi0, D.phi0, N * sizeof(double), hipMemcpyHostToDevice, b->stream));
    LBMB_CK(hipMemcpyAsync(d_T0, D.T0, N * sizeof(double), hipMemcpyHostToDevice, b->stream));
    if (lbmk::launch_init(K, I, S, 0, d_phi0, d_T0, b->stream)) return bdev_error(hipGetLastError(), "batch init");
    // the host copies above read from ptab/otab entries and the caller's arrays: wait before they can change
    LBMB_CK(hipStreamSynchronize(b->stream));
    b->slot_drop[s] = i;
    D.r.status = LBM_DROP_RUNNING;
    D.r.slot = s;
    D.r.steps = 0;
    fresh.push_back(s);
  }
  if (fresh.empty()) return LBM_OK;
  b->active.clear();
  for (int s = 0; s < b->slots; ++s)
    if (b->slot_drop[s] >= 0) b->active.push_back(s);
  int rc = sample_now(b, fresh);
  if (rc) return rc;
  for (int s : fresh) {
    Drop& D = b->drops[b->slot_drop[s]];
    D.r.liquid0 = D.r.liquid = D.prev_liq = b->h_liq[2 * s];
    D.prev_step = 0;
  }
  return LBM_OK;
}

void retire(lbm_batch* b, int s, int status) {
  Drop& D = b->drops[b->slot_drop[s]];
  D.r.status = status;
  D.r.slot = -1;
  b->slot_drop[s] = -1;
}

// Bookkeeping after one chunk: step counts, liquid volumes, freezing times;
// returns the slots whose droplets finished.
std::vector<int> after_chunk(lbm_batch* b, bool until_frozen, std::vector<int>& finished_status) {
  std::vector<int> done;
  finished_status.clear();
  for (int s : b->active) {
    Drop& D = b->drops[b->slot_drop[s]];
    D.r.steps += b->sample_every;
    const double liq = b->h_liq[2 * s], bad = b->h_liq[2 * s + 1];
    D.r.liquid = liq;
    if (!(bad == 0.0) || !std::isfinite(liq)) {
      done.push_back(s);
      finished_status.push_back(LBM_DROP_NONFINITE);
      continue;
    }
    const double thr = b->freeze_frac * D.r.liquid0;
    if (std::isnan(D.r.t_freeze) && liq <= thr) {
      const double dl = D.prev_liq - liq;
      const double frac = dl > 0.0 ? (D.prev_liq - thr) / dl : 1.0;
      D.r.t_freeze = (double)D.prev_step + std::min(std::max(frac, 0.0), 1.0) * (double)(D.r.steps - D.prev_step);
      const double alpha = D.P.k_l / (D.P.rho_l * D.P.cp_l);
      D.r.t_star = D.radius > 0.0 ? alpha * D.r.t_freeze / (D.radius * D.radius) : std::nan("");
    }
    D.prev_liq = liq;
    D.prev_step = D.r.steps;
    if (!until_frozen) continue;
    if (!std::isnan(D.r.t_freeze)) {
      done.push_back(s);
      finished_status.push_back(LBM_DROP_FROZEN);
    } else if (b->max_steps > 0 && D.r.steps >= b->max_steps) {
      done.push_back(s);
      finished_status.push_back(LBM_DROP_LIMIT);
    }
  }
  return done;
}

}  // namespace

extern "C" {

int lbm_batch_workspace_bytes(const lbm_params* p, int32_t n, int32_t slots, size_t* bytes) {
  if (!p || n < 1 || slots < 1 || slots > 65535 || !bytes) return LBM_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (lbmk::validate_params(&p[i]) || p[i].storage != p[0].storage) return LBM_EINVAL;
    if (max_tiles(p[i].nx, p[i].ny) > 65536) return LBM_EINVAL;
  }
  *bytes = layout(p, n, std::min(slots, n)).total;
  return LBM_OK;
}

int lbm_batch_init(const lbm_params* p, int32_t n, const double* const* phi0, const double* const* T0,
                   const double* radius, int32_t slots, void* d_workspace, size_t ws_bytes, void* hip_stream,
                   lbm_batch** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  size_t need = 0;
  int rc = lbm_batch_workspace_bytes(p, n, slots, &need);
  if (rc) {
    g_batch_error = "invalid batch parameters";
    return rc;
  }
  if (!phi0 || !T0) return LBM_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!phi0[i] || !T0[i]) return LBM_EINVAL;
    const long long N = (long long)p[i].nx * p[i].ny;
    for (long long k = 0; k < N; ++k)
      if (!std::isfinite(phi0[i][k]) || !std::isfinite(T0[i][k])) {
        g_batch_error = "non-finite initial field";
        return LBM_EINVAL;
      }
    // 16-bit storage needs the temperature span to fit its FP16 node
    // references: refuse here rather than when the droplet reaches a slot
    lbmk::KParams K;
    lbmk::IParams I;
    double Href;
    lbmk::fill_constants(p[i], K, I, Href);
    if (lbmk::storage_setup(p[i], T0[i], N, K)) {
      g_batch_error = "temperature span too wide for the FP16 node references of 16-bit storage";
      return LBM_EINVAL;
    }
  }
  if (d_workspace && (ws_bytes < need || ((uintptr_t)d_workspace & 255))) {
    g_batch_error = "workspace too small or not 256-byte aligned";
    return LBM_EINVAL;
  }
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_ENOMEM;
  b->n = n;
  b->slots = std::min(slots, n);
  b->storage = p[0].storage;
  b->L = layout(p, n, b->slots);
  b->stream = (hipStream_t)hip_stream;
  b->cap_stream = nullptr;
  b->exec = nullptr;
  b->graph_valid = false;
  b->h_liq = nullptr;
  b->h_steps = nullptr;
  b->next = 0;
  b->nblocks = 0;
  b->sample_every = 100;
  b->max_steps = 0;
  b->freeze_frac = 0.01;
  b->tile_variant = 0;
  b->xcd_group = 1;
  b->tune_reps = 0;
  b->tuned_active = 0;
  b->store_mode = 0;
  b->nt = false;
  b->use_graph = true;
  b->persist = -1;
  b->bar_limit = 0;
  b->clock_khz = 0;
  b->persist_grid = 0;
  b->h_bar = nullptr;
  b->drops.resize(n);
  for (int i = 0; i < n; ++i) {
    Drop& D = b->drops[i];
    D.P = p[i];
    D.phi0 = phi0[i];
    D.T0 = T0[i];
    D.radius = radius ? radius[i] : 0.0;
    std::memset(&D.r, 0, sizeof(D.r));
    D.r.status = LBM_DROP_QUEUED;
    D.r.slot = -1;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    D.r.t_freeze = D.r.t_star = D.r.height = D.r.base_radius = D.r.tip_angle_deg = nan;
    D.prev_liq = 0.0;
    D.prev_step = 0;
  }
  b->slot_drop.assign(b->slots, -1);
  b->ptab.resize(b->slots);
  b->otab.resize(2 * (size_t)b->slots);
  b->shape.assign(4 * (size_t)b->slots, 0.0);
  hipError_t e = hipGetDevice(&b->device);
  if (e == hipSuccess) e = hipStreamCreate(&b->cap_stream);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_liq, sizeof(double) * 2 * b->slots, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_steps, sizeof(unsigned) * b->slots, hipHostMallocDefault);
  if (e == hipSuccess) std::memset(b->h_steps, 0, sizeof(unsigned) * b->slots);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&b->h_bar, sizeof(unsigned long long) * lbmk::NPERSIST_WORDS, hipHostMallocDefault);
  int rate_khz = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, b->device);
  b->clock_khz = (unsigned long long)(rate_khz > 0 ? rate_khz : 100000);
  b->bar_limit = 2000ull * b->clock_khz;
  if (e != hipSuccess) {
    rc = bdev_error(e, "lbm_batch_init");
    lbm_batch_destroy(b);
    return rc;
  }
  if (d_workspace) {
    b->ws = (char*)d_workspace;
    b->own_ws = false;
  } else {
    e = hipMalloc((void**)&b->ws, b->L.total);
    if (e != hipSuccess) {
      b->ws = nullptr;
      lbm_batch_destroy(b);
      g_batch_error = "hipMalloc of the batch workspace failed";
      return LBM_ENOMEM;
    }
    b->own_ws = true;
  }
  std::vector<int> fresh;
  rc = refill(b, fresh);
  if (rc) {
    lbm_batch_destroy(b);
    return rc;
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_configure(lbm_batch* b, int32_t sample_every, int64_t max_steps, double freeze_frac,
                        int32_t interval_launch, int32_t wait_limit_us) {
  if (!b || sample_every < 2 || (sample_every & 1) || max_steps < 0 || !(freeze_frac > 0.0 && freeze_frac < 1.0))
    return LBM_EINVAL;
  if (interval_launch < LBM_INTERVAL_LAUNCHES || interval_launch > LBM_INTERVAL_PERSIST_PER_XCD) return LBM_EINVAL;
  if (wait_limit_us < 0) return LBM_EINVAL;
  const bool persist = interval_launch >= LBM_INTERVAL_PERSIST_FLAT;
  if (!persist && lbmk::is_two_step_any_storage(b->tile_variant) && sample_every % 4) {
    g_batch_error = "two steps per launch need a sampling interval that is a multiple of 4";
    return LBM_EINVAL;
  }
  b->sample_every = sample_every;
  b->max_steps = max_steps;
  b->freeze_frac = freeze_frac;
  b->use_graph = interval_launch == LBM_INTERVAL_GRAPH;
  b->persist = persist ? interval_launch - LBM_INTERVAL_PERSIST_FLAT : -1;
  b->bar_limit = (wait_limit_us ? (unsigned long long)wait_limit_us : 2000000ull) * b->clock_khz / 1000ull;
  drop_graph(b);
  if (persist && b->tile_variant != kPersistVariant) {  // the persistent kernel runs 64x8 tiles
    b->tile_variant = kPersistVariant;
    return upload_map(b);
  }
  return LBM_OK;
}

// Batch launch shapes: the single-step tiles 0-4 and, with a sampling
// interval that is a multiple of 4, the two-step variants 9 and 10; with
// persistent intervals, 64x8 only.
static bool batch_variant_ok(const lbm_batch* b, int v) {
  if (b->persist >= 0) return v == kPersistVariant;
  if (v >= 0 && v < lbmk::NBATCH_VARIANTS) return true;
  return lbmk::is_two_step_any_storage(v) && b->sample_every % 4 == 0;
}

int lbm_batch_set_launch(lbm_batch* b, int32_t tile_variant, int32_t xcd_group) {
  if (!b || !batch_variant_ok(b, tile_variant) || xcd_group < 0 || xcd_group > 2) return LBM_EINVAL;
  b->tile_variant = tile_variant;
  b->xcd_group = xcd_group;
  return upload_map(b);
}

int lbm_batch_set_store_mode(lbm_batch* b, int32_t mode) {
  if (!b || mode < 0 || mode > 2) return LBM_EINVAL;
  b->store_mode = mode;
  // mode 0 keeps cached stores: many small grids, each grouped on one XCD,
  // re-read their own output next step often enough that streaming stores
  // cost 7 % on the sweep even when the whole batch exceeds the cache
  b->nt = mode == 2;
  drop_graph(b);  // the captured launches name the kernel
  return LBM_OK;
}

int lbm_batch_autotune(lbm_batch* b, int32_t reps, int32_t* tile_variant, int32_t* xcd_group) {
  if (!b || reps < 1) return LBM_EINVAL;
  if (b->active.empty()) return LBM_OK;
  // Every resident droplet sits at an even step, so its state is in buffer
  // set 0; a launch with parity 0 reads set 0 and writes set 1 only, and can
  // be replayed without advancing anything.
  struct Events {
    hipEvent_t a = nullptr, c = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (c) (void)hipEventDestroy(c);
    }
  } ev;
  LBMB_CK(hipEventCreate(&ev.a));
  LBMB_CK(hipEventCreate(&ev.c));
  float best = 1e30f;
  int bv = b->tile_variant, bx = b->xcd_group;
  for (int v = 0; v < lbmk::NTILE_VARIANTS; ++v) {
    if (!batch_variant_ok(b, v)) continue;
    const float per_launch = lbmk::is_two_step_any_storage(v) ? 2.0f : 1.0f;  // steps per launch
    for (int x = 0; x <= 2; ++x) {
      b->tile_variant = v;
      b->xcd_group = x;
      int rc = upload_map(b);
      if (rc) return rc;
      if (lbmk::launch_batch(b->storage, v, false, b->nt, b->ws, b->d_ptab(), b->d_otab(), b->d_tmap(), b->d_steps(),
                             b->nblocks, 0, b->stream))
        return bdev_error(hipGetLastError(), "autotune launch");
      LBMB_CK(hipEventRecord(ev.a, b->stream));
      for (int r = 0; r < reps; ++r)
        if (lbmk::launch_batch(b->storage, v, false, b->nt, b->ws, b->d_ptab(), b->d_otab(), b->d_tmap(), b->d_steps(),
                               b->nblocks, 0, b->stream))
          return bdev_error(hipGetLastError(), "autotune launch");
      LBMB_CK(hipEventRecord(ev.c, b->stream));
      LBMB_CK(hipEventSynchronize(ev.c));
      float ms = 0.0f;
      LBMB_CK(hipEventElapsedTime(&ms, ev.a, ev.c));
      ms /= per_launch;  // compare time per step
      if (ms < best) {
        best = ms;
        bv = v;
        bx = x;
      }
    }
  }
  b->tile_variant = bv;
  b->xcd_group = bx;
  b->tune_reps = reps;
  b->tuned_active = (int)b->active.size();
  if (tile_variant) *tile_variant = bv;
  if (xcd_group) *xcd_group = bx;
  return upload_map(b);
}

int lbm_batch_step(lbm_batch* b, int64_t nsteps, int32_t until_frozen) {
  if (!b || nsteps < 0) return LBM_EINVAL;
  if (b->nblocks == 0 && !b->active.empty()) {
    int rc = upload_map(b);
    if (rc) return rc;
  }
  int64_t done_steps = 0;
  std::vector<int> status;
  while (done_steps < nsteps && !b->active.empty()) {
    int rc = run_chunk(b);
    if (rc) return rc;
    LBMB_CK(hipStreamSynchronize(b->stream));
    if (b->persist >= 0 && (rc = check_barrier(b))) return rc;
    done_steps += b->sample_every;
    std::vector<int> fin = after_chunk(b, until_frozen != 0, status);
    if (fin.empty()) continue;
    // shapes from the fields pass of this chunk, then free and refill the slots
    std::vector<int> shaped;
    for (size_t j = 0; j < fin.size(); ++j)
      if (status[j] != LBM_DROP_NONFINITE) shaped.push_back(fin[j]);
    rc = measure_shapes(b, shaped);
    if (rc) return rc;
    for (size_t j = 0; j < fin.size(); ++j) retire(b, fin[j], status[j]);
    std::vector<int> fresh;
    rc = refill(b, fresh);
    if (rc) return rc;
    b->active.clear();
    for (int s = 0; s < b->slots; ++s)
      if (b->slot_drop[s] >= 0) b->active.push_back(s);
    rc = upload_map(b);
    if (rc) return rc;
    // the tail of a sweep, with few droplets left, favours other launches:
    // re-tune once the resident set has halved since the last tuning
    if (b->tune_reps > 0 && !b->active.empty() && 2 * (int)b->active.size() <= b->tuned_active) {
      rc = lbm_batch_autotune(b, b->tune_reps, nullptr, nullptr);
      if (rc) return rc;
    }
  }
  return LBM_OK;
}

int lbm_batch_results(lbm_batch* b, lbm_drop_result* out) {
  if (!b || !out) return LBM_EINVAL;
  for (int i = 0; i < b->n; ++i) out[i] = b->drops[i].r;
  return LBM_OK;
}

int lbm_batch_fields(lbm_batch* b, int32_t drop, uint32_t mask, double* const* host_out) {
  if (!b || drop < 0 || drop >= b->n || !host_out || (mask >> lbmk::NFIELD)) return LBM_EINVAL;
  const int s = b->drops[drop].r.slot;
  if (s < 0 || b->drops[drop].r.status != LBM_DROP_RUNNING) {
    g_batch_error = "droplet is not resident";
    return LBM_ESTATE;
  }
  int rc = sample_now(b, std::vector<int>{s});  // fields pass of this slot (state untouched)
  if (rc) return rc;
  const lbm_params& P = b->drops[drop].P;
  const long long N = (long long)P.nx * P.ny;
  const double Href = P.cp_ref * P.T_melt + P.latent;
  const float* F = (const float*)(b->ws + b->otab[2 * s].fields);
  std::vector<float> stage(N);
  int j = 0;
  for (int f = 0; f < lbmk::NFIELD; ++f) {
    if (!(mask & (1u << f))) continue;
    if (!host_out[j]) return LBM_EINVAL;
    LBMB_CK(hipMemcpyAsync(stage.data(), F + (size_t)f * b->L.plane, N * sizeof(float), hipMemcpyDeviceToHost,
                           b->stream));
    LBMB_CK(hipStreamSynchronize(b->stream));
    const double add = f == 8 ? Href : 0.0;  // H is kept relative to H_ref on the device
    for (long long k = 0; k < N; ++k) host_out[j][k] = (double)stage[k] + add;
    ++j;
  }
  return LBM_OK;
}

int lbm_shape_of(const double* phi, int32_t nx, int32_t ny, double* out) {
  if (!phi || !out || nx < 1 || ny < 1 || (long long)nx * ny > (1LL << 30)) return LBM_EINVAL;
  const long long N = (long long)nx * ny;
  const size_t o_ptab = 0, o_otab = align_up(sizeof(lbmk::KParams)), o_slot = align_up(o_otab + 2 * sizeof(lbmk::StepOff));
  const size_t o_out = align_up(o_slot + sizeof(int)), o_phi = align_up(o_out + 4 * sizeof(double));
  const size_t total = o_phi + N * sizeof(float);
  std::vector<char> host(total, 0);
  lbmk::KParams K{};
  K.nx = nx;
  K.ny = ny;
  K.plane = (unsigned)lbmk::plane_floats(N);
  std::memcpy(host.data() + o_ptab, &K, sizeof(K));
  lbmk::StepOff off{};
  off.fields = o_phi;
  std::memcpy(host.data() + o_otab, &off, sizeof(off));
  float* hp = (float*)(host.data() + o_phi);
  for (long long k = 0; k < N; ++k) hp[k] = (float)phi[k];
  char* d = nullptr;
  LBMB_CK(hipMalloc((void**)&d, total));
  hipError_t e = hipMemcpy(d, host.data(), total, hipMemcpyHostToDevice);
  if (e == hipSuccess && lbmk::launch_batch_shape(d, (const lbmk::KParams*)(d + o_ptab),
                                                  (const lbmk::StepOff*)(d + o_otab), (const int*)(d + o_slot), 1,
                                                  (double*)(d + o_out), nullptr))
    e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(out, d + o_out, 4 * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return bdev_error(e, "lbm_shape_of");
  return LBM_OK;
}

const char* lbm_batch_last_error(void) { return g_batch_error.c_str(); }

void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  if (b->stream || b->cap_stream) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  if (b->own_ws && b->ws) (void)hipFree(b->ws);
  if (b->h_liq) (void)hipHostFree(b->h_liq);
  if (b->h_steps) (void)hipHostFree(b->h_steps);
  if (b->h_bar) (void)hipHostFree(b->h_bar);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}

}  // extern "C"
