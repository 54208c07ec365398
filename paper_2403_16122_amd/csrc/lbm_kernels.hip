// gfx950 kernels of the coupled phase-field / flow / enthalpy D2Q9 step
// (Huang, Wang, Chai & Shi, arXiv:2403.16122, Sec. 3).
//
// One fused kernel per time step.  A workgroup owns a TX x TY tile of nodes
// (one node per lane, TX lanes along x so a wavefront reads whole rows).
// It first rebuilds, for the tile plus a halo ring, the node-local
// macroscopic quantities of time t (pull-streamed g and h -> H, f_l, T,
// mass source, phi, rho; Eq. (9), (19), (26), (1)) into LDS, fills the wall
// ghost rows with the wetting condition (Eq. (39)-(41)), and then evaluates
// the isotropic stencils of Eq. (38), the forces, the flow macros and the
// three BGK collisions for its own nodes, writing post-collision
// populations to the other buffer.  Halo macros are recomputed rather than
// exchanged, so a step is one launch and HBM sees each population once per
// direction.
#include "lbm_internal.h"

#include <algorithm>
#include <type_traits>

namespace lbmk {
namespace {

// D2Q9 order: rest, +x, +y, -x, -y, (+x,+y), (-x,+y), (-x,-y), (+x,-y)
constexpr float W0 = 4.0f / 9.0f, W1 = 1.0f / 9.0f, W5 = 1.0f / 36.0f;
__device__ __forceinline__ constexpr float wt(int i) { return i == 0 ? W0 : (i < 5 ? W1 : W5); }
__device__ __forceinline__ constexpr int cxv(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__device__ __forceinline__ constexpr int cyv(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__device__ __forceinline__ constexpr int opp(int i) {
  return i == 0 ? 0 : (i < 5 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5);
}

// The first direction of each pair of opposite ones: 1, 2, 5, 6.
__device__ __forceinline__ constexpr int pair_dir(int j) { return j < 2 ? j + 1 : j + 3; }

__device__ __forceinline__ float clamp01(float v) { return fminf(fmaxf(v, 0.0f), 1.0f); }
__device__ __forceinline__ float mix3(float fs, float pc, float zs, float zl, float zg) {
  // Eq. (1) with the clamped order parameter, fs zs + (1 - fs)(pc zl +
  // (1 - pc) zg), as two multiply-adds: exactly zl, zg or zs in a pure phase
  const float fluid = __builtin_fmaf(pc, zl, (1.0f - pc) * zg);
  return __builtin_fmaf(fs, zs, (1.0f - fs) * fluid);
}
// Periodic x: one compare-and-shift covers |x| < 2 nx; the modulo only
// runs for grids narrower than a tile.
__device__ __forceinline__ int wrapx(int x, int nx) {
  int r = x < 0 ? x + nx : (x >= nx ? x - nx : x);
  if ((unsigned)r >= (unsigned)nx) r = ((x % nx) + nx) % nx;
  return r;
}

// Element access by a 32-bit index: the byte offset is formed in 32 bits so
// the load/store uses the scalar-base + 32-bit-vector-offset addressing form.
__device__ __forceinline__ float ld(const float* __restrict__ base, unsigned idx) {
  return *(const float*)((const char*)base + (idx << 2));
}
// NT: a streaming store, which does not keep the line in the caches (for
// state that cannot stay cache-resident until the next step reads it).
template <bool NT = false>
__device__ __forceinline__ void st(float* __restrict__ base, unsigned idx, float v) {
  float* a = (float*)((char*)base + (idx << 2));
  if constexpr (NT)
    __builtin_nontemporal_store(v, a);
  else
    *a = v;
}
template <bool NT, class T>
__device__ __forceinline__ void st_as(void* a, T v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, (T*)a);
  else
    *(T*)a = v;
}

// Plane j of an array of FP32 planes of pl elements: the same address for
// every lane (scalar arithmetic), so that an element is then addressed by
// the node's own 32-bit offset, shared by every plane.
__device__ __forceinline__ float* fplane(float* base, unsigned j, unsigned pl) {
  return (float*)((char*)base + (size_t)j * pl * sizeof(float));
}
__device__ __forceinline__ const float* fplane(const float* base, unsigned j, unsigned pl) {
  return (const float*)((const char*)base + (size_t)j * pl * sizeof(float));
}

// Hardware reciprocal (1 ulp); used identically wherever a node is rebuilt.
__device__ __forceinline__ float rcp(float v) { return __builtin_amdgcn_rcpf(v); }

// Population storage.  FP32 keeps the shifted populations as computed.  The
// 16-bit formats round them stochastically (the hardware's v_cvt_sr_*: the
// random word is added below the kept mantissa bits before truncation), so
// the rounding error has zero mean even where a node stores the same value
// step after step; round-to-nearest there loses phase-field mass steadily
// and shifts freezing times by percents.  The random word of a store is a
// hash of the node index and the step number, xor-ed with a constant per
// population, so results do not depend on the launch shape.  FP16 first multiplies by a per-lattice power of two (exact
// in FP32, undone on load) so that the small shifted values stay in its
// normal range; BF16 has FP32's exponent range and is not scaled.  Compute
// is FP32 throughout.
typedef __bf16 bf162v __attribute__((ext_vector_type(2)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));

// 32-bit finalizer of MurmurHash3 (a bijective avalanche mix).
__device__ __forceinline__ unsigned fmix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}
__device__ __forceinline__ unsigned sr_node(unsigned k, unsigned seed) {
  return fmix32(k * 0x9e3779b1u ^ seed * 0x85ebca77u);
}
// word of population j (0..26) of a node from its hash
__device__ __forceinline__ constexpr unsigned sr_pop(int j) { return 0x9e3779b9u * (unsigned)(j + 1); }
// One stored value: FP32 as is; 16-bit formats rounded stochastically with
// random word rnd (v_cvt_sr_f16_f32 / v_cvt_sr_bf16_f32).
template <class PT>
__device__ __forceinline__ PT cvt_store(float v, unsigned rnd);
template <>
__device__ __forceinline__ float cvt_store<float>(float v, unsigned) {
  return v;
}
template <>
__device__ __forceinline__ _Float16 cvt_store<_Float16>(float v, unsigned rnd) {
  // the conversion writes the low half; the high half is never read, so
  // it is left undefined (no register to clear first)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wuninitialized"
  half2v h;
  h = __builtin_amdgcn_cvt_sr_f16_f32(h, v, rnd, false);
#pragma clang diagnostic pop
  return h.x;
}
template <>
__device__ __forceinline__ __bf16 cvt_store<__bf16>(float v, unsigned rnd) {
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wuninitialized"
  bf162v h;
  h = __builtin_amdgcn_cvt_sr_bf16_f32(h, v, rnd, false);
#pragma clang diagnostic pop
  return h.x;
}
template <class PT>
struct PopIO;
// kNodeRef: the 16-bit formats keep h relative to the writing node's own
// temperature as well (exact algebra, like the phi reference of g), so the
// stored h values are non-equilibrium-sized; FP32 resolves the coarser
// shift relative to T_m well enough.  f is stored as computed in every
// format.
template <>
struct PopIO<float> {
  static constexpr bool kNodeRef = false;
  static constexpr bool kScaled = false;
  static __device__ __forceinline__ float get(const void* b, unsigned idx) { return ld((const float*)b, idx); }
  template <bool NT>
  static __device__ __forceinline__ void put(void* b, unsigned idx, float v, unsigned) {
    st<NT>((float*)b, idx, v);
  }
};
template <>
struct PopIO<_Float16> {
  static constexpr bool kNodeRef = true;
  static constexpr bool kScaled = true;
  static __device__ __forceinline__ float get(const void* b, unsigned idx) {
    return (float)*(const _Float16*)((const char*)b + (idx << 1));
  }
  template <bool NT>
  static __device__ __forceinline__ void put(void* b, unsigned idx, float v, unsigned rnd) {
    st_as<NT, _Float16>((char*)b + (idx << 1), cvt_store<_Float16>(v, rnd));
  }
};
template <>
struct PopIO<__bf16> {
  static constexpr bool kNodeRef = true;
  static constexpr bool kScaled = false;
  static __device__ __forceinline__ float get(const void* b, unsigned idx) {
    return (float)*(const __bf16*)((const char*)b + (idx << 1));
  }
  template <bool NT>
  static __device__ __forceinline__ void put(void* b, unsigned idx, float v, unsigned rnd) {
    st_as<NT, __bf16>((char*)b + (idx << 1), cvt_store<__bf16>(v, rnd));
  }
};
// Node references.  FP32 storage keeps phi_ref, the reference of the stored
// g, as an FP32 plane.  The node-reference formats keep the pair
// (phi_ref, th) as two FP16 values in one 32-bit word per node: the writer
// first rounds its phi and T - T_m to FP16 and shifts by the rounded
// values, so writer and readers use identical references.
template <bool NR>
struct RefIO;
template <>
struct RefIO<false> {
  static __device__ __forceinline__ void load(const void* b, unsigned k, float& r, float& th) {
    r = ld((const float*)b, k);
    th = 0.0f;
  }
  static __device__ __forceinline__ void round(float phi, float dT, float& r, float& th) {
    r = phi;
    th = 0.0f;
  }
  template <bool NT = false>
  static __device__ __forceinline__ void store(void* b, unsigned k, float r, float) {
    st<NT>((float*)b, k, r);
  }
};
template <>
struct RefIO<true> {
  static __device__ __forceinline__ void load(const void* b, unsigned k, float& r, float& th) {
    const half2v v = *(const half2v*)((const char*)b + (k << 2));
    r = (float)v.x;
    th = (float)v.y;
  }
  static __device__ __forceinline__ void round(float phi, float dT, float& r, float& th) {
    r = (float)(_Float16)phi;
    th = (float)(_Float16)dT;
  }
  template <bool NT = false>
  static __device__ __forceinline__ void store(void* b, unsigned k, float r, float th) {
    half2v v;
    v.x = (_Float16)r;  // exact: r and th are already FP16 values
    v.y = (_Float16)th;
    st_as<NT, half2v>((char*)b + (k << 2), v);
  }
};

// rnd: the node's hash (sr_node) xor sr_pop(population); unused for FP32
template <class PT, int LAT, bool NT = false>
__device__ __forceinline__ void pop_st(void* B, unsigned idx, float v, const KParams& P, unsigned rnd) {
  if constexpr (PopIO<PT>::kScaled) v *= P.sc_st[LAT];
  PopIO<PT>::template put<NT>(B, idx, v, rnd);
}
// The same value into an LDS array of the storage type (two steps per
// launch keep the first step's populations as stored, bit for bit).
template <class PT, int LAT>
__device__ __forceinline__ void pop_lds_st(PT* dst, float v, const KParams& P, unsigned rnd) {
  if constexpr (PopIO<PT>::kScaled) v *= P.sc_st[LAT];
  *dst = cvt_store<PT>(v, rnd);
}
// Pull-stream the 9 populations of one lattice into node (x, y).  Sources
// beyond a wall are replaced by the bounce-back of the node's own opposite
// population (half-way rule); for h at the bottom wall by the
// anti-bounce-back Dirichlet value -h_opp + 2 w_i cp_ref (T_w - T_m) in the
// shifted variables.
//
// Addressing: direction i of lattice LAT is read relative to the plane
// pbase(i) = min(i, opp(i)) of that lattice, a base address that is the same
// for every lane (kept in scalar registers), plus a 32-bit byte offset that
// depends only on the node and the direction: a neighbour's population at
// (i - pbase(i)) planes + its index, or, beyond a wall, the node's own
// opposite population at (opp(i) - pbase(i)) planes + the node's index --
// both non-negative.  The offsets are therefore shared by g, f and h.
__device__ __forceinline__ constexpr int pbase(int i) { return i < opp(i) ? i : opp(i); }

__device__ __forceinline__ unsigned pull_off(const KParams& P, int i, int x, int y, int xm, int xp) {
  const unsigned pl = P.plane;
  const unsigned nx = (unsigned)P.nx;
  const bool bot = (y == 0), top = (y == P.ny - 1);
  const unsigned rowc = (unsigned)y * nx;
  const unsigned rowd = rowc - nx, rowu = rowc + nx;  // used only away from the walls
  const int cy = cyv(i), cx = cxv(i);
  const bool wall = (cy > 0 && bot) || (cy < 0 && top);
  const unsigned sx = (unsigned)(cx > 0 ? xm : (cx < 0 ? xp : x));
  const unsigned sk = (cy > 0 ? rowd : (cy < 0 ? rowu : rowc)) + sx;
  return wall ? (unsigned)(opp(i) - pbase(i)) * pl + rowc + (unsigned)x : (unsigned)(i - pbase(i)) * pl + sk;
}

// The stored value of direction i of lattice LAT pulled from element offset
// `off` (pull_off) of its base plane.
template <int LAT, class PT>
__device__ __forceinline__ PT pull_raw(const void* __restrict__ A, const KParams& P, int i, unsigned off) {
  const char* base = (const char*)A + (size_t)(LAT * 9 + pbase(i)) * P.plane * sizeof(PT);
  return *(const PT*)(base + (off * (unsigned)sizeof(PT)));
}

template <int LAT, class PT>
__device__ __forceinline__ void pull9(const void* __restrict__ A, const KParams& P, int x, int y,
                                      int xm, int xp, float q[9]) {
  const bool bot = (y == 0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int cy = cyv(i);
    float v = (float)pull_raw<LAT, PT>(A, P, i, pull_off(P, i, x, y, xm, xp));
    if constexpr (PopIO<PT>::kScaled) v *= P.sc_ld[LAT];
    if (LAT == 2 && cy > 0) v = bot ? (P.hwall[i] - v) : v;
    q[i] = v;
  }
}

// Re-express freshly pulled g populations (node at LDS cell (c, r), row y)
// in the reference of the receiving node: q_i += w_i (phi_ref(src) - phi_ref(self)).
// The reference tile holds phi_ref of cell (c, r) at sref[r + 1][c + 1].
template <int RX>
__device__ __forceinline__ float rebase_g(float q[9], const float (*sref)[RX], const KParams& P,
                                          int y, int c, int r) {
  // the same node is rebuilt by its own lane and as a halo cell of its
  // neighbours' tiles: no FMA contraction, so both round identically
#pragma clang fp contract(off)
  const bool bot = (y == 0), top = (y == P.ny - 1);
  const float rself = sref[r + 1][c + 1];
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int cy = cyv(i), cx = cxv(i);
    const bool wall = (cy > 0 && bot) || (cy < 0 && top);
    const float rs = wall ? rself : sref[r + 1 - cy][c + 1 - cx];
    q[i] += wt(i) * (rs - rself);
  }
  return rself;
}

// The same for h under the node-reference storage: stored h_i is relative
// to w_i cp_ref th(writer), th = T - T_m of the writer's step.  Received
// populations move to the receiver's reference; the anti-bounce-back ones
// at the bottom wall (built from the node's own populations) to
// -h_opp + 2 w_i cp_ref (T_w - T_m - th) in that reference.
template <int RX>
__device__ __forceinline__ float rebase_h(float q[9], const float (*sth)[RX], const KParams& P,
                                          int y, int c, int r) {
#pragma clang fp contract(off)
  const bool bot = (y == 0), top = (y == P.ny - 1);
  const float tself = sth[r + 1][c + 1];
  const float cw = P.cp_ref * tself;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int cy = cyv(i), cx = cxv(i);
    if (cy > 0 && bot) {
      q[i] -= (2.0f * wt(i)) * cw;
    } else if (!(cy < 0 && top)) {
      q[i] += wt(i) * (P.cp_ref * sth[r + 1 - cy][c + 1 - cx] - cw);
    }
  }
  return tself;
}

struct Macro {
  float g[9], h[9];
  float E;      // H - H_l + L f_s^H(n-1): the enthalpy excess over the stored latent part
  float dT;     // T - T_m
  float fprev;  // f_s^H of the previous step
  float cp, kk, fl, fsH, mdot, phi, fsol, rho, mu;
  float r;      // reference phi of the received g populations (own previous phi)
  float dl;     // phi - r, resolved to the precision of the small stored numbers
  float th;     // reference T - T_m of the received h populations (node-reference storage)
};

// Node-local macroscopic quantities of time t (Eq. (29), (9), (19), (26), (1)).
//
// Storage of h: every population is kept relative to the equilibrium of
// liquid at rest at T_m (h_i - h_i^ref), and the rest population, which
// carries the latent heat, is additionally kept relative to L f_s^H of the
// previous step: s_0 = (h_0 - h_0^ref) + L f_s^H(n-1).  Both shifts are
// exact algebra; together they keep every stored value small, so FP32
// resolves H to ~1e-7 of the sensible part in liquid, mushy and solid
// nodes alike instead of ~1e-6 of H ~ L.
// Issue the loads of one node's macroscopic inputs: pulled g and h (wall
// rules applied) and f_s^H of the previous step.
template <class PT>
__device__ __forceinline__ void load_node(const void* __restrict__ A,
                                          const float* __restrict__ fsH_prev, const KParams& P,
                                          int x, int y, Macro& m) {
  const int xm = x == 0 ? P.nx - 1 : x - 1;
  const int xp = x == P.nx - 1 ? 0 : x + 1;
  pull9<0, PT>(A, P, x, y, xm, xp, m.g);
  pull9<2, PT>(A, P, x, y, xm, xp, m.h);
  m.fprev = ld(fsH_prev, (unsigned)(y * P.nx + x));
}

// The 16-bit formats hold pulled populations as loaded, two per register,
// from the load to their first use after the tile's barrier, and convert
// then (the same conversion, scale and wall rule as pull9, in the same
// order): the loads in flight across the barrier take half the registers.
template <class PT>
struct Raw9 {
  typedef PT v2 __attribute__((ext_vector_type(2)));
  v2 p[5];
};

template <int LAT, class PT>
__device__ __forceinline__ void pull9_raw(const void* __restrict__ A, const KParams& P, int x, int y, int xm,
                                          int xp, Raw9<PT>& r) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const PT v = pull_raw<LAT, PT>(A, P, i, pull_off(P, i, x, y, xm, xp));
    if (i & 1)
      r.p[i >> 1].y = v;
    else
      r.p[i >> 1].x = v;
  }
}

template <int LAT, class PT>
__device__ __forceinline__ void unpack9(const Raw9<PT>& r, const KParams& P, int y, float q[9]) {
  const bool bot = (y == 0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    float v = (float)((i & 1) ? r.p[i >> 1].y : r.p[i >> 1].x);
    if constexpr (PopIO<PT>::kScaled) v *= P.sc_ld[LAT];
    if (LAT == 2 && cyv(i) > 0) v = bot ? (P.hwall[i] - v) : v;
    q[i] = v;
  }
}

template <class PT>
__device__ __forceinline__ void load_node_raw(const void* __restrict__ A, const float* __restrict__ fsH_prev,
                                              const KParams& P, int x, int y, Raw9<PT>& g, Raw9<PT>& h,
                                              float& fprev) {
  const int xm = x == 0 ? P.nx - 1 : x - 1;
  const int xp = x == P.nx - 1 ? 0 : x + 1;
  pull9_raw<0, PT>(A, P, x, y, xm, xp, g);
  pull9_raw<2, PT>(A, P, x, y, xm, xp, h);
  fprev = ld(fsH_prev, (unsigned)(y * P.nx + x));
}

// Node-local macroscopic quantities of time t (Eq. (29), (9), (19), (26), (1))
// from the loaded inputs; m.g must already be rebased to reference rs and,
// under NODEREF, m.h to m.th.
template <bool NODEREF>
__device__ __forceinline__ void finish_macro(const KParams& P, float rs, Macro& m) {
  // computed both for own nodes and for halo cells: no FMA contraction, so
  // every tile shape yields bit-identical values
#pragma clang fp contract(off)
  const float fprev = m.fprev;
  float D0 = 0.0f, hs = 0.0f;  // D0 = sum g_i - r
#pragma unroll
  for (int i = 0; i < 9; ++i) D0 += m.g[i];
  const float G0 = rs + D0;
#pragma unroll
  for (int i = 1; i < 9; ++i) hs += m.h[i];
  const float pc0 = clamp01(G0);
  const float fs_lag = pc0 * fprev;  // cp and k use the lagged solid fraction
  const float cp = mix3(fs_lag, pc0, P.cp_s, P.cp_l, P.cp_g);
  const float kk = mix3(fs_lag, pc0, P.k_s, P.k_l, P.k_g);
  // H - H_l = E - L f_s^H(n-1) and H - H_s = E + L (1 - f_s^H(n-1)) for
  // H_s = cp T_m, H_l = cp T_m + L (Eq. (9))
  float E = hs + m.h[0] + (P.cp_ref - cp) * P.T_melt;
  if (NODEREF) E = E + P.cp_ref * m.th;
  const float dHl = E - P.latent * fprev;
  const float dHs = E + P.latent * (1.0f - fprev);
  const float fl = clamp01(E * P.inv_latent + (1.0f - fprev));
  const float rcpc = rcp(cp);
  const float dT = dHs < 0.0f ? dHs * rcpc : (dHl > 0.0f ? dHl * rcpc : 0.0f);
  const float fsH = 1.0f - fl;
  const float mdot = P.mdot_coef * pc0 * (fsH - fprev);
  // phi from Eq. (26) with div(u) = mdot; phi - r = (D0 + r mdot/2)/(1 - mdot/2)
  const float rden = rcp(1.0f - 0.5f * mdot);
  const float dl = (D0 + 0.5f * rs * mdot) * rden;
  const float phi = rs + dl;
  const float pc = clamp01(phi);
  m.r = rs;
  m.dl = dl;
  const float fsol = pc * fsH;
  m.E = E;
  m.dT = dT;
  m.cp = cp;
  m.kk = kk;
  m.fl = fl;
  m.fsH = fsH;
  m.mdot = mdot;
  m.phi = phi;
  m.fsol = fsol;
  m.rho = mix3(fsol, pc, P.rho_s, P.rho_l, P.rho_g);
  m.mu = mix3(fsol, pc, P.mu_s, P.mu_l, P.mu_g);
}

// Gradients and Laplacian of Eq. (38) at one node: phi (with its
// Laplacian) and rho at time t, and q = S/3 - p of the lagged p and S.
struct Grads {
  float phx, phy, lphi, rx, ry, qx, qy;  // q = S/3 - p (only its gradient enters Eq. (36))
};

// 3 sum_{i>0} w_i c_i z_i and 6 sum_{i>0} w_i (z_i - z_0) over the 8 neighbours.
__device__ __forceinline__ void stencil(float C, float E, float Wv, float N, float S, float NE,
                                        float NW, float SW, float SE, float& gx, float& gy,
                                        float* lap) {
#pragma clang fp contract(off)
  // differences of neighbours in the same row (for x) or column (for y)
  // first: exact where the field varies only across them (a layered flow
  // keeps a zero x-gradient in FP32)
  gx = __builtin_fmaf(E - Wv, 1.0f / 3.0f, ((NE - NW) + (SE - SW)) * (1.0f / 12.0f));
  gy = __builtin_fmaf(N - S, 1.0f / 3.0f, ((NE - SE) + (NW - SW)) * (1.0f / 12.0f));
  if (lap)
    *lap = __builtin_fmaf((E + N + Wv + S) - 4.0f * C, 2.0f / 3.0f, ((NE + NW + SW + SE) - 4.0f * C) * (1.0f / 6.0f));
}

// Wetting ghost value (Eq. (39)-(41)) beyond a wall row: a0 = phi - 1 of
// the adjacent row at columns c-1, c, c+1 and a1 the same for the next row;
// returns phi - 1 of the ghost cell.
__device__ __forceinline__ float wetting_ghost(float a0m, float a0c, float a0p, float a1m, float a1p,
                                               float tv) {
#pragma clang fp contract(off)
  const float d0 = 0.5f * (a0p - a0m);
  const float d1 = 0.5f * (a1p - a1m);
  return a0c + tv * fabsf(1.5f * d0 - 0.5f * d1);
}

// Everything after the stencils for one node k: interface terms (Eq. (3),
// (12), (13)), forces (Eq. (11)), flow macros (Eq. (34)-(36)) and the three
// BGK collisions with their stores, or the output fields when FIELDS.
// LS > 0: the node's results go to LDS instead, for a second step in the
// same launch: the 27 populations as stored (storage type, same rounding)
// at lop[j * LS] in the global plane order, and the references, (phi u),
// f_s^H, p and S as FP32 at loa[AUX_* * LS].  dseed: the step's offset
// from P.seed (stochastic rounding of 16-bit storage).
enum { AUX_REF = 0, AUX_PHIUX = 1, AUX_PHIUY = 2, AUX_FSH = 3, AUX_P = 4, AUX_S = 5, AUX_TH = 6 };
template <class PT>
constexpr int aux_planes() {
  return PopIO<PT>::kNodeRef ? 7 : 6;
}
template <bool FIELDS, class PT, bool STREAM = false, int LS = 0>
__device__ __forceinline__ void update_node(const KParams& P, const StepIO& io, const Macro& m,
                                            const float f[9], float phiux, float phiuy,
                                            const Grads& d, unsigned k, PT* lop = nullptr, float* loa = nullptr,
                                            unsigned dseed = 0) {
  static_assert(LS == 0 || !FIELDS, "LDS results: time steps only");
  const float phi = m.phi, rho = m.rho;
  const float om = (1.0f - m.r) - m.dl;  // 1 - phi without cancellation in either bulk
  // interface terms (Eq. (3), (12), (13))
  const float lam = P.four_over_W * phi * om;
  const float gn2 = d.phx * d.phx + d.phy * d.phy;
  float lnx = 0.0f, lny = 0.0f;
  if (gn2 > 1e-24f) {
    const float s = lam * rsqrtf(gn2);
    lnx = s * d.phx;
    lny = s * d.phy;
  }
  const float muphi = -P.beta4 * phi * om * (phi - 0.5f) - P.kappa * d.lphi;
  const float smask = 1.0f - P.chi * m.fsol;
  const float T = P.T_melt + m.dT;
  // explicit FMAs: contraction here is otherwise left to the code
  // generator, which may fuse either product with the sum depending on the
  // surrounding kernel, and every launch variant must round alike
  const float gcoef = __builtin_fmaf(-P.bq_coef, T - P.bq_Tref, rho);
  const float smu = smask * muphi;
  const float Fx = __builtin_fmaf(gcoef, P.gx, smu * d.phx);
  const float Fy = __builtin_fmaf(gcoef, P.gy, smu * d.phy);

  // flow populations (Eq. (34)-(35)), loaded in phase 0
  const float mx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const float my = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  const float rrho = rcp(rho);
  const float usx = (mx + 0.5f * Fx) * rrho, usy = (my + 0.5f * Fy) * rrho;
  const float fbx = -m.fsol * usx, fby = -m.fsol * usy;  // f = f_s (u_s - u*), u_s = 0
  const float ux = usx + 0.5f * fbx, uy = usy + 0.5f * fby;
  const float Ssrc = rho * m.mdot + ux * d.rx + uy * d.ry;
  // Ft = F - grad p + (grad rho + grad S) / 3, with q = S/3 - p
  const float Ftx = __builtin_fmaf(1.0f / 3.0f, d.rx, Fx + d.qx);
  const float Fty = __builtin_fmaf(1.0f / 3.0f, d.ry, Fy + d.qy);
  const float uFt = ux * Ftx + uy * Fty;
  const float usq = ux * ux + uy * uy;
  const float tauf = 3.0f * m.mu * rrho + 0.5f;
  const float F0 = W0 * (Ssrc - 3.0f * uFt);
  float sumf = 0.0f;
#pragma unroll
  for (int i = 1; i < 9; ++i) sumf += f[i];
  const float p = 0.6f * (sumf + 0.5f * Ssrc + tauf * F0 + rho * (W0 * (-1.5f * usq)));

  if (FIELDS) {
    float* __restrict__ fields = io.fields;
    const unsigned pl = P.plane;
    st(fplane(fields, 0, pl), k, phi);
    st(fplane(fields, 1, pl), k, T);
    st(fplane(fields, 2, pl), k, ux);
    st(fplane(fields, 3, pl), k, uy);
    st(fplane(fields, 4, pl), k, p);
    st(fplane(fields, 5, pl), k, m.fsol);
    st(fplane(fields, 6, pl), k, m.fl);
    st(fplane(fields, 7, pl), k, rho);
    st(fplane(fields, 8, pl), k, m.E - P.latent * m.fprev - (P.cp_ref - m.cp) * P.T_melt);
    st(fplane(fields, 9, pl), k, m.mdot);
    return;
  }

  const unsigned pl = P.plane;
  void* __restrict__ B = io.B;
  float r_new, th_new;  // references the stored g and h take this step
  const unsigned rb = PopIO<PT>::kNodeRef ? sr_node(k, P.seed + dseed) : 0u;  // stochastic-rounding hash
  // The three BGK collisions, each written per pair of opposite directions
  // (i, opp(i)): an equilibrium or source term splits into a part even in
  // c_i (u.u, (c_i.u)^2, (c_i.u)(c_i.F), constants), shared by the pair, and
  // a part odd in c_i, added for i and subtracted for opp(i).  The update
  // keeps the non-equilibrium form f_i - (f_i - f_i^eq)/tau (+ source), with
  // f_i - f_i^eq formed by one fused multiply-add from the stored value, so
  // the rounding stays at the size of the small non-equilibrium part.
  // flow collision (Eq. (30)-(33))
  {
    const float itau = rcp(tauf), sf = 1.0f - 0.5f * itau;
    const float Gx = Fx + rho * fbx, Gy = Fy + rho * fby;
    // feq_i = w_i (e0 + 4.5 rho (c.u)^2 +- 3 rho (c.u)) - 3 p [i = 0],
    // F_i = w_i (s0 + 9 (c.u)(c.Ft) +- 3 (c.G))
    const float e0 = 3.0f * p - 1.5f * rho * usq, s0 = Ssrc - 3.0f * uFt;
    const float r3 = 3.0f * rho, r45 = 4.5f * rho;
    // the change -(f_i - feq_i)/tau + sf F_i is formed first (small), and
    // added to the stored value in one rounding
    float fn[9];
    {
      const float feq0 = W0 * e0 - 3.0f * p;
      fn[0] = f[0] + __builtin_fmaf(-itau, f[0] - feq0, sf * (W0 * s0));
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = pair_dir(j), o = opp(i);
      const float cx = (float)cxv(i), cy = (float)cyv(i), w = wt(i);
      const float cu = cx * ux + cy * uy, cF = cx * Ftx + cy * Fty, cG = cx * Gx + cy * Gy;
      const float ev = __builtin_fmaf(r45 * cu, cu, e0), od = r3 * cu;
      const float fe = __builtin_fmaf(9.0f * cu, cF, s0), fo = 3.0f * cG;
      const float sw = sf * w;
      const float ni = __builtin_fmaf(-w, ev + od, f[i]);  // f_i - feq_i
      const float no = __builtin_fmaf(-w, ev - od, f[o]);
      fn[i] = f[i] + __builtin_fmaf(-itau, ni, sw * (fe + fo));
      fn[o] = f[o] + __builtin_fmaf(-itau, no, sw * (fe - fo));
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if constexpr (LS > 0)
        pop_lds_st<PT, 1>(lop + (9 + i) * LS, fn[i], P, rb ^ sr_pop(9 + i));
      else
        pop_st<PT, 1, STREAM>(B, (9 + i) * pl + k, fn[i], P, rb ^ sr_pop(9 + i));
    }
  }
  // phase-field collision (Eq. (21), (24), (25), (37))
  {
    const float pux = phi * ux, puy = phi * uy;
    const float dpx = pux - phiux, dpy = puy - phiuy;
    const float ax = 3.0f * dpx + lnx, ay = 3.0f * dpy + lny;
    const float pm = phi * m.mdot;
    // the new reference is this step's phi (as stored); re-express the
    // populations and the equilibrium relative to it
    RefIO<PopIO<PT>::kNodeRef>::round(phi, m.dT, r_new, th_new);
    const float dr = m.r - r_new;  // exact for nearby floats
    const float dln = m.dl + dr;   // phi - phi_ref(new)
    // g_i - w_i phi_ref(new) = g_i(stored) + w_i dr; its equilibrium is
    // w_i (dln +- 3 phi c.u) and its source w_i (phi mdot +- c.a)
    const float itg = P.inv_tau_g, srg = P.src_g, ph3 = 3.0f * phi;
    float gn[9];
    {
      const float gi = m.g[0] + W0 * dr;
      gn[0] = gi - (gi - W0 * dln) * itg + srg * (W0 * pm);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = pair_dir(j), o = opp(i);
      const float cx = (float)cxv(i), cy = (float)cyv(i), w = wt(i);
      const float cu = cx * ux + cy * uy, ca = cx * ax + cy * ay;
      const float od = ph3 * cu, sw = srg * w;
      const float gi = __builtin_fmaf(w, dr, m.g[i]), go = __builtin_fmaf(w, dr, m.g[o]);
      const float ni = __builtin_fmaf(-w, dln + od, gi), no = __builtin_fmaf(-w, dln - od, go);
      gn[i] = __builtin_fmaf(-itg, ni, __builtin_fmaf(sw, pm + ca, gi));
      gn[o] = __builtin_fmaf(-itg, no, __builtin_fmaf(sw, pm - ca, go));
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if constexpr (LS > 0)
        pop_lds_st<PT, 0>(lop + i * LS, gn[i], P, rb ^ sr_pop(i));
      else
        pop_st<PT, 0, STREAM>(B, i * pl + k, gn[i], P, rb ^ sr_pop(i));
    }
    if constexpr (LS > 0) {
      loa[AUX_REF * LS] = r_new;
      if constexpr (PopIO<PT>::kNodeRef) loa[AUX_TH * LS] = th_new;
      loa[AUX_PHIUX * LS] = pux;
      loa[AUX_PHIUY * LS] = puy;
    } else {
      RefIO<PopIO<PT>::kNodeRef>::template store<STREAM>(io.ref_out, k, r_new, th_new);
      st<STREAM>(io.phiu_out, k, pux);
      st<STREAM>(fplane(io.phiu_out, 1, pl), k, puy);
    }
  }
  // enthalpy collision (Eq. (27)-(28)) in the shifted variables
  constexpr bool NR = PopIO<PT>::kNodeRef;
  {
    const float itau = rcp(m.kk * P.three_over_cpref + 0.5f);
    const float cpT = m.cp * T;
    const float crd = NR ? P.cp_ref * (m.dT - m.th) : P.cp_ref * m.dT;
    // node reference: move from the received reference th to this step's
    const float cmove = NR ? P.cp_ref * (m.th - th_new) : 0.0f;
    // h_i^eq = w_i (e0 + 4.5 cp T (c.u)^2 +- 3 cp T (c.u)) for i > 0
    const float e0 = crd - 1.5f * cpT * usq, c3 = 3.0f * cpT, c45 = 4.5f * cpT;
    float hn[9];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = pair_dir(j), o = opp(i);
      const float cx = (float)cxv(i), cy = (float)cyv(i), w = wt(i);
      const float cu = cx * ux + cy * uy;
      const float ev = __builtin_fmaf(c45 * cu, cu, e0), od = c3 * cu;
      const float ni = __builtin_fmaf(-w, ev + od, m.h[i]), no = __builtin_fmaf(-w, ev - od, m.h[o]);
      hn[i] = __builtin_fmaf(-itau, ni, m.h[i]);
      hn[o] = __builtin_fmaf(-itau, no, m.h[o]);
      if (NR) {
        hn[i] = __builtin_fmaf(w, cmove, hn[i]);
        hn[o] = __builtin_fmaf(w, cmove, hn[o]);
      }
    }
    float hs = 0.0f;
#pragma unroll
    for (int i = 1; i < 9; ++i) hs += m.h[i];
    // rest population: h0eq - h0 = sum_{i>0} h_i - cp_ref dT + w0 (cp_ref dT - 1.5 cp T u.u);
    // the stored value moves by that relaxation plus L (f_s^H(n) - f_s^H(n-1))
    const float d0 = (hs - crd + W0 * (crd - 1.5f * cpT * usq)) * itau;
    hn[0] = m.h[0] + d0 + P.latent * (m.fsH - m.fprev);
    if (NR) hn[0] += W0 * cmove;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if constexpr (LS > 0)
        pop_lds_st<PT, 2>(lop + (18 + i) * LS, hn[i], P, rb ^ sr_pop(18 + i));
      else
        pop_st<PT, 2, STREAM>(B, (18 + i) * pl + k, hn[i], P, rb ^ sr_pop(18 + i));
    }
  }
  if constexpr (LS > 0) {
    loa[AUX_FSH * LS] = m.fsH;
    loa[AUX_P * LS] = p;
    loa[AUX_S * LS] = Ssrc;
  } else {
    st<STREAM>(io.fsH_out, k, m.fsH);
    st<STREAM>(io.p_out, k, p);
    st<STREAM>(io.S_out, k, Ssrc);
  }
}

// Workgroup -> tile.  Workgroups are dispatched round-robin over the 8
// XCDs (block b runs on XCD b mod 8).  Mode 0 keeps that order (the XCDs
// sweep the grid together, row of tiles after row of tiles).  Mode 1 hands
// each XCD one contiguous band of `band` tiles in row-major order.  Mode 2
// hands each XCD a band of `band` tile columns, which it sweeps row by row:
// the XCDs still work on the same rows at the same time, while the x and y
// neighbours of a tile, whose halo cells it re-reads, are mostly on its own
// XCD and in its L2.  Returns ntiles or more for padding workgroups.
__device__ __forceinline__ int map_tile(int b, int mode, int band, int ntx, int ntiles) {
  if (mode == 1) return (b & 7) * band + (b >> 3);
  if (mode == 2) {
    const int i = b >> 3, col = (b & 7) * band + i % band;
    return col < ntx ? (i / band) * ntx + col : ntiles;
  }
  return b;
}

// Halo cell of a macro region LXR x LYR around an inner block of TXR x
// TYR cells (two columns and one row on each side): lane q < 2 LXR + 4 TYR
// takes the bottom row, the top row, then the side columns row by row.
template <int LXR, int LYR, int TXR>
__device__ __forceinline__ void ring_cell(int q, int& hr, int& hc) {
  if (q < LXR) {
    hr = 0;
    hc = q;
  } else if (q < 2 * LXR) {
    hr = LYR - 1;
    hc = q - LXR;
  } else {
    const int u = q - 2 * LXR;
    hr = 1 + (u >> 2);
    const int s = u & 3;
    hc = s < 2 ? s : TXR + s;
  }
}

// Fill of a W x H LDS tile in two halves, so that the loads of several
// fills are all in flight before the first LDS store (one memory round trip
// for every fill of a phase, overlapping the node pulls issued before them).
// Lane t owns column c = t % W and the rows t / W + q G (G = NT / W rows at
// a time): colv(c) is worked out once per lane, ldv(r, colv) gives the value
// (type V) of cell (c, r), stv(r, c, v) stores it.  The lanes beyond G W and
// the rows beyond H load a duplicate of the last row (in bounds, never
// stored), so the loads need no branch.
template <int W, int H, int NT, class V>
struct TileFill {
  static constexpr int G = NT / W;
  static_assert(G >= 1, "tile row wider than the workgroup");
  static constexpr int NQ = (H + G - 1) / G;
  int c, r0;
  V v[NQ];
  template <class CV, class LD>
  __device__ __forceinline__ void load(int t, CV colv, LD ldv) {
    c = t % W;
    r0 = t / W;
    const auto cv = colv(c);
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = ldv(min(r0 + q * G, H - 1), cv);
  }
  // Cells from global memory: (c, r) takes the node at column wrapx(gx0 + c)
  // and row clamp(gy0 + r, 0, ny - 1); ldk(k) loads node k.
  template <class LD>
  __device__ __forceinline__ void load_grid(int t, int gx0, int gy0, int nx, int ny, LD ldk) {
    load(
        t, [&](int cc) { return wrapx(gx0 + cc, nx); },
        [&](int r, int gx) { return ldk((unsigned)(min(max(gy0 + r, 0), ny - 1) * nx + gx)); });
  }
  template <class ST>
  __device__ __forceinline__ void store(int t, ST stv) const {
    if (t >= G * W) return;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int r = r0 + q * G;
      if ((q + 1) * G <= H || r < H) stv(r, c, v[q]);
    }
  }
};

struct RefPair {
  float r, th;
};
template <bool NR>
__device__ __forceinline__ RefPair load_ref(const void* b, unsigned k) {
  RefPair v;
  RefIO<NR>::load(b, k, v.r, v.th);
  return v;
}
struct PS {
  float p, s;
};
// q = S/3 - p of one cell (the combination whose gradient Eq. (36) takes)
__device__ __forceinline__ float q_of(PS v) { return __builtin_fmaf(v.s, 1.0f / 3.0f, -v.p); }

// Wetting ghost rows (Eq. (39)-(41)) of a macro region of width LXR: the
// row rb below grid row 0 and the row rt above grid row ny-1, where present.
template <int LXR>
__device__ __forceinline__ void ghost_rows(const KParams& P, float (*sphi)[LXR], float (*srho)[LXR],
                                           const float (*sfsH)[LXR], bool gb, int rb, bool gt, int rt, int t,
                                           int nt) {
  for (int j = t; j < 2 * LXR; j += nt) {
    const bool isb = j < LXR;
    const int c = isb ? j : j - LXR;
    if (c < 1 || c > LXR - 2) continue;
    int r, r0, r1;
    float tv;
    if (isb) {
      if (!gb) continue;
      r = rb;
      r0 = rb + 1;
      r1 = rb + 2;
      tv = P.tan_b;
    } else {
      if (!gt) continue;
      r = rt;
      r0 = rt - 1;
      r1 = rt - 2;
      tv = P.tan_t;
    }
    const float pg = wetting_ghost(sphi[r0][c - 1], sphi[r0][c], sphi[r0][c + 1], sphi[r1][c - 1],
                                   sphi[r1][c + 1], tv);
    const float pcg = clamp01(1.0f + pg);
    sphi[r][c] = pg;
    srho[r][c] = mix3(pcg * sfsH[r0][c], pcg, P.rho_s, P.rho_l, P.rho_g);
  }
}

template <int LXR>
__device__ __forceinline__ void tile_grads(const float (*sphi)[LXR], const float (*srho)[LXR],
                                           const float (*sq)[LXR], int r, int c, Grads& d) {
#define LBM_GRAD(arr, ox, oy, lap)                                                                 \
  stencil(arr[r][c], arr[r][c + 1], arr[r][c - 1], arr[r + 1][c], arr[r - 1][c], arr[r + 1][c + 1], \
          arr[r + 1][c - 1], arr[r - 1][c - 1], arr[r - 1][c + 1], ox, oy, lap)
  LBM_GRAD(sphi, d.phx, d.phy, &d.lphi);
  LBM_GRAD(srho, d.rx, d.ry, nullptr);
  LBM_GRAD(sq, d.qx, d.qy, nullptr);
#undef LBM_GRAD
}

// One TX x TY tile (origin x0, y0) of the fused step; shared by the
// single-grid kernel and the batched one.  MACRO_IN: the collide pass of
// the unfused two-kernel step; phi - 1, rho and f_s^H of every node were
// written by k_macro to the first three output-field planes, and the halo
// is read from there instead of being rebuilt from pulled populations.
template <int TX, int TY, bool FIELDS, class PT, bool MACRO_IN = false, bool STREAM = false>
__device__ __forceinline__ void step_tile(const KParams& P, const StepIO& io, int x0, int y0) {
  constexpr int NT = TX * TY;
  constexpr int LX = TX + 4, LY = TY + 2;  // LDS column c <-> x0 + c - 2, row r <-> y0 + r - 1
  constexpr int RX = LX + 2, RY = LY + 2;  // reference tile: one more cell on every side
  __shared__ float s_phi[LY][LX];  // phi - 1 (stencils are blind to the constant)
  __shared__ float s_rho[LY][LX];
  __shared__ float s_fsH[LY][LX];
  __shared__ float s_q[LY][LX];  // q = S/3 - p of the lagged p and S
  __shared__ float s_ref[RY][RX];  // phi of the previous step, reference of the stored g
  constexpr bool NR = PopIO<PT>::kNodeRef;
  __shared__ float s_th[NR ? RY : 1][NR ? RX : 1];  // reference T - T_m of the stored h

  const void* __restrict__ A = io.A;
  const int nx = P.nx, ny = P.ny;
  const int t = threadIdx.x;
  const int lx = t % TX, ly = t / TX;
  const int x = x0 + lx, y = y0 + ly;
  const int xw = wrapx(x, nx);
  const bool yin = y < ny;
  const bool active = yin && x < nx;

  // ---- phase 0: issue every global load of the tile at once ---------------
  // This node's pulled g, h, f and history values, the one halo cell this
  // lane rebuilds, and the previous-step fields with halo for LDS.  A single
  // memory round trip then feeds the whole step.
  constexpr int NRING = 2 * LX + 4 * TY;
  static_assert(NRING <= NT, "one halo cell per lane at most");
  constexpr bool RAW = !std::is_same<PT, float>::value;  // 16-bit: hold the loads packed
  Macro m, mh;
  float f[9], phiux = 0.0f, phiuy = 0.0f;
  Raw9<PT> rg, rh, rf, rgh, rhh;
  if (yin) {
    if constexpr (RAW)
      load_node_raw<PT>(A, io.fsH_in, P, xw, y, rg, rh, m.fprev);
    else
      load_node<PT>(A, io.fsH_in, P, xw, y, m);
  }
  if (active) {
    const int xm = x == 0 ? nx - 1 : x - 1;
    const int xp = x == nx - 1 ? 0 : x + 1;
    if constexpr (RAW)
      pull9_raw<1, PT>(A, P, x, y, xm, xp, rf);
    else
      pull9<1, PT>(A, P, x, y, xm, xp, f);
    phiux = ld(io.phiu_in, (unsigned)(y * nx + x));
    phiuy = ld(fplane(io.phiu_in, 1, P.plane), (unsigned)(y * nx + x));
  }
  int hr = 0, hc = 0;
  bool halo = false;
  if (!MACRO_IN && t < NRING) {
    ring_cell<LX, LY, TX>(t, hr, hc);
    const int gy = y0 + hr - 1;
    halo = gy >= 0 && gy < ny;
    if (halo) {
      if constexpr (RAW)
        load_node_raw<PT>(A, io.fsH_in, P, wrapx(x0 + hc - 2, nx), gy, rgh, rhh, mh.fprev);
      else
        load_node<PT>(A, io.fsH_in, P, wrapx(x0 + hc - 2, nx), gy, mh);
    }
  }
  // phi_ref with a two-cell halo (rows beyond a wall are never read; the
  // clamp keeps the load in bounds), and the lagged p and S with one cell
  // (rows beyond a wall copy the adjacent row)
  {
    TileFill<RX, RY, NT, RefPair> fr;
    TileFill<LX, LY, NT, PS> fp;
    fr.load_grid(t, x0 - 3, y0 - 2, nx, ny, [&](unsigned kk) { return load_ref<NR>(io.ref_in, kk); });
    fp.load_grid(t, x0 - 2, y0 - 1, nx, ny, [&](unsigned kk) { return PS{ld(io.p_in, kk), ld(io.S_in, kk)}; });
    fr.store(t, [&](int r, int c, RefPair v) {
      s_ref[r][c] = v.r;
      if constexpr (NR) s_th[r][c] = v.th;
    });
    fp.store(t, [&](int r, int c, PS v) { s_q[r][c] = q_of(v); });
  }
  if constexpr (MACRO_IN) {
    for (int j = t; j < LX * LY; j += NT) {
      const int r = j / LX, c = j - (j / LX) * LX;
      const int kk = min(max(y0 + r - 1, 0), ny - 1) * nx + wrapx(x0 + c - 2, nx);
      s_phi[r][c] = ld(io.fields, (unsigned)kk);
      s_rho[r][c] = ld(fplane(io.fields, 1, P.plane), (unsigned)kk);
      s_fsH[r][c] = ld(fplane(io.fields, 2, P.plane), (unsigned)kk);
    }
  }
  __syncthreads();

  // ---- phase 1: macroscopic quantities of time t into LDS ----------------
  if (yin) {
    if constexpr (RAW) {
      unpack9<0, PT>(rg, P, y, m.g);
      unpack9<2, PT>(rh, P, y, m.h);
    }
    const float rs = rebase_g<RX>(m.g, s_ref, P, y, lx + 2, ly + 1);
    if constexpr (NR) m.th = rebase_h<RX>(m.h, s_th, P, y, lx + 2, ly + 1);
    finish_macro<NR>(P, rs, m);
    s_phi[ly + 1][lx + 2] = (m.r - 1.0f) + m.dl;
    s_rho[ly + 1][lx + 2] = m.rho;
    s_fsH[ly + 1][lx + 2] = m.fsH;
  }
  if (halo) {
    const int yh = y0 + hr - 1;
    if constexpr (RAW) {
      unpack9<0, PT>(rgh, P, yh, mh.g);
      unpack9<2, PT>(rhh, P, yh, mh.h);
    }
    const float rs = rebase_g<RX>(mh.g, s_ref, P, yh, hc, hr);
    if constexpr (NR) mh.th = rebase_h<RX>(mh.h, s_th, P, yh, hc, hr);
    finish_macro<NR>(P, rs, mh);
    s_phi[hr][hc] = (mh.r - 1.0f) + mh.dl;
    s_rho[hr][hc] = mh.rho;
    s_fsH[hr][hc] = mh.fsH;
  }
  __syncthreads();

  // ---- wall ghost rows: wetting condition, Eq. (39)-(41) -----------------
  const bool has_bot = (y0 == 0), has_top = (ny <= y0 + TY);
  if (has_bot || has_top) {
    ghost_rows<LX>(P, s_phi, s_rho, s_fsH, has_bot, 0, has_top, ny - y0 + 1, t, NT);
    __syncthreads();
  }
  if (!active) return;  // no barrier below

  // ---- phase 2: stencils (Eq. (38)), forces, flow macros, collisions -----
  Grads d;
  tile_grads<LX>(s_phi, s_rho, s_q, ly + 1, lx + 2, d);
  if constexpr (RAW) unpack9<1, PT>(rf, P, y, f);
  update_node<FIELDS, PT, STREAM>(P, io, m, f, phiux, phiuy, d, (unsigned)(y * nx + x));
}

template <int TX, int TY, bool FIELDS, class PT, bool STREAM = false>
__global__ __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(6))) void k_step(
    KParams P, StepIO io, int ntx, int ntiles, int band, int mode) {
  const int tile = map_tile(blockIdx.x, mode, band, ntx, ntiles);
  if (tile >= ntiles) return;  // whole workgroup leaves before any barrier
  step_tile<TX, TY, FIELDS, PT, false, STREAM>(P, io, (tile % ntx) * TX, (tile / ntx) * TY);
}

// ---- many steps per launch (persistent grid) -----------------------------
// Every step pulls the halo its neighbours wrote in the step before, so one
// launch over several steps needs a grid-wide barrier between them.  It is
// only safe when every workgroup is resident at once, which a cooperative
// launch guarantees (the runtime refuses a grid that does not fit).
//
// Barrier words (64-bit, zeroed before the launch): bar[0] arrivals at the
// flat barrier, bar[1] the time-out flag, bar[2] XCD arrivals of the per-XCD
// barrier, bar[3 + x] arrivals of workgroups on XCD x, bar[11 + x] the
// number of workgroups on XCD x.  Every wait polls with a bound of `limit`
// wall-clock ticks; a wait that exceeds it sets bar[1], no workgroup waits
// once it is set, and the kernel stops stepping, so every wave reaches the
// end whatever happens and the host reports the flag.
enum { BAR_FLAT = 0, BAR_FLAG = 1, BAR_XCD = 2, BAR_ARRIVE = 3, BAR_COUNT = 11 };
static_assert(BAR_COUNT + 8 == NPERSIST_WORDS, "barrier words");

__device__ __forceinline__ bool spin_until(unsigned long long* ctr, unsigned long long target,
                                           unsigned long long* flag, unsigned long long limit) {
  const unsigned long long t0 = wall_clock64();
  while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull) return false;
    if (wall_clock64() - t0 > limit) {
      __hip_atomic_store(flag, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// Flat barrier: barrier k (from 1) is complete once bar[0] reaches
// k * gridDim.x.  Each wave first waits for its own stores; thread 0 then
// publishes the workgroup's stores at agent scope (the 8 XCDs' L2s are not
// coherent: release writes the dirty lines of its XCD's L2 back) before it
// arrives, and after the wait acquires the others' (L2 invalidate).
__device__ __forceinline__ bool grid_barrier(unsigned long long* bar, unsigned long long target,
                                             unsigned long long limit) {
  __shared__ unsigned s_go;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_s_waitcnt(0);  // the write-back has completed before the arrival counts
    __hip_atomic_fetch_add(bar + BAR_FLAT, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool go = spin_until(bar + BAR_FLAT, target, bar + BAR_FLAG, limit);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
    s_go = go;
  }
  __syncthreads();
  return s_go != 0;
}

// Per-XCD barrier.  An XCD's L2 is shared by all of its CUs, so one
// write-back publishes the stores of every workgroup on it once they have
// reached it: each wave waits for its stores (they are then in its XCD's
// L2), thread 0 counts the workgroup's arrival on its XCD, and the
// workgroup that completes that count writes the L2 back and arrives for
// the whole XCD at bar[2].  Barrier k is complete once bar[2] reaches
// k * (XCDs with workgroups); every workgroup then invalidates as above.
// One write-back per XCD and step instead of one per workgroup.
struct XcdPlace {
  unsigned xcd;              // XCC_ID of the workgroup's XCD
  unsigned long long nwg;    // workgroups on that XCD
  unsigned long long nxcd;   // XCDs with workgroups
};

// Where each workgroup runs, counted once per launch behind a flat barrier.
__device__ __forceinline__ bool xcd_census(unsigned long long* bar, unsigned long long limit, XcdPlace& pl) {
  __shared__ unsigned s_xcd;
  __shared__ unsigned long long s_nwg, s_nxcd;
  if (threadIdx.x == 0) {
    // hardware register XCC_ID (hwreg 20), bits 3:0
    s_xcd = (unsigned)__builtin_amdgcn_s_getreg((3 << 11) | 20) & 7u;
    __hip_atomic_fetch_add(bar + BAR_COUNT + s_xcd, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (!grid_barrier(bar, gridDim.x, limit)) return false;
  if (threadIdx.x == 0) {
    unsigned long long n = 0;
    for (int x = 0; x < 8; ++x)
      n += __hip_atomic_load(bar + BAR_COUNT + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1ull : 0ull;
    s_nxcd = n;
    s_nwg = __hip_atomic_load(bar + BAR_COUNT + s_xcd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  pl = XcdPlace{s_xcd, s_nwg, s_nxcd};
  return true;
}

__device__ __forceinline__ bool xcd_barrier(unsigned long long* bar, unsigned k, const XcdPlace& pl,
                                            unsigned long long limit) {
  __shared__ unsigned s_go;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long before =
        __hip_atomic_fetch_add(bar + BAR_ARRIVE + pl.xcd, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (before + 1 == (unsigned long long)k * pl.nwg) {  // the XCD's last arrival of barrier k
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __builtin_amdgcn_s_waitcnt(0);
      __hip_atomic_fetch_add(bar + BAR_XCD, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const bool go = spin_until(bar + BAR_XCD, (unsigned long long)k * pl.nxcd, bar + BAR_FLAG, limit);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
    s_go = go;
  }
  __syncthreads();
  return s_go != 0;
}

// The buffers of the step after io's: its outputs become the inputs.
__device__ __forceinline__ StepIO next_io(const StepIO& io) {
  return StepIO{io.B, const_cast<void*>(io.A), io.phiu_out, const_cast<float*>(io.phiu_in),
                io.ref_out, const_cast<void*>(io.ref_in), io.fsH_out, const_cast<float*>(io.fsH_in),
                io.p_out, const_cast<float*>(io.p_in), io.S_out, const_cast<float*>(io.S_in), io.fields};
}

// nsteps single steps in one launch from the buffers io: step s reads what
// step s - 1 wrote and seeds the stochastic rounding with P.seed + s,
// exactly as nsteps k_step launches would.  Workgroup b takes the tiles
// k_step's workgroups b, b + gridDim.x, ... would take; gridDim.x is a
// multiple of 8 (or the whole launch), so each tile stays on the XCD the
// tile order gives it.  per_xcd selects the barrier between steps.
template <int TX, int TY, class PT, bool STREAM>
__global__ __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(4))) void k_persist(
    KParams P, StepIO io, int nsteps, int ntx, int ntiles, int band, int mode, int vgrid, int per_xcd,
    unsigned long long* bar, unsigned long long limit) {
  const unsigned seed0 = P.seed;
  XcdPlace pl{0u, 0ull, 0ull};
  if (per_xcd && nsteps > 1 && !xcd_census(bar, limit, pl)) return;
  for (int s = 0; s < nsteps; ++s, io = next_io(io)) {
    P.seed = seed0 + (unsigned)s;
    for (int v = blockIdx.x; v < vgrid; v += gridDim.x) {
      const int tile = map_tile(v, mode, band, ntx, ntiles);  // uniform over the workgroup
      if (tile < ntiles) step_tile<TX, TY, false, PT, false, STREAM>(P, io, (tile % ntx) * TX, (tile / ntx) * TY);
      __syncthreads();  // the next tile refills the LDS
    }
    if (s + 1 < nsteps) {
      const bool go = per_xcd ? xcd_barrier(bar, (unsigned)(s + 1), pl, limit)
                              : grid_barrier(bar, (unsigned long long)(s + 1) * gridDim.x, limit);
      if (!go) return;
    }
  }
}

__global__ void k_zero_words(unsigned long long* w, int n) {
  if ((int)threadIdx.x < n) w[threadIdx.x] = 0ull;
}

// ---- two steps per launch (FP32) -----------------------------------------
// The second step of a TX x TY tile reads first-step results on the tile
// plus 3 columns and 2 rows on each side (its halo macros pull from one cell
// further, and their reference phi one more).  The workgroup first runs the
// step on that region E from global memory, keeping its results in LDS, then
// runs the second step on the tile from LDS and writes it out: one read and
// one write of the state per two steps, for ~1.3x the arithmetic (the
// overlap of neighbouring regions is computed by both tiles).  Every node
// goes through the same macro and update code as in k_step, so the results
// are bitwise those of two single steps.

// Pull-stream one lattice into E cell (ex, ey) of grid row y from
// first-step results in LDS (plane j at ep[j * ES], the storage type),
// converted to FP32 with the lattice's load scale, and with pull9's wall
// rules.
template <int LAT, int EX, int ES, class PT>
__device__ __forceinline__ void pull9_lds(const PT* __restrict__ ep, const KParams& P, int ex, int ey, int y,
                                          float q[9]) {
  const bool bot = (y == 0), top = (y == P.ny - 1);
  const int e = ey * EX + ex;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int cy = cyv(i), cx = cxv(i);
    const bool wall = (cy > 0 && bot) || (cy < 0 && top);
    const int idx = wall ? (LAT * 9 + opp(i)) * ES + e : (LAT * 9 + i) * ES + e - cy * EX - cx;
    float v = (float)ep[idx];
    if constexpr (PopIO<PT>::kScaled) v *= P.sc_ld[LAT];
    if (LAT == 2 && cy > 0) v = bot ? (P.hwall[i] - v) : v;
    q[i] = v;
  }
}

template <int EX, int ES, class PT>
__device__ __forceinline__ void load_node_lds(const PT* __restrict__ ep, const float* __restrict__ ea,
                                              const KParams& P, int ex, int ey, int y, Macro& m) {
  pull9_lds<0, EX, ES>(ep, P, ex, ey, y, m.g);
  pull9_lds<2, EX, ES>(ep, P, ex, ey, y, m.h);
  m.fprev = ea[AUX_FSH * ES + ey * EX + ex];
}

template <int TX, int TY, bool STREAM = false>
__global__ __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(2))) void k_step2(
    KParams P, StepIO io, int ntx, int ntiles, int band, int mode) {
  constexpr int NT = TX * TY;
  constexpr int EX = TX + 6, EY = TY + 4, ES = EX * EY;  // E: cell (ex, ey) <-> (x0 - 3 + ex, y0 - 2 + ey)
  // first step: macro cells (c, r) <-> (x0 - 5 + c, y0 - 3 + r); reference tile one more cell around
  constexpr int LXA = EX + 4, LYA = EY + 2, RXA = LXA + 2, RYA = LYA + 2;
  constexpr int NRA = 2 * LXA + 4 * EY;  // macro cells of the first step outside E
  // second step: the single-step layout, macro cells (c, r) <-> (x0 - 2 + c, y0 - 1 + r)
  constexpr int LX = TX + 4, LY = TY + 2;
  constexpr int NRB = 2 * LX + 4 * TY;
  static_assert(ES <= 2 * NT && NRA <= NT && NRB <= NT, "lane assignment");
  static_assert(EX == LX + 2 && EY == LY + 2, "E doubles as the second step's reference tile");
  __shared__ float s_ep[27 * ES];  // first-step populations
  __shared__ float s_ea[6 * ES];   // and references, (phi u), f_s^H, p, S
  __shared__ float s_work[4 * LYA * LXA + RYA * RXA];

  const int tile = map_tile(blockIdx.x, mode, band, ntx, ntiles);
  if (tile >= ntiles) return;  // whole workgroup leaves before any barrier
  const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
  const void* __restrict__ A = io.A;
  const int nx = P.nx, ny = P.ny;
  const int t = threadIdx.x;

  // ===== step n -> n+1 on E, from global memory, results to LDS ===========
  {
    float(*sphi)[LXA] = reinterpret_cast<float(*)[LXA]>(s_work);
    float(*srho)[LXA] = sphi + LYA;
    float(*sfsH)[LXA] = srho + LYA;
    float(*sq)[LXA] = sfsH + LYA;  // q = S/3 - p
    float(*sref)[RXA] = reinterpret_cast<float(*)[RXA]>(s_work + 4 * LYA * LXA);
    const int xa0 = x0 - 5, ya0 = y0 - 3;

    // phase 0: every global load at once (two E cells per lane at most,
    // one macro cell outside E, the reference tile and lagged p, S)
    Macro m[2], mh;
    float f[2][9], pux[2] = {0.0f, 0.0f}, puy[2] = {0.0f, 0.0f};
    bool on[2];
    int ex[2], ey[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int e = t + s * NT;
      ex[s] = e % EX;
      ey[s] = e / EX;
      const int y = y0 - 2 + ey[s];
      on[s] = e < ES && y >= 0 && y < ny;
      if (on[s]) {
        const int x = wrapx(x0 - 3 + ex[s], nx);
        load_node<float>(A, io.fsH_in, P, x, y, m[s]);
        const int xm = x == 0 ? nx - 1 : x - 1;
        const int xp = x == nx - 1 ? 0 : x + 1;
        pull9<1, float>(A, P, x, y, xm, xp, f[s]);
        pux[s] = ld(io.phiu_in, (unsigned)(y * nx + x));
        puy[s] = ld(fplane(io.phiu_in, 1, P.plane), (unsigned)(y * nx + x));
      }
    }
    int hr = 0, hc = 0;
    bool halo = false;
    if (t < NRA) {
      ring_cell<LXA, LYA, EX>(t, hr, hc);
      const int gy = ya0 + hr;
      halo = gy >= 0 && gy < ny;
      if (halo) load_node<float>(A, io.fsH_in, P, wrapx(xa0 + hc, nx), gy, mh);
    }
    {
      TileFill<RXA, RYA, NT, float> fr;
      TileFill<LXA, LYA, NT, PS> fp;
      fr.load_grid(t, xa0 - 1, ya0 - 1, nx, ny, [&](unsigned kk) { return ld((const float*)io.ref_in, kk); });
      fp.load_grid(t, xa0, ya0, nx, ny, [&](unsigned kk) { return PS{ld(io.p_in, kk), ld(io.S_in, kk)}; });
      fr.store(t, [&](int r, int c, float v) { sref[r][c] = v; });
      fp.store(t, [&](int r, int c, PS v) {
        sq[r][c] = q_of(v);
      });
    }
    __syncthreads();

    // phase 1: macros of time n
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (!on[s]) continue;
      const int c = ex[s] + 2, r = ey[s] + 1;
      const float rs = rebase_g<RXA>(m[s].g, sref, P, ya0 + r, c, r);
      finish_macro<false>(P, rs, m[s]);
      sphi[r][c] = (m[s].r - 1.0f) + m[s].dl;
      srho[r][c] = m[s].rho;
      sfsH[r][c] = m[s].fsH;
    }
    if (halo) {
      const float rs = rebase_g<RXA>(mh.g, sref, P, ya0 + hr, hc, hr);
      finish_macro<false>(P, rs, mh);
      sphi[hr][hc] = (mh.r - 1.0f) + mh.dl;
      srho[hr][hc] = mh.rho;
      sfsH[hr][hc] = mh.fsH;
    }
    __syncthreads();

    const int rb = -1 - ya0, rt = ny - ya0;  // rows of y = -1 and y = ny
    const bool gb = rb >= 0 && rb < LYA, gt = rt >= 0 && rt < LYA;
    if (gb || gt) {
      ghost_rows<LXA>(P, sphi, srho, sfsH, gb, rb, gt, rt, t, NT);
      __syncthreads();
    }

    // phase 2: stencils, collisions; results of time n+1 to LDS
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (!on[s]) continue;
      Grads d;
      tile_grads<LXA>(sphi, srho, sq, ey[s] + 1, ex[s] + 2, d);
      const int e = ey[s] * EX + ex[s];
      update_node<false, float, false, ES>(P, io, m[s], f[s], pux[s], puy[s], d, 0u, s_ep + e, s_ea + e);
    }
    __syncthreads();
  }

  // ===== step n+1 -> n+2 on the tile, from LDS, results to global =========
  float(*sphi)[LX] = reinterpret_cast<float(*)[LX]>(s_work);
  float(*srho)[LX] = sphi + LY;
  float(*sfsH)[LX] = srho + LY;
  float(*sq)[LX] = sfsH + LY;  // q = S/3 - p
  const float(*sref)[EX] = reinterpret_cast<const float(*)[EX]>(s_ea + AUX_REF * ES);
  const int lx = t % TX, ly = t / TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool yin = y < ny;
  const bool active = yin && x < nx;
  Macro m, mh;
  float f[9], phiux = 0.0f, phiuy = 0.0f;
  if (yin) load_node_lds<EX, ES>(s_ep, s_ea, P, lx + 3, ly + 2, y, m);
  if (active) {
    const int e = (ly + 2) * EX + lx + 3;
    pull9_lds<1, EX, ES>(s_ep, P, lx + 3, ly + 2, y, f);
    phiux = s_ea[AUX_PHIUX * ES + e];
    phiuy = s_ea[AUX_PHIUY * ES + e];
  }
  int hr = 0, hc = 0;
  bool halo = false;
  if (t < NRB) {
    ring_cell<LX, LY, TX>(t, hr, hc);
    const int gy = y0 + hr - 1;
    halo = gy >= 0 && gy < ny;
    if (halo) load_node_lds<EX, ES>(s_ep, s_ea, P, hc + 1, hr + 1, gy, mh);
  }
  {
    TileFill<LX, LY, NT, PS> fp;
    fp.load(
        t, [](int cc) { return cc; },
        [&](int rr, int cc) {
          const int e = (min(max(y0 + rr - 1, 0), ny - 1) - y0 + 2) * EX + cc + 1;
          return PS{s_ea[AUX_P * ES + e], s_ea[AUX_S * ES + e]};
        });
    fp.store(t, [&](int rr, int cc, PS v) {
      sq[rr][cc] = q_of(v);
    });
  }
  if (yin) {
    const float rs = rebase_g<EX>(m.g, sref, P, y, lx + 2, ly + 1);
    finish_macro<false>(P, rs, m);
    sphi[ly + 1][lx + 2] = (m.r - 1.0f) + m.dl;
    srho[ly + 1][lx + 2] = m.rho;
    sfsH[ly + 1][lx + 2] = m.fsH;
  }
  if (halo) {
    const float rs = rebase_g<EX>(mh.g, sref, P, y0 + hr - 1, hc, hr);
    finish_macro<false>(P, rs, mh);
    sphi[hr][hc] = (mh.r - 1.0f) + mh.dl;
    srho[hr][hc] = mh.rho;
    sfsH[hr][hc] = mh.fsH;
  }
  __syncthreads();
  const bool has_bot = (y0 == 0), has_top = (ny <= y0 + TY);
  if (has_bot || has_top) {
    ghost_rows<LX>(P, sphi, srho, sfsH, has_bot, 0, has_top, ny - y0 + 1, t, NT);
    __syncthreads();
  }
  if (!active) return;  // no barrier below
  Grads d;
  tile_grads<LX>(sphi, srho, sq, ly + 1, lx + 2, d);
  update_node<false, float, STREAM>(P, io, m, f, phiux, phiuy, d, (unsigned)(y * nx + x));
}

// The same two steps with more lanes than tile nodes: every lane owns at
// most one cell of each step (an E cell or a cell of the first step's macro
// ring; a tile node or a halo cell of the second).  NT lanes: 2 TX TY for
// 32x16 tiles (one workgroup, 4 waves per SIMD), 3 TX TY for 32x8 tiles
// (two workgroups, 6 waves per SIMD).  Any storage format: the first
// step's populations stay in LDS as stored (16-bit values rounded exactly
// as a single step rounds them, with that step's random words), so the
// second step reads what it would read from memory, and both steps are
// bitwise those of single steps.  The first step runs with the step number
// P.seed, the second with P.seed + 1.  Shared by the single-grid and the
// batched kernels.
template <int TX, int TY, int NT, class PT, bool STREAM>
__device__ __forceinline__ void step2w_tile(const KParams& P, const StepIO& io, int x0, int y0) {
  constexpr int NTILE = TX * TY;
  constexpr int EX = TX + 6, EY = TY + 4, ES = EX * EY;  // E: cell (ex, ey) <-> (x0 - 3 + ex, y0 - 2 + ey)
  // first step: macro cells (c, r) <-> (x0 - 5 + c, y0 - 3 + r); reference tiles one more cell around
  constexpr int LXA = EX + 4, LYA = EY + 2, RXA = LXA + 2, RYA = LYA + 2;
  constexpr int NRA = 2 * LXA + 4 * EY;  // macro cells of the first step outside E
  // second step: the single-step layout, macro cells (c, r) <-> (x0 - 2 + c, y0 - 1 + r)
  constexpr int LX = TX + 4, LY = TY + 2;
  constexpr int NRB = 2 * LX + 4 * TY;
  constexpr bool NR = PopIO<PT>::kNodeRef;
  static_assert(ES + NRA <= NT && NTILE + NRB <= NT, "one cell per lane in each step");
  static_assert(EX == LX + 2 && EY == LY + 2, "E doubles as the second step's reference tile");
  static_assert((27 * ES * sizeof(PT)) % 4 == 0, "FP32 planes after the populations");
  __shared__ PT s_ep[27 * ES];                 // first-step populations, as stored
  __shared__ float s_ea[aux_planes<PT>() * ES];  // references, (phi u), f_s^H, p, S
  __shared__ float s_work[4 * LYA * LXA + (NR ? 2 : 1) * RYA * RXA];

  const void* __restrict__ A = io.A;
  const int nx = P.nx, ny = P.ny;
  const int t = threadIdx.x;

  // ===== step n -> n+1 on E, from global memory, results to LDS ===========
  {
    float(*sphi)[LXA] = reinterpret_cast<float(*)[LXA]>(s_work);
    float(*srho)[LXA] = sphi + LYA;
    float(*sfsH)[LXA] = srho + LYA;
    float(*sq)[LXA] = sfsH + LYA;  // q = S/3 - p
    float(*sref)[RXA] = reinterpret_cast<float(*)[RXA]>(s_work + 4 * LYA * LXA);
    float(*sth)[RXA] = sref + RYA;  // node-reference storage only
    const int xa0 = x0 - 5, ya0 = y0 - 3;

    Macro m;
    float f[9], pux = 0.0f, puy = 0.0f;
    int c = 0, r = 0;   // this lane's macro cell of the first step
    bool on = false;    // an E cell inside the grid: macros and update
    bool ring = false;  // a macro-ring cell inside the grid: macros only
    unsigned k = 0;     // its node index
    if (t < ES) {
      c = t % EX + 2;
      r = t / EX + 1;
      const int y = ya0 + r;
      on = y >= 0 && y < ny;
      if (on) {
        const int x = wrapx(xa0 + c, nx);
        k = (unsigned)(y * nx + x);
        load_node<PT>(A, io.fsH_in, P, x, y, m);
        const int xm = x == 0 ? nx - 1 : x - 1;
        const int xp = x == nx - 1 ? 0 : x + 1;
        pull9<1, PT>(A, P, x, y, xm, xp, f);
        pux = ld(io.phiu_in, k);
        puy = ld(fplane(io.phiu_in, 1, P.plane), k);
      }
    } else if (t - ES < NRA) {
      ring_cell<LXA, LYA, EX>(t - ES, r, c);
      const int gy = ya0 + r;
      ring = gy >= 0 && gy < ny;
      if (ring) load_node<PT>(A, io.fsH_in, P, wrapx(xa0 + c, nx), gy, m);
    }
    {
      TileFill<RXA, RYA, NT, RefPair> fr;
      TileFill<LXA, LYA, NT, PS> fp;
      fr.load_grid(t, xa0 - 1, ya0 - 1, nx, ny, [&](unsigned kk) { return load_ref<NR>(io.ref_in, kk); });
      fp.load_grid(t, xa0, ya0, nx, ny, [&](unsigned kk) { return PS{ld(io.p_in, kk), ld(io.S_in, kk)}; });
      fr.store(t, [&](int rr, int cc, RefPair v) {
        sref[rr][cc] = v.r;
        if constexpr (NR) sth[rr][cc] = v.th;
      });
      fp.store(t, [&](int rr, int cc, PS v) {
        sq[rr][cc] = q_of(v);
      });
    }
    __syncthreads();

    if (on || ring) {
      const float rs = rebase_g<RXA>(m.g, sref, P, ya0 + r, c, r);
      if constexpr (NR) m.th = rebase_h<RXA>(m.h, sth, P, ya0 + r, c, r);
      finish_macro<NR>(P, rs, m);
      sphi[r][c] = (m.r - 1.0f) + m.dl;
      srho[r][c] = m.rho;
      sfsH[r][c] = m.fsH;
    }
    __syncthreads();

    const int rb = -1 - ya0, rt = ny - ya0;  // rows of y = -1 and y = ny
    const bool gb = rb >= 0 && rb < LYA, gt = rt >= 0 && rt < LYA;
    if (gb || gt) {
      ghost_rows<LXA>(P, sphi, srho, sfsH, gb, rb, gt, rt, t, NT);
      __syncthreads();
    }

    if (on) {
      Grads d;
      tile_grads<LXA>(sphi, srho, sq, r, c, d);
      const int e = (r - 1) * EX + (c - 2);
      update_node<false, PT, false, ES>(P, io, m, f, pux, puy, d, k, s_ep + e, s_ea + e, 0u);
    }
    __syncthreads();
  }

  // ===== step n+1 -> n+2 on the tile, from LDS, results to global =========
  float(*sphi)[LX] = reinterpret_cast<float(*)[LX]>(s_work);
  float(*srho)[LX] = sphi + LY;
  float(*sfsH)[LX] = srho + LY;
  float(*sq)[LX] = sfsH + LY;  // q = S/3 - p
  const float(*sref)[EX] = reinterpret_cast<const float(*)[EX]>(s_ea + AUX_REF * ES);
  const float(*sth)[EX] = reinterpret_cast<const float(*)[EX]>(s_ea + AUX_TH * ES);  // node-reference storage
  Macro m;
  float f[9], phiux = 0.0f, phiuy = 0.0f;
  int c = 0, r = 0, y = 0;  // this lane's macro cell of the second step and its grid row
  bool mac = false, active = false;
  if (t < NTILE) {
    const int lx = t % TX, ly = t / TX;
    c = lx + 2;
    r = ly + 1;
    y = y0 + ly;
    mac = y < ny;
    active = mac && x0 + lx < nx;
  } else if (t - NTILE < NRB) {
    ring_cell<LX, LY, TX>(t - NTILE, r, c);
    y = y0 + r - 1;
    mac = y >= 0 && y < ny;
  }
  if (mac) load_node_lds<EX, ES>(s_ep, s_ea, P, c + 1, r + 1, y, m);
  if (active) {
    const int e = (r + 1) * EX + c + 1;
    pull9_lds<1, EX, ES>(s_ep, P, c + 1, r + 1, y, f);
    phiux = s_ea[AUX_PHIUX * ES + e];
    phiuy = s_ea[AUX_PHIUY * ES + e];
  }
  {
    TileFill<LX, LY, NT, PS> fp;
    fp.load(
        t, [](int cc) { return cc; },
        [&](int rr, int cc) {
          const int e = (min(max(y0 + rr - 1, 0), ny - 1) - y0 + 2) * EX + cc + 1;
          return PS{s_ea[AUX_P * ES + e], s_ea[AUX_S * ES + e]};
        });
    fp.store(t, [&](int rr, int cc, PS v) {
      sq[rr][cc] = q_of(v);
    });
  }
  if (mac) {
    const float rs = rebase_g<EX>(m.g, sref, P, y, c, r);
    if constexpr (NR) m.th = rebase_h<EX>(m.h, sth, P, y, c, r);
    finish_macro<NR>(P, rs, m);
    sphi[r][c] = (m.r - 1.0f) + m.dl;
    srho[r][c] = m.rho;
    sfsH[r][c] = m.fsH;
  }
  __syncthreads();
  const bool has_bot = (y0 == 0), has_top = (ny <= y0 + TY);
  if (has_bot || has_top) {
    ghost_rows<LX>(P, sphi, srho, sfsH, has_bot, 0, has_top, ny - y0 + 1, t, NT);
    __syncthreads();
  }
  if (!active) return;  // no barrier below
  Grads d;
  tile_grads<LX>(sphi, srho, sq, r, c, d);
  update_node<false, PT, STREAM>(P, io, m, f, phiux, phiuy, d, (unsigned)(y * nx + x0 + c - 2), nullptr, nullptr,
                                 1u);
}

template <int TX, int TY, int NT, class PT, bool STREAM = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT >= 1024 ? 4 : 6))) void k_step2w(
    KParams P, StepIO io, int ntx, int ntiles, int band, int mode) {
  const int tile = map_tile(blockIdx.x, mode, band, ntx, ntiles);
  if (tile >= ntiles) return;  // whole workgroup leaves before any barrier
  step2w_tile<TX, TY, NT, PT, STREAM>(P, io, (tile % ntx) * TX, (tile / ntx) * TY);
}

// Unfused two-kernel step, kept to measure what fusion saves.  Pass 1
// (k_macro) pulls g and h and writes phi - 1, rho and f_s^H of time t of
// every node to the first three output-field planes; pass 2 (k_collide)
// pulls all 27 populations again, rebuilds its own node's macros and takes
// the halo values from those planes.  The arithmetic is the fused kernel's,
// so the results are bitwise equal.
template <int TX, int TY, class PT>
__global__ __launch_bounds__(TX* TY) void k_macro(KParams P, StepIO io, int ntx, int ntiles, int band, int mode) {
  const int tile = map_tile(blockIdx.x, mode, band, ntx, ntiles);
  if (tile >= ntiles) return;
  constexpr int RX = TX + 2, RR = TY + 2;  // reference tile: row q <-> y0 + q - 1, column c <-> x0 + c - 1
  constexpr bool NR = PopIO<PT>::kNodeRef;
  __shared__ float s_ref[RR][RX];
  __shared__ float s_th[NR ? RR : 1][NR ? RX : 1];
  const int nx = P.nx, ny = P.ny;
  const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
  const int t = threadIdx.x, lx = t % TX, ly = t / TX;
  const int x = x0 + lx, y = y0 + ly;
  const bool active = y < ny && x < nx;
  Macro m;
  if (active) load_node<PT>(io.A, io.fsH_in, P, x, y, m);
  {
    TileFill<RX, RR, TX * TY, RefPair> fr;
    fr.load_grid(t, x0 - 1, y0 - 1, nx, ny, [&](unsigned kk) { return load_ref<NR>(io.ref_in, kk); });
    fr.store(t, [&](int q, int c, RefPair v) {
      s_ref[q][c] = v.r;
      if constexpr (NR) s_th[q][c] = v.th;
    });
  }
  __syncthreads();
  if (!active) return;
  // rebase_* read cell (c, r) at [r + 1][c + 1]: the node is cell (lx, ly)
  const float rs = rebase_g<RX>(m.g, s_ref, P, y, lx, ly);
  if constexpr (NR) m.th = rebase_h<RX>(m.h, s_th, P, y, lx, ly);
  finish_macro<NR>(P, rs, m);
  const unsigned k = (unsigned)(y * nx + x);
  io.fields[k] = (m.r - 1.0f) + m.dl;
  io.fields[P.plane + k] = m.rho;
  io.fields[2u * P.plane + k] = m.fsH;
}

template <int TX, int TY, class PT>
__global__ __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(6))) void k_collide(
    KParams P, StepIO io, int ntx, int ntiles, int band, int mode) {
  const int tile = map_tile(blockIdx.x, mode, band, ntx, ntiles);
  if (tile >= ntiles) return;
  step_tile<TX, TY, false, PT, true>(P, io, (tile % ntx) * TX, (tile / ntx) * TY);
}

__device__ __forceinline__ StepIO io_of(char* base, const StepOff& o) {
  return StepIO{base + o.A, base + o.B, (const float*)(base + o.phiu_in), (float*)(base + o.phiu_out),
                base + o.ref_in, base + o.ref_out, (const float*)(base + o.fsH_in), (float*)(base + o.fsH_out),
                (const float*)(base + o.p_in), (float*)(base + o.p_out), (const float*)(base + o.S_in),
                (float*)(base + o.S_out), (float*)(base + o.fields)};
}

// Many grids in one launch: workgroup b updates tile tmap[b] & 0xffff of the
// grid in slot tmap[b] >> 16 (entries of ~0u are padding), with that slot's
// constants and its buffer set for parity `par`.
template <int TX, int TY, bool FIELDS, class PT, bool STREAM = false>
__global__ __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(6))) void k_batch(
    char* __restrict__ base, const KParams* __restrict__ ptab, const StepOff* __restrict__ otab,
    const unsigned* __restrict__ tmap, const unsigned* __restrict__ steps, int s) {
  const unsigned e = tmap[blockIdx.x];
  if (e == ~0u) return;
  const int slot = (int)(e >> 16), tile = (int)(e & 0xffffu);
  const int par = s & 1;
  KParams P = ptab[slot];
  P.seed = steps[slot] + (unsigned)s;  // the grid's own step number
  const StepIO io = io_of(base, otab[2 * slot + par]);
  const int ntx = (P.nx + TX - 1) / TX;
  step_tile<TX, TY, FIELDS, PT, false, STREAM>(P, io, (tile % ntx) * TX, (tile / ntx) * TY);
}

// Two steps s, s + 1 (s even) of many grids in one launch, on the tiles of
// step2w_tile: workgroup b runs tile tmap[b] of slot tmap[b] >> 16.  The
// launch reads buffer set par = (s / 2) & 1 and writes the other one, so an
// interval whose step count is a multiple of 4 ends in the buffer a run of
// single steps ends in.
template <int TX, int TY, int NT, class PT, bool STREAM = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT >= 1024 ? 4 : 6))) void k_batch2w(
    char* __restrict__ base, const KParams* __restrict__ ptab, const StepOff* __restrict__ otab,
    const unsigned* __restrict__ tmap, const unsigned* __restrict__ steps, int s) {
  const unsigned e = tmap[blockIdx.x];
  if (e == ~0u) return;
  const int slot = (int)(e >> 16), tile = (int)(e & 0xffffu);
  const int par = (s >> 1) & 1;
  KParams P = ptab[slot];
  P.seed = steps[slot] + (unsigned)s;  // the grid's own step number (the second step adds one)
  const StepIO io = io_of(base, otab[2 * slot + par]);
  const int ntx = (P.nx + TX - 1) / TX;
  step2w_tile<TX, TY, NT, PT, STREAM>(P, io, (tile % ntx) * TX, (tile / ntx) * TY);
}

// nsteps single steps of many grids in one cooperative launch: the tiles of
// the map tmap (as k_batch takes them, workgroup b the entries b,
// b + gridDim.x, ...; gridDim.x a multiple of 8 keeps each on its XCD),
// step s reading buffer set s & 1 of every slot, with the barrier of
// k_persist between steps.
template <class PT, bool STREAM>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_persist(
    char* __restrict__ base, const KParams* __restrict__ ptab, const StepOff* __restrict__ otab,
    const unsigned* __restrict__ tmap, const unsigned* __restrict__ steps, int nblocks, int nsteps, int per_xcd,
    unsigned long long* bar, unsigned long long limit) {
  constexpr int TX = 64, TY = 8;
  XcdPlace pl{0u, 0ull, 0ull};
  if (per_xcd && nsteps > 1 && !xcd_census(bar, limit, pl)) return;
  for (int s = 0; s < nsteps; ++s) {
    for (int v = blockIdx.x; v < nblocks; v += gridDim.x) {
      const unsigned e = tmap[v];  // uniform over the workgroup
      if (e != ~0u) {
        const int slot = (int)(e >> 16), tile = (int)(e & 0xffffu);
        KParams P = ptab[slot];
        P.seed = steps[slot] + (unsigned)s;  // the grid's own step number
        const StepIO io = io_of(base, otab[2 * slot + (s & 1)]);
        const int ntx = (P.nx + TX - 1) / TX;
        step_tile<TX, TY, false, PT, false, STREAM>(P, io, (tile % ntx) * TX, (tile / ntx) * TY);
      }
      __syncthreads();  // the next tile refills the LDS
    }
    if (s + 1 < nsteps) {
      const bool go = per_xcd ? xcd_barrier(bar, (unsigned)(s + 1), pl, limit)
                              : grid_barrier(bar, (unsigned long long)(s + 1) * gridDim.x, limit);
      if (!go) return;
    }
  }
}

// Initial state (no time-stepping yet): u = 0, p = 0, liquid fraction 1,
// each lattice at its equilibrium; computed in FP64 and rounded once.
template <class PT>
__global__ void k_init(KParams P, IParams I, const double* __restrict__ phi0,
                       const double* __restrict__ T0, void* __restrict__ A,
                       float* __restrict__ phiu, void* __restrict__ ref, float* __restrict__ fsH,
                       float* __restrict__ p, float* __restrict__ S) {
  const long long N = (long long)P.nx * P.ny;
  const long long pl = P.plane;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < N;
       k += (long long)gridDim.x * blockDim.x) {
    const double ph = phi0[k];
    const double pc = ph < 0.0 ? 0.0 : (ph > 1.0 ? 1.0 : ph);
    const double cp = pc * I.cp_l + (1.0 - pc) * I.cp_g;
    const double H0 = cp * T0[k] + I.latent;
    const double Hs = cp * I.T_melt, Hl = Hs + I.latent;
    const double fl = H0 <= Hs ? 0.0 : (H0 >= Hl ? 1.0 : (H0 - Hs) / (Hl - Hs));
    const double T = H0 < Hs ? H0 / cp : (H0 > Hl ? I.T_melt + (H0 - Hl) / cp : I.T_melt);
    const double dT = T - I.T_melt;
    const double Href = I.cp_ref * I.T_melt + I.latent;
    const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    const float fs0 = (float)(1.0 - fl);
    // references of the stored g (and, node-reference storage, h)
    float ref0, th0;
    RefIO<PopIO<PT>::kNodeRef>::round((float)ph, (float)dT, ref0, th0);
    RefIO<PopIO<PT>::kNodeRef>::store(ref, (unsigned)k, ref0, th0);
    for (int i = 0; i < 9; ++i) {
      const unsigned rb = sr_node((unsigned)k, P.seed);
      pop_st<PT, 0>(A, (unsigned)(i * pl + k), (float)(w[i] * (ph - (double)ref0)), P, rb ^ sr_pop(i));
      pop_st<PT, 1>(A, (unsigned)((9 + i) * pl + k), 0.0f, P, rb ^ sr_pop(9 + i));
      const double hs = i == 0 ? (H0 - Href) - I.cp_ref * dT + w[0] * I.cp_ref * dT + I.latent * (double)fs0
                               : w[i] * I.cp_ref * dT;
      pop_st<PT, 2>(A, (unsigned)((18 + i) * pl + k), (float)(hs - w[i] * I.cp_ref * (double)th0), P,
                    rb ^ sr_pop(18 + i));
    }
    phiu[k] = 0.0f;
    phiu[pl + k] = 0.0f;
    fsH[k] = fs0;
    p[k] = 0.0f;
    S[k] = 0.0f;
  }
}

// Populations of one lattice as FP32.  FP32 storage: as stored (shifted
// variables).  Node-reference formats: with the node references added back
// (w_i phi_ref to g, w_i cp_ref th to h), i.e. in the shifted variables of
// FP32 storage.
template <class PT>
__global__ void k_expand(KParams P, const void* __restrict__ A, const void* __restrict__ ref, int lattice,
                         float* __restrict__ out) {
  const unsigned N = (unsigned)P.nx * (unsigned)P.ny;
  const unsigned pl = P.plane;
  const float s = PopIO<PT>::kScaled ? P.sc_ld[lattice] : 1.0f;
  for (unsigned k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x) {
    float r = 0.0f, th = 0.0f;
    if (PopIO<PT>::kNodeRef) RefIO<PopIO<PT>::kNodeRef>::load(ref, k, r, th);
    const float add = lattice == 0 ? r : (lattice == 2 ? P.cp_ref * th : 0.0f);
    for (int i = 0; i < 9; ++i) {
      float v = PopIO<PT>::get(A, (lattice * 9 + i) * pl + k) * s;
      if (PopIO<PT>::kNodeRef) v += wt(i) * add;
      out[i * pl + k] = v;
    }
  }
}

// Diagnostics: per-block FP64 partial sums of the output fields, then one
// block combines the partials in a fixed order (deterministic).
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}

__global__ __launch_bounds__(256) void k_reduce1(KParams P, const float* __restrict__ F,
                                                 double Href, double* __restrict__ part) {
  const long long N = (long long)P.nx * P.ny;
  const long long pl = P.plane;
  const int xc = P.nx / 2;
  double v[RED_NVAL] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long k = blockIdx.x * 256LL + threadIdx.x; k < N; k += (long long)gridDim.x * 256) {
    const double ph = F[k], T = F[pl + k], ux = F[2 * pl + k], uy = F[3 * pl + k];
    const double pr = F[4 * pl + k], fs = F[5 * pl + k], fl = F[6 * pl + k], Ht = F[8 * pl + k];
    const double pc = ph < 0.0 ? 0.0 : (ph > 1.0 ? 1.0 : ph);
    const double um = sqrt(ux * ux + uy * uy);
    v[0] += ph;
    v[1] += pc;
    v[2] += fs;
    v[3] += pc * fl;
    v[4] += Ht + Href;
    v[5] = fmax(v[5], um);
    if (!isfinite(ph) || !isfinite(T) || !isfinite(um) || !isfinite(pr)) v[6] += 1.0;
    if ((int)(k % P.nx) == xc) v[7] += fs;
  }
  __shared__ double sh[4][RED_NVAL];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < RED_NVAL; ++j) {
    const double r = j == 5 ? wave_max(v[j]) : wave_sum(v[j]);
    if (lane == 0) sh[wv][j] = r;
  }
  __syncthreads();
  if (threadIdx.x < RED_NVAL) {
    const int j = threadIdx.x;
    double r = sh[0][j];
    for (int w = 1; w < 4; ++w) r = j == 5 ? fmax(r, sh[w][j]) : r + sh[w][j];
    part[blockIdx.x * RED_NVAL + j] = r;
  }
}

__global__ __launch_bounds__(64) void k_reduce2(double* __restrict__ part, int nblocks) {
  const int j = threadIdx.x;
  if (j >= RED_NVAL) return;
  double r = part[j];
  for (int b = 1; b < nblocks; ++b) r = j == 5 ? fmax(r, part[b * RED_NVAL + j]) : r + part[b * RED_NVAL + j];
  part[RED_BLOCKS * RED_NVAL + j] = r;  // final values after the partials
}

// ---- per-grid reductions of a batch (one workgroup per grid) -------------
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}
__device__ __forceinline__ double block_max256(double v, double* sh) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

__global__ __launch_bounds__(256) void k_batch_liquid(const char* __restrict__ base,
                                                      const KParams* __restrict__ ptab,
                                                      const StepOff* __restrict__ otab,
                                                      const int* __restrict__ slots, double* __restrict__ out) {
  __shared__ double sh[4];
  const int slot = slots[blockIdx.x];
  const int nx = ptab[slot].nx, ny = ptab[slot].ny;
  const unsigned pl = ptab[slot].plane;
  const float* __restrict__ F = (const float*)(base + otab[2 * slot].fields);
  const unsigned N = (unsigned)nx * (unsigned)ny;
  double s = 0.0, bad = 0.0;
  for (unsigned k = threadIdx.x; k < N; k += 256) {
    const float ph = F[k], T = F[pl + k], ux = F[2 * pl + k], uy = F[3 * pl + k], fl = F[6 * pl + k];
    s += (double)clamp01(ph) * (double)fl;
    if (!isfinite(ph) || !isfinite(T) || !isfinite(ux) || !isfinite(uy)) bad += 1.0;
  }
  s = block_sum256(s, sh);
  bad = block_sum256(bad, sh);
  if (threadIdx.x == 0) {
    out[2 * slot] = s;
    out[2 * slot + 1] = bad;
  }
}

// Outermost phi = 1/2 crossings of one row of phi (linear interpolation);
// false if no value reaches 1/2.
__device__ bool row_crossings(const float* __restrict__ row, int nx, double& xl, double& xr) {
  int a = -1, b = -1;
  for (int x = 0; x < nx; ++x)
    if (row[x] >= 0.5f) {
      if (a < 0) a = x;
      b = x;
    }
  if (a < 0) return false;
  xl = a == 0 ? 0.0 : (a - 1) + (0.5 - (double)row[a - 1]) / ((double)row[a] - (double)row[a - 1]);
  xr = b == nx - 1 ? (double)(nx - 1) : b + ((double)row[b] - 0.5) / ((double)row[b] - (double)row[b + 1]);
  return true;
}

__global__ __launch_bounds__(256) void k_batch_shape(const char* __restrict__ base,
                                                     const KParams* __restrict__ ptab,
                                                     const StepOff* __restrict__ otab,
                                                     const int* __restrict__ slots, double* __restrict__ out) {
  __shared__ double sh[4];
  const int slot = slots[blockIdx.x];
  const int nx = ptab[slot].nx, ny = ptab[slot].ny;
  const float* __restrict__ phi = (const float*)(base + otab[2 * slot].fields);  // field plane 0
  // height: highest phi = 1/2 crossing over the columns, from the wall at y = -1/2
  double top = -1e300;
  for (int x = threadIdx.x; x < nx; x += 256) {
    for (int y = ny - 1; y >= 0; --y) {
      const float v = phi[y * nx + x];
      if (v >= 0.5f) {
        const double yc = y == ny - 1 ? (double)y
                                      : y + ((double)v - 0.5) / ((double)v - (double)phi[(y + 1) * nx + x]);
        top = fmax(top, yc);
        break;
      }
    }
  }
  top = block_max256(top, sh);
  const bool any = top > -1e299;
  const double H = any ? top + 0.5 : nan("");
  // base half-width from the crossings on row 0
  double xl0 = 0.0, xr0 = 0.0;
  const bool has_base = row_crossings(phi, nx, xl0, xr0);
  // tip: least-squares lines x(y) through the left and right crossings of
  // the rows whose height y + 1/2 lies in [0.75 H, 0.95 H]
  double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // left n, y, x, yy, xy; right n, y, x, yy, xy
  if (any) {
    for (int y = threadIdx.x; y < ny; y += 256) {
      const double hy = y + 0.5;
      if (hy < 0.75 * H || hy > 0.95 * H) continue;
      double xl, xr;
      if (!row_crossings(phi + y * nx, nx, xl, xr)) continue;
      s[0] += 1.0; s[1] += y; s[2] += xl; s[3] += (double)y * y; s[4] += y * xl;
      s[5] += 1.0; s[6] += y; s[7] += xr; s[8] += (double)y * y; s[9] += y * xr;
    }
  }
  for (int j = 0; j < 10; ++j) s[j] = block_sum256(s[j], sh);
  if (threadIdx.x == 0) {
    double ang = nan("");
    if (s[0] >= 2.0) {
      const double bl = (s[0] * s[4] - s[2] * s[1]) / (s[0] * s[3] - s[1] * s[1]);
      const double br = (s[5] * s[9] - s[7] * s[6]) / (s[5] * s[8] - s[6] * s[6]);
      ang = (atan(bl) - atan(br)) * (180.0 / M_PI);
    }
    out[4 * slot + 0] = H;
    out[4 * slot + 1] = has_base ? 0.5 * (xr0 - xl0) : nan("");
    out[4 * slot + 2] = ang;
    out[4 * slot + 3] = s[0];
  }
}

template <int TX, int TY, class PT>
int launch_tile(const KParams& P, const State& S, int cur, bool fields_only, int xcd, hipStream_t st) {
  const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
  const int ntiles = ntx * nty;
  int band = 0, grid = ntiles;
  if (xcd == 1) {
    band = (ntiles + 7) / 8;
    grid = 8 * band;
  } else if (xcd == 2) {
    band = (ntx + 7) / 8;
    grid = 8 * band * nty;
  }
  const StepIO io = make_io(S, cur);
  if (fields_only)
    hipLaunchKernelGGL((k_step<TX, TY, true, PT>), dim3(grid), dim3(TX * TY), 0, st, P, io, ntx, ntiles, band, xcd);
  else if (P.stream_stores)
    hipLaunchKernelGGL((k_step<TX, TY, false, PT, true>), dim3(grid), dim3(TX * TY), 0, st, P, io, ntx, ntiles, band,
                       xcd);
  else
    hipLaunchKernelGGL((k_step<TX, TY, false, PT>), dim3(grid), dim3(TX * TY), 0, st, P, io, ntx, ntiles, band, xcd);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

namespace {

template <int TX, int TY, class PT>
int launch_unfused(const KParams& P, const State& S, int cur, bool fields_only, int xcd, hipStream_t st) {
  if (fields_only) return launch_tile<TX, TY, PT>(P, S, cur, true, xcd, st);
  const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
  const int ntiles = ntx * nty;
  int band = 0, grid = ntiles;
  if (xcd == 1) {
    band = (ntiles + 7) / 8;
    grid = 8 * band;
  } else if (xcd == 2) {
    band = (ntx + 7) / 8;
    grid = 8 * band * nty;
  }
  const StepIO io = make_io(S, cur);
  hipLaunchKernelGGL((k_macro<TX, TY, PT>), dim3(grid), dim3(TX * TY), 0, st, P, io, ntx, ntiles, band, xcd);
  hipLaunchKernelGGL((k_collide<TX, TY, PT>), dim3(grid), dim3(TX * TY), 0, st, P, io, ntx, ntiles, band, xcd);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int TX, int TY>
int launch_tile2(const KParams& P, const State& S, int cur, int xcd, hipStream_t st) {
  const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
  const int ntiles = ntx * nty;
  int band = 0, grid = ntiles;
  if (xcd == 1) {
    band = (ntiles + 7) / 8;
    grid = 8 * band;
  } else if (xcd == 2) {
    band = (ntx + 7) / 8;
    grid = 8 * band * nty;
  }
  const StepIO io = make_io(S, cur);
  if (P.stream_stores)
    hipLaunchKernelGGL((k_step2<TX, TY, true>), dim3(grid), dim3(TX * TY), 0, st, P, io, ntx, ntiles, band, xcd);
  else
    hipLaunchKernelGGL((k_step2<TX, TY, false>), dim3(grid), dim3(TX * TY), 0, st, P, io, ntx, ntiles, band, xcd);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <class PT>
int launch_step_t(const KParams& P, const State& S, int cur, bool fields_only, int tile_variant,
                  int xcd_remap, hipStream_t st) {
  switch (tile_variant) {
    case 5:
      return launch_unfused<64, 8, PT>(P, S, cur, fields_only, xcd_remap, st);
    case 1:
      return launch_tile<32, 8, PT>(P, S, cur, fields_only, xcd_remap, st);
    case 6:  // single steps (an odd remainder) and field output of the two-step variants
    case 7:
    case 8:
    case 9:
    case 10:
    case 2:
      return launch_tile<64, 8, PT>(P, S, cur, fields_only, xcd_remap, st);
    case 3:
      return launch_tile<64, 16, PT>(P, S, cur, fields_only, xcd_remap, st);
    case 4:
      return launch_tile<128, 4, PT>(P, S, cur, fields_only, xcd_remap, st);
    default:
      return launch_tile<64, 4, PT>(P, S, cur, fields_only, xcd_remap, st);
  }
}

int grid_of(const KParams& P) {
  const long long N = (long long)P.nx * P.ny;
  return (int)std::min<long long>((N + 255) / 256, 4096);
}

}  // namespace

int launch_init(const KParams& P, const IParams& I, const State& S, int cur, const double* d_phi0,
                const double* d_T0, hipStream_t st) {
  const int grid = grid_of(P);
  if (P.storage == STORE_FP16)
    hipLaunchKernelGGL(k_init<_Float16>, dim3(grid), dim3(256), 0, st, P, I, d_phi0, d_T0, S.pops[cur],
                       S.phiu[cur], S.ref[cur], S.fsH[cur], S.p[cur], S.S[cur]);
  else if (P.storage == STORE_BF16)
    hipLaunchKernelGGL(k_init<__bf16>, dim3(grid), dim3(256), 0, st, P, I, d_phi0, d_T0, S.pops[cur],
                       S.phiu[cur], S.ref[cur], S.fsH[cur], S.p[cur], S.S[cur]);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(grid), dim3(256), 0, st, P, I, d_phi0, d_T0, S.pops[cur],
                       S.phiu[cur], S.ref[cur], S.fsH[cur], S.p[cur], S.S[cur]);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_step(const KParams& P, const State& S, int cur, bool fields_only, int tile_variant,
                int xcd_remap, hipStream_t st) {
  if (P.storage == STORE_FP16)
    return launch_step_t<_Float16>(P, S, cur, fields_only, tile_variant, xcd_remap, st);
  if (P.storage == STORE_BF16)
    return launch_step_t<__bf16>(P, S, cur, fields_only, tile_variant, xcd_remap, st);
  return launch_step_t<float>(P, S, cur, fields_only, tile_variant, xcd_remap, st);
}

template <int TX, int TY, int NT, class PT>
int launch_tile2w(const KParams& P, const State& S, int cur, int xcd, hipStream_t st) {
  const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
  const int ntiles = ntx * nty;
  int band = 0, grid = ntiles;
  if (xcd == 1) {
    band = (ntiles + 7) / 8;
    grid = 8 * band;
  } else if (xcd == 2) {
    band = (ntx + 7) / 8;
    grid = 8 * band * nty;
  }
  const StepIO io = make_io(S, cur);
  if (P.stream_stores)
    hipLaunchKernelGGL((k_step2w<TX, TY, NT, PT, true>), dim3(grid), dim3(NT), 0, st, P, io, ntx, ntiles, band,
                       xcd);
  else
    hipLaunchKernelGGL((k_step2w<TX, TY, NT, PT, false>), dim3(grid), dim3(NT), 0, st, P, io, ntx, ntiles, band,
                       xcd);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <class PT>
int launch_step2w_t(const KParams& P, const State& S, int cur, int tile_variant, int xcd_remap, hipStream_t st) {
  if (tile_variant == TWO_STEP_VARIANT + 3) return launch_tile2w<32, 16, 1024, PT>(P, S, cur, xcd_remap, st);
  return launch_tile2w<32, 8, 768, PT>(P, S, cur, xcd_remap, st);
}

int launch_step2(const KParams& P, const State& S, int cur, int tile_variant, int xcd_remap, hipStream_t st) {
  if (P.storage != STORE_FP32) {
    if (!is_two_step_any_storage(tile_variant)) return -1;
    if (P.storage == STORE_FP16) return launch_step2w_t<_Float16>(P, S, cur, tile_variant, xcd_remap, st);
    return launch_step2w_t<__bf16>(P, S, cur, tile_variant, xcd_remap, st);
  }
  switch (tile_variant) {
    case TWO_STEP_VARIANT + 3:
    case TWO_STEP_VARIANT + 4:
      return launch_step2w_t<float>(P, S, cur, tile_variant, xcd_remap, st);
    case TWO_STEP_VARIANT:
      return launch_tile2<64, 8>(P, S, cur, xcd_remap, st);
    case TWO_STEP_VARIANT + 1:
      return launch_tile2<32, 8>(P, S, cur, xcd_remap, st);
    case TWO_STEP_VARIANT + 2:
      return launch_tile2<32, 16>(P, S, cur, xcd_remap, st);
    default:
      return -1;
  }
}

namespace {

template <int TX, int TY, class PT>
hipError_t launch_persist_t(const KParams& P, const State& S, int cur, int nsteps, int xcd, int per_xcd,
                            unsigned long long* bar, unsigned long long limit, int* grid_out, hipStream_t st) {
  const int ntx = (P.nx + TX - 1) / TX, nty = (P.ny + TY - 1) / TY;
  int ntiles = ntx * nty, band = 0, vgrid = ntiles;
  if (xcd == 1) {
    band = (ntiles + 7) / 8;
    vgrid = 8 * band;
  } else if (xcd == 2) {
    band = (ntx + 7) / 8;
    vgrid = 8 * band * nty;
  }
  const void* fn = P.stream_stores ? (const void*)k_persist<TX, TY, PT, true> : (const void*)k_persist<TX, TY, PT, false>;
  int dev = 0, ncu = 0, coop = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, TX * TY, 0);
  if (e != hipSuccess) return e;
  if (!coop) return hipErrorNotSupported;
  // co-resident workgroups, a multiple of 8 so that the XCD of a tile is the
  // one its place in the tile order gives it
  const int cap = (per_cu * ncu) & ~7;
  if (cap < 8) return hipErrorCooperativeLaunchTooLarge;
  int grid = vgrid < cap ? vgrid : cap;
  *grid_out = grid;
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, bar, (int)NPERSIST_WORDS);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  KParams Pa = P;
  StepIO io = make_io(S, cur);
  void* args[] = {&Pa, &io, &nsteps, (void*)&ntx, &ntiles, &band, &xcd, &vgrid, &per_xcd, &bar, &limit};
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(TX * TY), args, 0, st);
}

}  // namespace

hipError_t launch_persist(const KParams& P, const State& S, int cur, int nsteps, int xcd_remap, int per_xcd,
                          unsigned long long* bar, unsigned long long limit_ticks, int* grid_out, hipStream_t st) {
  if (P.storage == STORE_FP16)
    return launch_persist_t<64, 8, _Float16>(P, S, cur, nsteps, xcd_remap, per_xcd, bar, limit_ticks, grid_out, st);
  if (P.storage == STORE_BF16)
    return launch_persist_t<64, 8, __bf16>(P, S, cur, nsteps, xcd_remap, per_xcd, bar, limit_ticks, grid_out, st);
  return launch_persist_t<64, 8, float>(P, S, cur, nsteps, xcd_remap, per_xcd, bar, limit_ticks, grid_out, st);
}

int launch_expand(const KParams& P, const State& S, int cur, int lattice, hipStream_t st) {
  const int grid = grid_of(P);
  if (P.storage == STORE_FP16)
    hipLaunchKernelGGL(k_expand<_Float16>, dim3(grid), dim3(256), 0, st, P, S.pops[cur], S.ref[cur], lattice,
                       S.fields);
  else if (P.storage == STORE_BF16)
    hipLaunchKernelGGL(k_expand<__bf16>, dim3(grid), dim3(256), 0, st, P, S.pops[cur], S.ref[cur], lattice,
                       S.fields);
  else
    hipLaunchKernelGGL(k_expand<float>, dim3(grid), dim3(256), 0, st, P, S.pops[cur], S.ref[cur], lattice,
                       S.fields);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

void tile_shape(int tile_variant, int* tx, int* ty) {
  static const int T[NBATCH_VARIANTS][2] = {{64, 4}, {32, 8}, {64, 8}, {64, 16}, {128, 4}};
  if (tile_variant == TWO_STEP_VARIANT + 3) {  // two steps per launch, 32x16 tiles
    *tx = 32;
    *ty = 16;
    return;
  }
  if (tile_variant == TWO_STEP_VARIANT + 4) {  // two steps per launch, 32x8 tiles
    *tx = 32;
    *ty = 8;
    return;
  }
  const int v = tile_variant >= 0 && tile_variant < NBATCH_VARIANTS ? tile_variant : 0;
  *tx = T[v][0];
  *ty = T[v][1];
}

namespace {
template <int TX, int TY, class PT>
int launch_batch_t(bool fields_only, bool nt, char* base, const KParams* ptab, const StepOff* otab,
                   const unsigned* tmap, const unsigned* steps, int nblocks, int s, hipStream_t st) {
  if (fields_only)
    hipLaunchKernelGGL((k_batch<TX, TY, true, PT>), dim3(nblocks), dim3(TX * TY), 0, st, base, ptab, otab, tmap,
                       steps, s);
  else if (nt)
    hipLaunchKernelGGL((k_batch<TX, TY, false, PT, true>), dim3(nblocks), dim3(TX * TY), 0, st, base, ptab, otab,
                       tmap, steps, s);
  else
    hipLaunchKernelGGL((k_batch<TX, TY, false, PT>), dim3(nblocks), dim3(TX * TY), 0, st, base, ptab, otab, tmap,
                       steps, s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
template <int TX, int TY, int NT, class PT>
int launch_batch2_t(bool nt, char* base, const KParams* ptab, const StepOff* otab, const unsigned* tmap,
                    const unsigned* steps, int nblocks, int s, hipStream_t st) {
  if (nt)
    hipLaunchKernelGGL((k_batch2w<TX, TY, NT, PT, true>), dim3(nblocks), dim3(NT), 0, st, base, ptab, otab, tmap,
                       steps, s);
  else
    hipLaunchKernelGGL((k_batch2w<TX, TY, NT, PT, false>), dim3(nblocks), dim3(NT), 0, st, base, ptab, otab, tmap,
                       steps, s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
template <class PT>
int launch_batch_v(int variant, bool fields_only, bool nt, char* base, const KParams* ptab, const StepOff* otab,
                   const unsigned* tmap, const unsigned* steps, int nblocks, int s, hipStream_t st) {
  if (variant == TWO_STEP_VARIANT + 3) {  // fields pass on the same 32x16 tiles
    if (fields_only) return launch_batch_t<32, 16, PT>(true, false, base, ptab, otab, tmap, steps, nblocks, s, st);
    return launch_batch2_t<32, 16, 1024, PT>(nt, base, ptab, otab, tmap, steps, nblocks, s, st);
  }
  if (variant == TWO_STEP_VARIANT + 4) {
    if (fields_only) return launch_batch_t<32, 8, PT>(true, false, base, ptab, otab, tmap, steps, nblocks, s, st);
    return launch_batch2_t<32, 8, 768, PT>(nt, base, ptab, otab, tmap, steps, nblocks, s, st);
  }
  switch (variant) {
    case 0:
      return launch_batch_t<64, 4, PT>(fields_only, nt, base, ptab, otab, tmap, steps, nblocks, s, st);
    case 1:
      return launch_batch_t<32, 8, PT>(fields_only, nt, base, ptab, otab, tmap, steps, nblocks, s, st);
    case 2:
      return launch_batch_t<64, 8, PT>(fields_only, nt, base, ptab, otab, tmap, steps, nblocks, s, st);
    case 3:
      return launch_batch_t<64, 16, PT>(fields_only, nt, base, ptab, otab, tmap, steps, nblocks, s, st);
    case 4:
      return launch_batch_t<128, 4, PT>(fields_only, nt, base, ptab, otab, tmap, steps, nblocks, s, st);
    default:
      return -1;
  }
}
}  // namespace

int launch_batch(int storage, int tile_variant, bool fields_only, bool nt, char* d_base, const KParams* d_ptab,
                 const StepOff* d_otab, const unsigned* d_tmap, const unsigned* d_steps, int nblocks, int s,
                 hipStream_t st) {
  if (nblocks <= 0) return 0;
  if (storage == STORE_FP16)
    return launch_batch_v<_Float16>(tile_variant, fields_only, nt, d_base, d_ptab, d_otab, d_tmap, d_steps, nblocks, s,
                                    st);
  if (storage == STORE_BF16)
    return launch_batch_v<__bf16>(tile_variant, fields_only, nt, d_base, d_ptab, d_otab, d_tmap, d_steps, nblocks, s,
                                  st);
  return launch_batch_v<float>(tile_variant, fields_only, nt, d_base, d_ptab, d_otab, d_tmap, d_steps, nblocks, s, st);
}

namespace {

template <class PT>
hipError_t launch_batch_persist_t(bool nt, int per_xcd, char* d_base, const KParams* d_ptab, const StepOff* d_otab,
                                  const unsigned* d_tmap, const unsigned* d_steps, int nblocks, int nsteps,
                                  unsigned long long* bar, unsigned long long limit, int* grid_out, hipStream_t st) {
  const void* fn = nt ? (const void*)k_batch_persist<PT, true> : (const void*)k_batch_persist<PT, false>;
  int dev = 0, ncu = 0, coop = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 512, 0);
  if (e != hipSuccess) return e;
  if (!coop) return hipErrorNotSupported;
  const int cap = (per_cu * ncu) & ~7;  // co-resident workgroups, a multiple of 8
  if (cap < 8) return hipErrorCooperativeLaunchTooLarge;
  int grid = nblocks < cap ? nblocks : cap;
  *grid_out = grid;
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, bar, (int)NPERSIST_WORDS);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  void* args[] = {&d_base, (void*)&d_ptab, (void*)&d_otab, (void*)&d_tmap, (void*)&d_steps, &nblocks, &nsteps,
                  &per_xcd, &bar, &limit};
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(512), args, 0, st);
}

}  // namespace

hipError_t launch_batch_persist(int storage, bool nt, int per_xcd, char* d_base, const KParams* d_ptab,
                                const StepOff* d_otab, const unsigned* d_tmap, const unsigned* d_steps, int nblocks,
                                int nsteps, unsigned long long* bar, unsigned long long limit_ticks, int* grid_out,
                                hipStream_t st) {
  if (nblocks <= 0 || nsteps <= 0) return hipErrorInvalidValue;
  if (storage == STORE_FP16)
    return launch_batch_persist_t<_Float16>(nt, per_xcd, d_base, d_ptab, d_otab, d_tmap, d_steps, nblocks, nsteps, bar,
                                            limit_ticks, grid_out, st);
  if (storage == STORE_BF16)
    return launch_batch_persist_t<__bf16>(nt, per_xcd, d_base, d_ptab, d_otab, d_tmap, d_steps, nblocks, nsteps, bar,
                                          limit_ticks, grid_out, st);
  return launch_batch_persist_t<float>(nt, per_xcd, d_base, d_ptab, d_otab, d_tmap, d_steps, nblocks, nsteps, bar,
                                       limit_ticks, grid_out, st);
}

int launch_batch_liquid(const char* d_base, const KParams* d_ptab, const StepOff* d_otab, const int* d_slots,
                        int nslots, double* d_out, hipStream_t st) {
  if (nslots <= 0) return 0;
  hipLaunchKernelGGL(k_batch_liquid, dim3(nslots), dim3(256), 0, st, d_base, d_ptab, d_otab, d_slots, d_out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_batch_shape(const char* d_base, const KParams* d_ptab, const StepOff* d_otab, const int* d_slots,
                       int nslots, double* d_out, hipStream_t st) {
  if (nslots <= 0) return 0;
  hipLaunchKernelGGL(k_batch_shape, dim3(nslots), dim3(256), 0, st, d_base, d_ptab, d_otab, d_slots, d_out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_reduce(const KParams& P, const State& S, double Href, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce1, dim3(RED_BLOCKS), dim3(256), 0, st, P, S.fields, Href, S.part);
  hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(64), 0, st, S.part, RED_BLOCKS);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace lbmk
