// Surrogate network of the parametric sweep on gfx950 matrix cores.
//
// An ensemble of E networks maps the droplet parameters (R, theta, Ste,
// gamma, bubble count; normalised by the caller) to 3 outputs through two
// hidden layers of 128 GELU units.  Weights live as FP32 master copies
// (Adam) and as BF16 copies that feed v_mfma_f32_32x32x16_bf16 with FP32
// accumulation.  Three kernels:
//   k_mlp_rows   one wavefront per 32 samples: forward pass, and for
//                training the output gradient and the back-propagated
//                hidden gradients (every product on the matrix cores);
//                stores BF16 activations/gradients row-major for the next
//                kernel and FP32 per-wavefront partial bias gradients and
//                losses;
//   k_mlp_wgrad  weight gradients dW = G^T A summed over samples (split-K,
//                LDS-transposed tiles, matrix cores);
//   k_mlp_update deterministic reduction of the partials, Adam update and
//                repacking of the BF16 copies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"

namespace {

constexpr int IN = 5, INP = 16, HID = 128, OUT = 3, OUTP = 32;
// FP32 parameters per member, host order: W1 (HID x IN), b1, W2 (HID x HID), b2, W3 (OUT x HID), b3
constexpr int OW1 = 0, OB1 = OW1 + HID * IN, OW2 = OB1 + HID, OB2 = OW2 + HID * HID, OW3 = OB2 + HID,
              OB3 = OW3 + OUT * HID, NPAR = OB3 + OUT;
// BF16 copies per member: W1p (HID x INP), W2 (HID x HID), W2T, W3p (OUTP x HID), W3T (HID x OUTP)
constexpr int PW1 = 0, PW2 = PW1 + HID * INP, PW2T = PW2 + HID * HID, PW3 = PW2T + HID * HID, PW3T = PW3 + OUTP * HID,
              NPACK = PW3T + HID * OUTP;
// FP32 biases per member (padded): b1 (HID), b2 (HID), b3 (OUTP)
constexpr int NBIAS = HID + HID + OUTP;
// weight-gradient partial per member and K-chunk: dW1 (HID x INP), dW2 (HID x HID), dW3 (OUTP x HID)
constexpr int GW1 = 0, GW2 = GW1 + HID * INP, GW3 = GW2 + HID * HID, NGW = GW3 + OUTP * HID;
constexpr int SAMPLES_PER_BLOCK = 128;  // 4 wavefronts x 32 rows
constexpr int KCHUNK = 512;             // samples per weight-gradient workgroup
constexpr int SPAD = HID + 8;           // LDS row pitch of a 32 x 128 BF16 tile (keeps 16-B alignment)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int r = 0; r < 16; ++r) z[r] = 0.0f;
  return z;
}
__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *(const bf16x8*)p; }
// Row of accumulator element r of lane l (column is l & 31).
__device__ __forceinline__ int drow(int r, int kg) { return 8 * (r >> 2) + 4 * kg + (r & 3); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

struct RowsArgs {
  const float* x;     // [n][IN]
  const float* t;     // [n][OUT] (training)
  const float* mask;  // [n][OUT] (training)
  float* y;           // [E][n][OUT] (inference; may be null in training)
  const __bf16* pack; // [E][NPACK]
  const float* bias;  // [E][NBIAS]
  __bf16* Xg;         // [E][np][INP]   training: stored operands of the weight gradients
  __bf16* H1g;        // [E][np][HID]
  __bf16* H2g;        // [E][np][HID]
  __bf16* dYg;        // [E][np][OUTP]
  __bf16* dZ1g;       // [E][np][HID]
  __bf16* dZ2g;       // [E][np][HID]
  float* bpart;       // [E][nwaves][NBIAS] partial bias gradients
  float* lpart;       // [E][nwaves] partial losses
  int n, np;          // samples; padded sample count (multiple of KCHUNK)
  float w0, w1, w2;   // output weights of the loss
};

// Copy this wavefront's 32 x 128 BF16 stage tile to rows s0.. of a
// row-major [np][HID] array (16-byte stores).
__device__ __forceinline__ void store_tile(const __bf16 (*stage)[SPAD], __bf16* dst, int s0, int lane) {
#pragma unroll
  for (int it = 0; it < 8; ++it) {
    const int v = it * 64 + lane;     // 512 vectors of 8 values
    const int row = v >> 4, c8 = (v & 15) * 8;
    *(bf16x8*)(dst + (size_t)(s0 + row) * HID + c8) = *(const bf16x8*)&stage[row][c8];
  }
}

template <bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp_rows(RowsArgs a) {
  __shared__ __bf16 stage[4][32][SPAD];
  const int e = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 31, kg = lane >> 5;
  const int s0 = blockIdx.x * SAMPLES_PER_BLOCK + wave * 32;
  const __bf16* P = a.pack + (size_t)e * NPACK;
  const float* bias = a.bias + (size_t)e * NBIAS;
  __bf16 (*st)[SPAD] = stage[wave];

  // ---- layer 1: z1 = x W1^T + b1 (x padded to 16 inputs)
  bf16x8 ax;
  {
    const int s = s0 + i;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * kg + j;
      ax[j] = (__bf16)((k < IN && s < a.n) ? a.x[(size_t)s * IN + k] : 0.0f);
    }
  }
  f32x16 z1[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    z1[nb] = mfma(ax, ld8(P + PW1 + (nb * 32 + i) * INP + 8 * kg), zero16());
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      z1[nb][r] += bias[nb * 32 + i];
      st[drow(r, kg)][nb * 32 + i] = (__bf16)gelu(z1[nb][r]);
    }
  }
  __syncthreads();
  if (TRAIN) {
    store_tile(st, a.H1g + (size_t)e * a.np * HID, s0, lane);
    // x operand (BF16, padded), one lane per sample row
    if (kg == 0) {
      __bf16* xr = a.Xg + ((size_t)e * a.np + s0 + i) * INP;
      bf16x8 lo, hi;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int s = s0 + i;
        lo[j] = (__bf16)((j < IN && s < a.n) ? a.x[(size_t)s * IN + j] : 0.0f);
        hi[j] = (__bf16)0.0f;
      }
      *(bf16x8*)xr = lo;
      *(bf16x8*)(xr + 8) = hi;
    }
  }
  // ---- layer 2: z2 = h1 W2^T + b2
  f32x16 z2[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) z2[nb] = zero16();
#pragma unroll
  for (int kb = 0; kb < HID / 16; ++kb) {
    const bf16x8 av = ld8(&st[i][kb * 16 + 8 * kg]);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) z2[nb] = mfma(av, ld8(P + PW2 + (nb * 32 + i) * HID + kb * 16 + 8 * kg), z2[nb]);
  }
  __syncthreads();
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      z2[nb][r] += bias[HID + nb * 32 + i];
      st[drow(r, kg)][nb * 32 + i] = (__bf16)gelu(z2[nb][r]);
    }
  __syncthreads();
  if (TRAIN) store_tile(st, a.H2g + (size_t)e * a.np * HID, s0, lane);
  // ---- layer 3: y = h2 W3^T + b3 (outputs padded to 32)
  f32x16 yv = zero16();
#pragma unroll
  for (int kb = 0; kb < HID / 16; ++kb)
    yv = mfma(ld8(&st[i][kb * 16 + 8 * kg]), ld8(P + PW3 + i * HID + kb * 16 + 8 * kg), yv);
#pragma unroll
  for (int r = 0; r < 16; ++r) yv[r] += bias[2 * HID + i];
  if (!TRAIN) {
    if (i < OUT)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int s = s0 + drow(r, kg);
        if (s < a.n) a.y[((size_t)e * a.n + s) * OUT + i] = yv[r];
      }
    return;
  }

  // ---- backward: dY = 2 w (y - t) mask / n
  const float wj = i == 0 ? a.w0 : (i == 1 ? a.w1 : a.w2);
  const float inv_n = 1.0f / (float)a.n;
  float lsum = 0.0f, db3 = 0.0f;
  __syncthreads();  // the stage tile is reused for dY
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = drow(r, kg), s = s0 + row;
    float d = 0.0f;
    if (i < OUT && s < a.n) {
      const float res = (yv[r] - a.t[(size_t)s * OUT + i]) * a.mask[(size_t)s * OUT + i];
      lsum += wj * res * res * inv_n;
      d = 2.0f * wj * res * inv_n;
    }
    db3 += d;
    st[row][i] = (__bf16)d;  // columns 0..31 of the tile: dY padded to 32 outputs
  }
  __syncthreads();
  {
    // dY rows to global (32 values of 2 B per row: 4 vectors)
    __bf16* dst = a.dYg + (size_t)e * a.np * OUTP;
    for (int v = lane; v < 32 * 4; v += 64) {
      const int row = v >> 2, c8 = (v & 3) * 8;
      *(bf16x8*)(dst + (size_t)(s0 + row) * OUTP + c8) = *(const bf16x8*)&st[row][c8];
    }
  }
  // dH2 = dY W3 (K = 32 outputs), dZ2 = dH2 * gelu'(z2)
  f32x16 g[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) g[nb] = zero16();
#pragma unroll
  for (int kb = 0; kb < OUTP / 16; ++kb) {
    const bf16x8 av = ld8(&st[i][kb * 16 + 8 * kg]);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) g[nb] = mfma(av, ld8(P + PW3T + (nb * 32 + i) * OUTP + kb * 16 + 8 * kg), g[nb]);
  }
  float db2[4];
  __syncthreads();
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    db2[nb] = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float d = (s0 + drow(r, kg) < a.n) ? g[nb][r] * gelu_d(z2[nb][r]) : 0.0f;
      db2[nb] += d;
      st[drow(r, kg)][nb * 32 + i] = (__bf16)d;
    }
  }
  __syncthreads();
  store_tile(st, a.dZ2g + (size_t)e * a.np * HID, s0, lane);
  // dH1 = dZ2 W2 (K = 128), dZ1 = dH1 * gelu'(z1)
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) g[nb] = zero16();
#pragma unroll
  for (int kb = 0; kb < HID / 16; ++kb) {
    const bf16x8 av = ld8(&st[i][kb * 16 + 8 * kg]);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) g[nb] = mfma(av, ld8(P + PW2T + (nb * 32 + i) * HID + kb * 16 + 8 * kg), g[nb]);
  }
  float db1[4];
  __syncthreads();
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    db1[nb] = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float d = (s0 + drow(r, kg) < a.n) ? g[nb][r] * gelu_d(z1[nb][r]) : 0.0f;
      db1[nb] += d;
      st[drow(r, kg)][nb * 32 + i] = (__bf16)d;
    }
  }
  __syncthreads();
  store_tile(st, a.dZ1g + (size_t)e * a.np * HID, s0, lane);
  // per-wavefront partials: the two half-waves (kg) hold the same columns
  const int wid = blockIdx.x * 4 + wave;
  const int nw = gridDim.x * 4;
  float* bp = a.bpart + ((size_t)e * nw + wid) * NBIAS;
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const float s1 = db1[nb] + __shfl_xor(db1[nb], 32, 64);
    const float s2 = db2[nb] + __shfl_xor(db2[nb], 32, 64);
    if (kg == 0) {
      bp[nb * 32 + i] = s1;
      bp[HID + nb * 32 + i] = s2;
    }
  }
  const float s3 = db3 + __shfl_xor(db3, 32, 64);
  if (kg == 0) bp[2 * HID + i] = s3;
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
  if (lane == 0) a.lpart[(size_t)e * nw + wid] = lsum;
}

struct WgradArgs {
  const __bf16 *Xg, *H1g, *H2g, *dYg, *dZ1g, *dZ2g;
  float* wpart;  // [E][nchunks][NGW]
  int np, nchunks;
};

// dW[out][in] = sum_s G[s][out] A[s][in] over one chunk of KCHUNK samples.
// blockIdx.x: chunk, blockIdx.y: product (0: dW1, 1: dW2, 2: dW3), blockIdx.z: member.
// Tiles of 32 samples are staged transposed in LDS so both operands are
// read as 8 consecutive samples.
__global__ __launch_bounds__(256) void k_mlp_wgrad(WgradArgs a) {
  __shared__ __bf16 GT[HID][32 + 8];
  __shared__ __bf16 AT[HID][32 + 8];
  const int chunk = blockIdx.x, prod = blockIdx.y, e = blockIdx.z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 31, kg = lane >> 5;
  const int M = prod == 2 ? OUTP : HID;       // output units (rows of dW)
  const int N = prod == 0 ? INP : HID;        // input units (columns of dW)
  const int gw = prod == 2 ? OUTP : HID;      // row width of G in memory
  const __bf16* G = prod == 0 ? a.dZ1g : (prod == 1 ? a.dZ2g : a.dYg);
  const __bf16* A = prod == 0 ? a.Xg : (prod == 1 ? a.H1g : a.H2g);
  G += (size_t)e * a.np * gw;
  A += (size_t)e * a.np * N;
  const int mb = wave;                         // this wavefront's 32 output rows
  const bool active = mb * 32 < M;
  const int nnb = N == INP ? 1 : 4;            // column blocks of 32 (dW1: 16 columns, padded)
  f32x16 acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = zero16();
  for (int t0 = chunk * KCHUNK; t0 < (chunk + 1) * KCHUNK; t0 += 32) {
    __syncthreads();
    // stage 32 samples of G (M wide) and A (N wide), transposed
    for (int v = threadIdx.x; v < 32 * (M / 8); v += 256) {
      const int s = v / (M / 8), c8 = (v % (M / 8)) * 8;
      const bf16x8 q = *(const bf16x8*)(G + (size_t)(t0 + s) * gw + c8);
#pragma unroll
      for (int j = 0; j < 8; ++j) GT[c8 + j][s] = q[j];
    }
    for (int v = threadIdx.x; v < 32 * (N / 8); v += 256) {
      const int s = v / (N / 8), c8 = (v % (N / 8)) * 8;
      const bf16x8 q = *(const bf16x8*)(A + (size_t)(t0 + s) * N + c8);
#pragma unroll
      for (int j = 0; j < 8; ++j) AT[c8 + j][s] = q[j];
    }
    if (N == INP)  // columns 16..31 of the padded dW1 block read zeros
      for (int v = threadIdx.x; v < 16 * 32; v += 256) AT[16 + (v >> 5)][v & 31] = (__bf16)0.0f;
    __syncthreads();
    if (active) {
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const bf16x8 av = ld8(&GT[mb * 32 + i][kb * 16 + 8 * kg]);
        for (int nb = 0; nb < nnb; ++nb) acc[nb] = mfma(av, ld8(&AT[nb * 32 + i][kb * 16 + 8 * kg]), acc[nb]);
      }
    }
  }
  if (!active) return;
  float* out = a.wpart + ((size_t)e * a.nchunks + chunk) * NGW + (prod == 0 ? GW1 : (prod == 1 ? GW2 : GW3));
  for (int nb = 0; nb < nnb; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int col = nb * 32 + i;
      if (col < N) out[(mb * 32 + drow(r, kg)) * N + col] = acc[nb][r];
    }
}

struct UpdateArgs {
  float* master;        // [E][NPAR]
  float* m1;            // [E][NPAR] Adam moments
  float* m2;
  float* grad;          // [E][NPAR] out: reduced gradient
  const float* wpart;   // [E][nchunks][NGW]
  const float* bpart;   // [E][nwaves][NBIAS]
  int nchunks, nwaves;
  int update;           // 0: gradient only
  float lr, b1, b2, eps, c1, c2;  // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
};

// One thread per parameter: reduce the partials in a fixed order, then Adam.
__global__ __launch_bounds__(256) void k_mlp_update(UpdateArgs a, int E) {
  const int gidx = blockIdx.x * 256 + threadIdx.x;
  if (gidx >= E * NPAR) return;
  const int e = gidx / NPAR, p = gidx - e * NPAR;
  double g = 0.0;
  if (p < OB1) {  // W1 (HID x IN) from dW1 (HID x INP)
    const int o = p / IN, c = p % IN;
    for (int k = 0; k < a.nchunks; ++k) g += a.wpart[((size_t)e * a.nchunks + k) * NGW + GW1 + o * INP + c];
  } else if (p < OW2) {
    for (int w = 0; w < a.nwaves; ++w) g += a.bpart[((size_t)e * a.nwaves + w) * NBIAS + (p - OB1)];
  } else if (p < OB2) {
    for (int k = 0; k < a.nchunks; ++k) g += a.wpart[((size_t)e * a.nchunks + k) * NGW + GW2 + (p - OW2)];
  } else if (p < OW3) {
    for (int w = 0; w < a.nwaves; ++w) g += a.bpart[((size_t)e * a.nwaves + w) * NBIAS + HID + (p - OB2)];
  } else if (p < OB3) {
    for (int k = 0; k < a.nchunks; ++k) g += a.wpart[((size_t)e * a.nchunks + k) * NGW + GW3 + (p - OW3)];
  } else {
    for (int w = 0; w < a.nwaves; ++w) g += a.bpart[((size_t)e * a.nwaves + w) * NBIAS + 2 * HID + (p - OB3)];
  }
  const float gf = (float)g;
  a.grad[gidx] = gf;
  if (!a.update) return;
  // Adam (Kingma & Ba, 2015), bias-corrected moments
  const float m = a.b1 * a.m1[gidx] + (1.0f - a.b1) * gf;
  const float v = a.b2 * a.m2[gidx] + (1.0f - a.b2) * gf * gf;
  a.m1[gidx] = m;
  a.m2[gidx] = v;
  a.master[gidx] -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
}

// BF16 copies (with the transposes the backward products read) and padded
// FP32 biases from the master parameters.
__global__ __launch_bounds__(256) void k_mlp_pack(const float* __restrict__ master, __bf16* __restrict__ pack,
                                                  float* __restrict__ bias, int E) {
  const int gidx = blockIdx.x * 256 + threadIdx.x;
  if (gidx >= E * NPACK) return;
  const int e = gidx / NPACK, q = gidx - e * NPACK;
  const float* P = master + (size_t)e * NPAR;
  float v;
  if (q < PW2) {
    const int o = q / INP, c = q % INP;
    v = c < IN ? P[OW1 + o * IN + c] : 0.0f;
  } else if (q < PW2T) {
    v = P[OW2 + (q - PW2)];
  } else if (q < PW3) {
    const int r = (q - PW2T) / HID, c = (q - PW2T) % HID;  // W2T[in][out] = W2[out][in]
    v = P[OW2 + c * HID + r];
  } else if (q < PW3T) {
    const int o = (q - PW3) / HID, c = (q - PW3) % HID;
    v = o < OUT ? P[OW3 + o * HID + c] : 0.0f;
  } else {
    const int r = (q - PW3T) / OUTP, c = (q - PW3T) % OUTP;  // W3T[in][out]
    v = c < OUT ? P[OW3 + c * HID + r] : 0.0f;
  }
  pack[gidx] = (__bf16)v;
  if (q < NBIAS) {
    float b;
    if (q < HID) b = P[OB1 + q];
    else if (q < 2 * HID) b = P[OB2 + q - HID];
    else b = (q - 2 * HID) < OUT ? P[OB3 + q - 2 * HID] : 0.0f;
    bias[(size_t)e * NBIAS + q] = b;
  }
}

thread_local std::string g_mlp_error;

int mdev_error(hipError_t e, const char* what) {
  g_mlp_error = std::string(what) + ": " + hipGetErrorString(e);
  return LBM_EDEVICE;
}
#define MLP_CK(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return mdev_error(e_, #expr); \
  } while (0)

// splitmix64 (Steele, Lea & Flood 2014) for the initial weights
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// ---- Forward pass without allocation ---------------------------------------
// lbm_mlp_forward_noalloc packs the caller's FP32 parameters into this
// library-owned buffer (the BF16 copies the matrix cores read, then the
// padded FP32 biases) and runs the forward kernel from there.  Each GPU the
// library runs on holds its own copy until the process ends; host code uses
// the per-device address from hipGetSymbolAddress, never the symbol itself.
constexpr int NOALLOC_MAX_E = 16;
constexpr int NOALLOC_MAX_N = 1 << 26;
constexpr size_t NOALLOC_PACK_BYTES = (size_t)NOALLOC_MAX_E * NPACK * sizeof(__bf16);
constexpr size_t NOALLOC_BYTES = NOALLOC_PACK_BYTES + (size_t)NOALLOC_MAX_E * NBIAS * sizeof(float);
static_assert(NOALLOC_PACK_BYTES % 256 == 0, "the bias block must stay 256-byte aligned");
static_assert(NOALLOC_MAX_E == LBM_MLP_NOALLOC_MAX_ENSEMBLE, "header limit");
static __device__ __align__(256) char scratch[NOALLOC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_on_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return mdev_error(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) {
    g_mlp_error = "device ordinal beyond the library's table of scratch addresses";
    return LBM_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return mdev_error(e, "hipGetSymbolAddress(scratch)");
    if (!p) {
      g_mlp_error = "hipGetSymbolAddress(scratch) returned no address";
      return LBM_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

}  // namespace

struct lbm_mlp {
  int E, max_batch, np_max, nchunks_max, nwaves_max;
  hipStream_t stream;
  float *master, *m1, *m2, *grad, *bias, *wpart, *bpart, *lpart;
  __bf16 *pack, *Xg, *H1g, *H2g, *dYg, *dZ1g, *dZ2g;
  int64_t t;  // Adam step count
  std::vector<float> host_l;
};

namespace {

int pack_all(lbm_mlp* m) {
  const int total = m->E * NPACK;
  hipLaunchKernelGGL(k_mlp_pack, dim3((total + 255) / 256), dim3(256), 0, m->stream, m->master, m->pack, m->bias,
                     m->E);
  MLP_CK(hipGetLastError());
  return LBM_OK;
}

int np_of(int n) { return (n + KCHUNK - 1) / KCHUNK * KCHUNK; }

// Forward + backward rows and the weight-gradient partials for a batch.
int run_grad(lbm_mlp* m, const float* x, const float* t, const float* mask, int n, const float* w) {
  RowsArgs a{};
  a.x = x;
  a.t = t;
  a.mask = mask;
  a.pack = m->pack;
  a.bias = m->bias;
  a.Xg = m->Xg;
  a.H1g = m->H1g;
  a.H2g = m->H2g;
  a.dYg = m->dYg;
  a.dZ1g = m->dZ1g;
  a.dZ2g = m->dZ2g;
  a.bpart = m->bpart;
  a.lpart = m->lpart;
  a.n = n;
  a.np = np_of(n);
  a.w0 = w ? w[0] : 1.0f;
  a.w1 = w ? w[1] : 1.0f;
  a.w2 = w ? w[2] : 1.0f;
  const int nblk = a.np / SAMPLES_PER_BLOCK;
  hipLaunchKernelGGL(k_mlp_rows<true>, dim3(nblk, m->E), dim3(256), 0, m->stream, a);
  MLP_CK(hipGetLastError());
  WgradArgs g{m->Xg, m->H1g, m->H2g, m->dYg, m->dZ1g, m->dZ2g, m->wpart, a.np, a.np / KCHUNK};
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(g.nchunks, 3, m->E), dim3(256), 0, m->stream, g);
  MLP_CK(hipGetLastError());
  return LBM_OK;
}

int run_update(lbm_mlp* m, int n, bool update, float lr) {
  const int np = np_of(n);
  UpdateArgs u{};
  u.master = m->master;
  u.m1 = m->m1;
  u.m2 = m->m2;
  u.grad = m->grad;
  u.wpart = m->wpart;
  u.bpart = m->bpart;
  u.nchunks = np / KCHUNK;
  u.nwaves = np / 32;
  u.update = update ? 1 : 0;
  u.lr = lr;
  u.b1 = 0.9f;
  u.b2 = 0.999f;
  u.eps = 1e-8f;
  if (update) {
    m->t += 1;
    u.c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)m->t)));
    u.c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)m->t)));
  }
  const int total = m->E * NPAR;
  hipLaunchKernelGGL(k_mlp_update, dim3((total + 255) / 256), dim3(256), 0, m->stream, u, m->E);
  MLP_CK(hipGetLastError());
  if (update) return pack_all(m);
  return LBM_OK;
}

// Loss per member from the per-wavefront partials (host, fixed order).
int read_loss(lbm_mlp* m, int n, double* out) {
  const int nw = np_of(n) / 32;
  m->host_l.resize((size_t)m->E * nw);
  MLP_CK(hipMemcpyAsync(m->host_l.data(), m->lpart, sizeof(float) * m->E * nw, hipMemcpyDeviceToHost, m->stream));
  MLP_CK(hipStreamSynchronize(m->stream));
  for (int e = 0; e < m->E; ++e) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += m->host_l[(size_t)e * nw + w];
    out[e] = s;
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_mlp_param_count(void) { return NPAR; }

int lbm_mlp_create(int32_t ensemble, uint64_t seed, int32_t max_batch, void* hip_stream, lbm_mlp** out) {
  if (!out || ensemble < 1 || ensemble > 64 || max_batch < 1 || max_batch > (1 << 22)) return LBM_EINVAL;
  *out = nullptr;
  lbm_mlp* m = new (std::nothrow) lbm_mlp();
  if (!m) return LBM_ENOMEM;
  m->E = ensemble;
  m->max_batch = max_batch;
  m->np_max = np_of(max_batch);
  m->stream = (hipStream_t)hip_stream;
  m->t = 0;
  const size_t E = ensemble, np = m->np_max;
  struct Buf {
    void** p;
    size_t bytes;
  } bufs[] = {
      {(void**)&m->master, E * NPAR * 4}, {(void**)&m->m1, E * NPAR * 4},          {(void**)&m->m2, E * NPAR * 4},
      {(void**)&m->grad, E * NPAR * 4},   {(void**)&m->bias, E * NBIAS * 4},       {(void**)&m->pack, E * NPACK * 2},
      {(void**)&m->Xg, E * np * INP * 2}, {(void**)&m->H1g, E * np * HID * 2},     {(void**)&m->H2g, E * np * HID * 2},
      {(void**)&m->dYg, E * np * OUTP * 2}, {(void**)&m->dZ1g, E * np * HID * 2}, {(void**)&m->dZ2g, E * np * HID * 2},
      {(void**)&m->wpart, E * (np / KCHUNK) * NGW * 4}, {(void**)&m->bpart, E * (np / 32) * NBIAS * 4},
      {(void**)&m->lpart, E * (np / 32) * 4},
  };
  for (auto& b : bufs) *b.p = nullptr;
  for (auto& b : bufs)
    if (hipMalloc(b.p, b.bytes) != hipSuccess) {
      g_mlp_error = "hipMalloc of the network buffers failed";
      lbm_mlp_destroy(m);
      return LBM_ENOMEM;
    }
  // He-uniform weights (bound sqrt(6 / fan_in)), zero biases, per member from seed + member
  std::vector<float> h(E * NPAR, 0.0f);
  for (size_t e = 0; e < E; ++e) {
    uint64_t s = seed + 0x632be59bd9b4e019ull * (e + 1);
    auto uni = [&]() { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); };
    float* P = h.data() + e * NPAR;
    const double b1 = std::sqrt(6.0 / IN), b2 = std::sqrt(6.0 / HID);
    for (int q = 0; q < HID * IN; ++q) P[OW1 + q] = (float)((2.0 * uni() - 1.0) * b1);
    for (int q = 0; q < HID * HID; ++q) P[OW2 + q] = (float)((2.0 * uni() - 1.0) * b2);
    for (int q = 0; q < OUT * HID; ++q) P[OW3 + q] = (float)((2.0 * uni() - 1.0) * b2);
  }
  int rc = lbm_mlp_set_params(m, h.data(), h.size());
  if (rc) {
    lbm_mlp_destroy(m);
    return rc;
  }
  *out = m;
  return LBM_OK;
}

int lbm_mlp_set_params(lbm_mlp* m, const float* host, size_t count) {
  if (!m || !host || count != (size_t)m->E * NPAR) return LBM_EINVAL;
  MLP_CK(hipMemcpyAsync(m->master, host, count * 4, hipMemcpyHostToDevice, m->stream));
  MLP_CK(hipMemsetAsync(m->m1, 0, count * 4, m->stream));
  MLP_CK(hipMemsetAsync(m->m2, 0, count * 4, m->stream));
  m->t = 0;
  int rc = pack_all(m);
  if (rc) return rc;
  MLP_CK(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

int lbm_mlp_get_params(lbm_mlp* m, float* host, size_t count) {
  if (!m || !host || count != (size_t)m->E * NPAR) return LBM_EINVAL;
  MLP_CK(hipMemcpyAsync(host, m->master, count * 4, hipMemcpyDeviceToHost, m->stream));
  MLP_CK(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

int lbm_mlp_forward(lbm_mlp* m, const float* d_x, int32_t n, float* d_y) {
  if (!m || !d_x || !d_y || n < 1) return LBM_EINVAL;
  RowsArgs a{};
  a.x = d_x;
  a.y = d_y;
  a.pack = m->pack;
  a.bias = m->bias;
  a.n = n;
  a.np = np_of(n);
  hipLaunchKernelGGL(k_mlp_rows<false>, dim3((n + SAMPLES_PER_BLOCK - 1) / SAMPLES_PER_BLOCK, m->E), dim3(256), 0,
                     m->stream, a);
  MLP_CK(hipGetLastError());
  return LBM_OK;
}

int lbm_mlp_forward_noalloc(const float* d_params, int32_t ensemble, const float* d_x, int32_t n, float* d_y,
                            void* hip_stream) {
  if (!d_params || !d_x || !d_y || n < 1) return LBM_EINVAL;
  if (ensemble < 1 || ensemble > NOALLOC_MAX_E || n > NOALLOC_MAX_N) {
    g_mlp_error = "lbm_mlp_forward_noalloc: ensemble must be 1.." + std::to_string(NOALLOC_MAX_E) +
                  " and n at most " + std::to_string(NOALLOC_MAX_N) + " (the static buffer's limits)";
    return LBM_EINVAL;
  }
  void* base = nullptr;
  int rc = scratch_on_current_device(&base);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  __bf16* pack = (__bf16*)base;
  float* bias = (float*)((char*)base + NOALLOC_PACK_BYTES);
  // every packed value and bias of members 0..ensemble-1 is rewritten here,
  // so nothing left by an earlier call is read
  const int total = ensemble * NPACK;
  hipLaunchKernelGGL(k_mlp_pack, dim3((total + 255) / 256), dim3(256), 0, st, d_params, pack, bias, (int)ensemble);
  MLP_CK(hipGetLastError());
  RowsArgs a{};
  a.x = d_x;
  a.y = d_y;
  a.pack = pack;
  a.bias = bias;
  a.n = n;
  a.np = np_of(n);
  hipLaunchKernelGGL(k_mlp_rows<false>, dim3((n + SAMPLES_PER_BLOCK - 1) / SAMPLES_PER_BLOCK, ensemble), dim3(256), 0,
                     st, a);
  MLP_CK(hipGetLastError());
  return LBM_OK;
}

int lbm_mlp_gradient(lbm_mlp* m, const float* d_x, const float* d_t, const float* d_mask, int32_t n,
                     const float* w3, float* host_grad, double* host_loss) {
  if (!m || !d_x || !d_t || !d_mask || n < 1 || n > m->max_batch || !host_grad || !host_loss) return LBM_EINVAL;
  int rc = run_grad(m, d_x, d_t, d_mask, n, w3);
  if (!rc) rc = run_update(m, n, false, 0.0f);
  if (rc) return rc;
  MLP_CK(hipMemcpyAsync(host_grad, m->grad, sizeof(float) * m->E * NPAR, hipMemcpyDeviceToHost, m->stream));
  return read_loss(m, n, host_loss);
}

int lbm_mlp_train(lbm_mlp* m, const float* d_x, const float* d_t, const float* d_mask, int32_t n, const float* w3,
                  float lr, int32_t steps, double* host_loss) {
  if (!m || !d_x || !d_t || !d_mask || n < 1 || n > m->max_batch || steps < 1 || !(lr > 0.0f) || !host_loss)
    return LBM_EINVAL;
  for (int s = 0; s < steps; ++s) {
    int rc = run_grad(m, d_x, d_t, d_mask, n, w3);
    if (!rc) rc = run_update(m, n, true, lr);
    if (rc) return rc;
  }
  return read_loss(m, n, host_loss);  // loss before the last update
}

const char* lbm_mlp_last_error(void) { return g_mlp_error.c_str(); }

void lbm_mlp_destroy(lbm_mlp* m) {
  if (!m) return;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  void* ptrs[] = {m->master, m->m1, m->m2, m->grad, m->bias, m->pack, m->Xg, m->H1g,
                  m->H2g,    m->dYg, m->dZ1g, m->dZ2g, m->wpart, m->bpart, m->lpart};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete m;
}

}  // extern "C"
