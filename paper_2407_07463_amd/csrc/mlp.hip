// Learned curvature: a multilayer perceptron 27 (zero-padded to 32) -> 128
// -> 128 -> 1 with ReLU on canonicalised 3x3x3 volume-fraction stencils,
// predicting kappa*Delta; its training step (forward, backward, Adam); and
// curvature that uses it with height functions as the fallback.
//
// The paper computes curvature with the single-tracer method (height
// functions); the network is an addition of this library. Arithmetic: the
// matrix products (layers 1 and 2 forward; dH1, dW2, dW1 backward) run on the
// matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation) with BF16
// operands: weights are FP32 masters rounded to nearest even for each use,
// the first-layer activations and the upstream gradients are rounded to BF16,
// and every input value x enters as two BF16 numbers hi = bf16(x),
// lo = bf16(x - hi) multiplied by the same weights (about 16 significant
// bits). The last layer (128 -> 1) is an FP32 dot product of the unrounded
// second-layer activations with the FP32 W3. Biases, loss and Adam in FP32.
// ReLU'(z) is (activation > 0). Batch reductions go through per-tile partial
// sums added in a fixed order, so every result is reproducible bit for bit.
//
// MFMA fragment layout (16x16x32, one wavefront): lane l holds
//   A[l%16][8*(l/16) + e], B[8*(l/16) + e][l%16] for e = 0..7 (bf16), and
//   D[4*(l/16) + r][l%16] for r = 0..3 (fp32).
//
// Per-sample activation record (bytes): h1 as BF16 [128] at 0, h2 as FP32
// [128] at 256 (768 in all). Training trace adds dL/dz2 and dL/dz1 as BF16
// [128] at 768 and 1024 (1280 in all).
#include <cstring>

#include "common.hpp"
#include "compact.hpp"
#include "curv_hf.hpp"
#include "plic.hpp"

namespace {

// Sum of each row of 16 lanes, received by every lane of the row, with the
// additions of the butterfly v + v[lane ^ 8], ^ 4, ^ 2, ^ 1 in the same order
// and on the same operands: after each step the partial sums repeat with the
// step's period, so rotating the row by the step reads the value the
// butterfly would. DPP row rotations (row_ror:8, 4, 2, 1) instead of LDS
// permutes. Every lane of the wavefront must be active.
__device__ __forceinline__ float row16_sum(float v) {
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xf, 0xf, false));
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x122, 0xf, 0xf, false));
  v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x121, 0xf, 0xf, false));
  return v;
}

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int NIN = 32, NH = 128;
constexpr int OFF_W1 = 0, OFF_B1 = NIN * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NH, NPARAMS = OFF_B3 + 4;
static_assert(NPARAMS == VOFMT_MLP_NPARAMS, "parameter layout");

constexpr int TILE = 64;  // samples per tile
constexpr int XP = 40;    // LDS row pitches (bf16 elements), padded against bank conflicts
constexpr int HP = 136;
constexpr int TP = 72;

// FP32 -> BF16, round to nearest even (the conversion instruction of gfx950).
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  const __bf16 h = (__bf16)f;
  uint16_t u;
  memcpy(&u, &h, 2);
  return u;
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// 8 consecutive bf16 (16 bytes, 16-byte aligned) as an MFMA operand
__device__ __forceinline__ bf16x8 frag(const uint16_t *p) {
  const uint4 v = *reinterpret_cast<const uint4 *>(p);
  bf16x8 r;
  memcpy(&r, &v, 16);
  return r;
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

constexpr int ACT_BYTES = 768, TRACE_BYTES = 1280;

// BF16 copies of the weights for one call: W1^T [128][32], W2^T [128][128],
// W2 [128][128] (for the backward product).
__global__ void k_mlp_prep(const float *__restrict__ P, uint16_t *__restrict__ w1t, uint16_t *__restrict__ w2t,
                           uint16_t *__restrict__ w2n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NIN * NH) {
    const int k = i / NH, j = i % NH;
    w1t[j * NIN + k] = bf16_bits(P[OFF_W1 + i]);
  }
  if (i < NH * NH) {
    const int k = i / NH, j = i % NH;
    const uint16_t b = bf16_bits(P[OFF_W2 + i]);
    w2t[j * NH + k] = b;
    w2n[i] = b;
  }
}

__device__ __forceinline__ uint16_t *act_h1(uint8_t *rec, int64_t s, int stride) {
  return reinterpret_cast<uint16_t *>(rec + s * stride);
}
__device__ __forceinline__ float *act_h2(uint8_t *rec, int64_t s, int stride) {
  return reinterpret_cast<float *>(rec + s * stride + 256);
}

// Forward pass, persistent over 64-sample tiles. acts (nullable): the
// activation records. With a target, also the upstream gradient g = dL/dy of
// every sample and the loss of every tile.
__global__ __launch_bounds__(256) void k_mlp_fwd(const float *__restrict__ P, const uint16_t *__restrict__ w1t_g,
                                                 const uint16_t *__restrict__ w2t_g, int m,
                                                 const float *__restrict__ x, float *__restrict__ y,
                                                 uint8_t *__restrict__ acts, const float *__restrict__ tgt,
                                                 float *__restrict__ g_out, float *__restrict__ loss_part) {
  __shared__ __attribute__((aligned(16))) uint16_t W1s[NH][XP];
  __shared__ __attribute__((aligned(16))) uint16_t W2s[NH][HP];
  __shared__ __attribute__((aligned(16))) uint16_t Xh[TILE][XP];
  __shared__ __attribute__((aligned(16))) uint16_t Xl[TILE][XP];
  __shared__ __attribute__((aligned(16))) uint16_t H1s[TILE][HP];
  __shared__ float b1s[NH], b2s[NH], w3s[NH];
  __shared__ float ypart[4][TILE];
  __shared__ float lpart[TILE];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < NH * NIN; i += 256) W1s[i / NIN][i % NIN] = w1t_g[i];
  for (int i = tid; i < NH * NH; i += 256) W2s[i / NH][i % NH] = w2t_g[i];
  for (int i = tid; i < NH; i += 256) {
    b1s[i] = P[OFF_B1 + i];
    b2s[i] = P[OFF_B2 + i];
    w3s[i] = P[OFF_W3 + i];
  }
  const float b3 = P[OFF_B3];
  const int ntiles = (m + TILE - 1) / TILE;
  const int lr = lane & 15, lq = lane >> 4;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int s0 = tile * TILE;
    __syncthreads();
    for (int i = tid; i < TILE * NIN; i += 256) {
      const int s = i / NIN, k = i % NIN;
      const float v = (k < 27 && s0 + s < m) ? x[(int64_t)(s0 + s) * 27 + k] : 0.0f;
      const uint16_t hi = bf16_bits(v);
      Xh[s][k] = hi;
      Xl[s][k] = bf16_bits(v - bf16_val(hi));
    }
    __syncthreads();
    // layer 1: wave w owns output columns [32w, 32w+32)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int jn = 0; jn < 2; ++jn) {
        const int nt = 2 * w + jn;
        const bf16x8 wf = frag(&W1s[16 * nt + lr][8 * lq]);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(frag(&Xh[16 * mt + lr][8 * lq]), wf, acc);
        acc = mfma(frag(&Xl[16 * mt + lr][8 * lq]), wf, acc);
        const int col = 16 * nt + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * mt + 4 * lq + r;
          const float z = acc[r] + b1s[col];
          const uint16_t h = bf16_bits(z > 0.0f ? z : 0.0f);
          H1s[row][col] = h;
          if (acts && s0 + row < m) act_h1(acts, s0 + row, ACT_BYTES)[col] = h;
        }
      }
    __syncthreads();
    // layer 2 and the layer-3 partial products
    float yp[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) yp[mt][r] = 0.0f;
#pragma unroll
    for (int jn = 0; jn < 2; ++jn) {
      const int nt = 2 * w + jn;
      const int col = 16 * nt + lr;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < NH; kk += 32)
          acc = mfma(frag(&H1s[16 * mt + lr][kk + 8 * lq]), frag(&W2s[16 * nt + lr][kk + 8 * lq]), acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * mt + 4 * lq + r;
          const float z = acc[r] + b2s[col];
          const float h = z > 0.0f ? z : 0.0f;
          if (acts && s0 + row < m) act_h2(acts, s0 + row, ACT_BYTES)[col] = h;
          yp[mt][r] = yp[mt][r] + h * w3s[col];
        }
      }
    }
    // sum the 16 columns of each row across lanes (fixed tree)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = yp[mt][r];
        v = row16_sum(v);
        if (lr == 0) ypart[w][16 * mt + 4 * lq + r] = v;
      }
    __syncthreads();
    if (tid < TILE) {
      const int s = s0 + tid;
      float lv = 0.0f;
      if (s < m) {
        const float yy = (((ypart[0][tid] + ypart[1][tid]) + ypart[2][tid]) + ypart[3][tid]) + b3;
        if (y) y[s] = yy;
        if (tgt) {
          const float t = tgt[s];
          const float a = fabsf(t) > 0.05f ? fabsf(t) : 0.05f;
          const float wgt = 1.0f / (a * a);
          const float d = yy - t;
          lv = (d * d) * wgt;
          g_out[s] = ((2.0f * d) * wgt) / (float)m;
        }
      }
      lpart[tid] = lv;
    }
    if (tgt) {
      __syncthreads();
      if (tid == 0) {
        float acc = 0.0f;
        for (int i = 0; i < TILE; ++i) acc += lpart[i];
        loss_part[tile] = acc;
      }
    }
  }
}

// Backward pass of one 64-sample tile: per-tile partial gradients of every
// parameter (added later in a fixed order). trace (nullable): the training
// records of the tile's samples.
__global__ __launch_bounds__(256) void k_mlp_bwd(const float *__restrict__ P, const uint16_t *__restrict__ w2n_g,
                                                 int m, const float *__restrict__ x, uint8_t *__restrict__ acts,
                                                 const float *__restrict__ g, float *__restrict__ partial,
                                                 uint8_t *__restrict__ trace) {
  __shared__ __attribute__((aligned(16))) uint16_t XTh[NIN][TP];
  __shared__ __attribute__((aligned(16))) uint16_t XTl[NIN][TP];
  __shared__ __attribute__((aligned(16))) uint16_t H1T[NH][TP];
  __shared__ __attribute__((aligned(16))) uint16_t D2[TILE][HP];
  __shared__ __attribute__((aligned(16))) uint16_t D2T[NH][TP];
  __shared__ __attribute__((aligned(16))) uint16_t D1T[NH][TP];
  __shared__ float gs[TILE];
  __shared__ float w3s[NH];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int tile = blockIdx.x, s0 = tile * TILE;
  float *part = partial + (int64_t)tile * NPARAMS;
  if (tid < TILE) gs[tid] = (s0 + tid < m) ? g[s0 + tid] : 0.0f;
  if (tid < NH) w3s[tid] = P[OFF_W3 + tid];
  for (int i = tid; i < TILE * NIN; i += 256) {
    const int s = i / NIN, k = i % NIN;
    const float v = (k < 27 && s0 + s < m) ? x[(int64_t)(s0 + s) * 27 + k] : 0.0f;
    const uint16_t hi = bf16_bits(v);
    XTh[k][s] = hi;
    XTl[k][s] = bf16_bits(v - bf16_val(hi));
  }
  for (int i = tid; i < TILE * NH; i += 256) {
    const int s = i / NH, k = i % NH;
    H1T[k][s] = (s0 + s < m) ? act_h1(acts, s0 + s, ACT_BYTES)[k] : (uint16_t)0;
  }
  __syncthreads();
  // dZ2 = bf16((h2 > 0) * g * W3)
  for (int i = tid; i < TILE * NH; i += 256) {
    const int s = i / NH, k = i % NH;
    const float h2 = (s0 + s < m) ? act_h2(acts, s0 + s, ACT_BYTES)[k] : 0.0f;
    const float d = (h2 > 0.0f) ? gs[s] * w3s[k] : 0.0f;
    const uint16_t b = bf16_bits(d);
    D2[s][k] = b;
    D2T[k][s] = b;
    if (trace && s0 + s < m) reinterpret_cast<uint16_t *>(trace + (int64_t)(s0 + s) * TRACE_BYTES + 768)[k] = b;
  }
  __syncthreads();
  // dH1 = dZ2 . W2^T; dZ1 = bf16((h1 > 0) * dH1); wave w owns hidden units [32w, 32w+32)
#pragma unroll
  for (int jn = 0; jn < 2; ++jn) {
    const int nt = 2 * w + jn;
    const int col = 16 * nt + lr;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < NH; kk += 32)
        acc = mfma(frag(&D2[16 * mt + lr][kk + 8 * lq]), frag(&w2n_g[(16 * nt + lr) * NH + kk + 8 * lq]), acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * mt + 4 * lq + r;
        const float h1 = bf16_val(H1T[col][row]);
        const uint16_t b = bf16_bits(h1 > 0.0f ? acc[r] : 0.0f);
        D1T[col][row] = b;
        if (trace && s0 + row < m)
          reinterpret_cast<uint16_t *>(trace + (int64_t)(s0 + row) * TRACE_BYTES + 1024)[col] = b;
      }
    }
  }
  __syncthreads();
  // dW2 = H1^T . dZ2 (128 x 128, K = 64 samples)
#pragma unroll
  for (int jn = 0; jn < 2; ++jn) {
    const int nt = 2 * w + jn;
    const int col = 16 * nt + lr;
    for (int mt = 0; mt < 8; ++mt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < TILE; kk += 32)
        acc = mfma(frag(&H1T[16 * mt + lr][kk + 8 * lq]), frag(&D2T[16 * nt + lr][kk + 8 * lq]), acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) part[OFF_W2 + (16 * mt + 4 * lq + r) * NH + col] = acc[r];
    }
  }
  // dW1 = X^T . dZ1 (32 x 128, K = 64 samples), X as hi + lo
#pragma unroll
  for (int jn = 0; jn < 2; ++jn) {
    const int nt = 2 * w + jn;
    const int col = 16 * nt + lr;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < TILE; kk += 32) {
        const bf16x8 d1 = frag(&D1T[16 * nt + lr][kk + 8 * lq]);
        acc = mfma(frag(&XTh[16 * mt + lr][kk + 8 * lq]), d1, acc);
        acc = mfma(frag(&XTl[16 * mt + lr][kk + 8 * lq]), d1, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) part[OFF_W1 + (16 * mt + 4 * lq + r) * NH + col] = acc[r];
    }
  }
  // dW3, the biases, and the padding, as sequential FP32 sums over the tile
  if (tid < NH) {
    const int k = tid;
    float a3 = 0.0f, a2 = 0.0f, a1 = 0.0f;
    for (int s = 0; s < TILE; ++s) {
      const float h2 = (s0 + s < m) ? act_h2(acts, s0 + s, ACT_BYTES)[k] : 0.0f;
      a3 = a3 + gs[s] * h2;
      a2 = a2 + bf16_val(D2T[k][s]);
      a1 = a1 + bf16_val(D1T[k][s]);
    }
    part[OFF_W3 + k] = a3;
    part[OFF_B2 + k] = a2;
    part[OFF_B1 + k] = a1;
  } else if (tid == NH) {
    float a = 0.0f;
    for (int s = 0; s < TILE; ++s) a = a + gs[s];
    part[OFF_B3] = a;
    part[OFF_B3 + 1] = 0.0f;
    part[OFF_B3 + 2] = 0.0f;
    part[OFF_B3 + 3] = 0.0f;
  }
  if (trace) {
    // the activation records of the tile, copied word by word
    for (int i = tid; i < TILE * (ACT_BYTES / 4); i += 256) {
      const int s = i / (ACT_BYTES / 4), q = i % (ACT_BYTES / 4);
      if (s0 + s < m)
        reinterpret_cast<uint32_t *>(trace + (int64_t)(s0 + s) * TRACE_BYTES)[q] =
            reinterpret_cast<const uint32_t *>(acts + (int64_t)(s0 + s) * ACT_BYTES)[q];
    }
  }
}

// Gradient = fixed-order sum of the tile partials; Adam on the FP32 masters.
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ P, float *__restrict__ Mo,
                                                  float *__restrict__ Vo, const float *__restrict__ partial, int ntiles,
                                                  int step, float lrate, float *__restrict__ grads,
                                                  const float *__restrict__ loss_part, float *__restrict__ loss_out,
                                                  int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NPARAMS) {
    float gsum = 0.0f;
    for (int t = 0; t < ntiles; ++t) gsum = gsum + partial[(int64_t)t * NPARAMS + i];
    if (grads) grads[i] = gsum;
    const float mm = 0.9f * Mo[i] + 0.1f * gsum;
    const float vv = 0.999f * Vo[i] + 0.001f * (gsum * gsum);
    Mo[i] = mm;
    Vo[i] = vv;
    // bias corrections 1 - beta^step, in FP64 so that small steps lose nothing
    const float c1 = (float)(1.0 - pow(0.9, (double)step)), c2 = (float)(1.0 - pow(0.999, (double)step));
    P[i] = P[i] - lrate * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
  }
  if (i == 0) {
    float l = 0.0f;
    for (int t = 0; t < ntiles; ++t) l = l + loss_part[t];
    loss_out[0] = l / (float)m;
  }
}

// ------------------------------------------------------------ stencils

// Canonical stencil of the cell (i, j, k), over the 48 symmetries of the
// cube and the exchange of the phases: when the centre exceeds 1/2 replace c
// by 1 - c (sign -1: the curvature changes sign); then reflect the axes along
// which the MYC normal of that block is negative and order the axes by
// increasing |m| (ties: lower axis first). Every canonical stencil has its
// centre at most 1/2 and a normal with non-negative ascending components.
// Its two steps, kept in registers (no arrays indexed at run time): the
// block of the cell (complemented when its centre exceeds 1/2; returns the
// sign), then the canonical position of every block entry, handed to `put`.
struct Canon {
  int o0, o1, o2;  // source axis of canonical axis 0, 1, 2
  int d0, d1, d2;  // and its direction (+1 or -1)
};

__device__ __forceinline__ void load_block(const double *__restrict__ c, int64_t p, int nx, int ny, int nz,
                                           double *b) {
  const int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((int64_t)nx * ny));
  const int xs[3] = {wrap_dec(i, nx), i, wrap_inc(i, nx)};
  const int ys[3] = {wrap_dec(j, ny), j, wrap_inc(j, ny)};
  const int zs[3] = {wrap_dec(k, nz), k, wrap_inc(k, nz)};
#pragma unroll
  for (int az = 0; az < 3; ++az)
#pragma unroll
    for (int ay = 0; ay < 3; ++ay)
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) b[ax + 3 * ay + 9 * az] = c[((int64_t)zs[az] * ny + ys[ay]) * nx + xs[ax]];
}

__device__ __forceinline__ int canonical_of_block(double *b, Canon &cn) {
  const int sign = (b[13] > 0.5) ? -1 : 1;
  if (sign < 0) {
#pragma unroll
    for (int q = 0; q < 27; ++q) b[q] = 1.0 - b[q];
  }
  double m0, m1, m2;
  plic::myc_normal(b, m0, m1, m2);
  auto mv = [&](int a) { return a == 0 ? m0 : (a == 1 ? m1 : m2); };
  int o0 = 0, o1 = 1, o2 = 2;
  auto order2 = [&](int &a, int &bb) {  // increasing |m|, ties to the lower axis
    if (fabs(mv(bb)) < fabs(mv(a)) || (fabs(mv(bb)) == fabs(mv(a)) && bb < a)) {
      const int t = a;
      a = bb;
      bb = t;
    }
  };
  order2(o0, o1);
  order2(o0, o2);
  order2(o1, o2);
  cn.o0 = o0;
  cn.o1 = o1;
  cn.o2 = o2;
  cn.d0 = (mv(o0) < 0.0) ? -1 : 1;
  cn.d1 = (mv(o1) < 0.0) ? -1 : 1;
  cn.d2 = (mv(o2) < 0.0) ? -1 : 1;
  return sign;
}

__device__ __forceinline__ int canonical_block(const double *__restrict__ c, int64_t p, int nx, int ny, int nz,
                                               double *b, Canon &cn) {
  load_block(c, p, nx, ny, nz, b);
  return canonical_of_block(b, cn);
}

// Entry a = (a0, a1, a2) of the block (offsets -1..1 along x, y, z) lands at
// canonical offsets q_k = d_k * a[o_k]: index (q0+1) + 3(q1+1) + 9(q2+1).
template <class Put>
__device__ __forceinline__ void canonical_scatter(const double *b, const Canon &cn, Put put) {
#pragma unroll
  for (int a2 = -1; a2 <= 1; ++a2)
#pragma unroll
    for (int a1 = -1; a1 <= 1; ++a1)
#pragma unroll
      for (int a0 = -1; a0 <= 1; ++a0) {
        auto along = [&](int o) { return o == 0 ? a0 : (o == 1 ? a1 : a2); };
        const int q0 = cn.d0 * along(cn.o0), q1 = cn.d1 * along(cn.o1), q2 = cn.d2 * along(cn.o2);
        put((q0 + 1) + 3 * (q1 + 1) + 9 * (q2 + 1), (float)b[(a0 + 1) + 3 * (a1 + 1) + 9 * (a2 + 1)]);
      }
}

// Canonical stencils of the listed cells: xs[q], sign[q] for cell list[q].
__global__ __launch_bounds__(256) void k_stencil_list(const double *__restrict__ c, int nx, int ny, int nz,
                                                      const int32_t *__restrict__ list, int n, float *__restrict__ xs,
                                                      int8_t *__restrict__ sgn) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int64_t p = list[q];
  double b[27];
  Canon cn;
  const int sg = canonical_block(c, p, nx, ny, nz, b, cn);
  float *row = xs + (int64_t)q * 27;
  canonical_scatter(b, cn, [&](int e, float v) { row[e] = v; });
  sgn[q] = (int8_t)sg;
}

// Height functions on the fallback cells: their value where valid (status
// 1..3), else the network's value stays (status 4 + 8).
__global__ __launch_bounds__(256) void k_curv_fallback(const double *__restrict__ c, int nx, int ny, int nz,
                                                       const int32_t *__restrict__ hf_list,
                                                       const int32_t *__restrict__ hf_count,
                                                       double *__restrict__ kappa, uint8_t *__restrict__ status) {
  const int n = *hf_count;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const int64_t p = hf_list[q];
    double k;
    uint8_t st;
    curv::hf_cell(c, p, nx, ny, nz, k, st);
    if (st >= 1 && st <= 3) {
      kappa[p] = k;
      status[p] = st;
    } else {
      status[p] = (uint8_t)(st | 8);
    }
  }
}

// Learned curvature of the listed mixed cells in one pass (persistent): each
// wavefront takes tiles of 32 cells on its own -- stencil gather and
// canonicalisation (one lane per cell), both matrix-core layers in its own LDS
// slice, the FP32 last layer -- and writes kappa = sign * y with status 8,
// appending cells with |kappa| < kappa_lo to the fallback list. No block
// barrier after the weights are staged. The arithmetic and the order of every
// sum are those of k_mlp_fwd, so y is bit-identical to vofmt_mlp_forward on
// the same stencils.
constexpr int FT = 32;     // cells per wavefront tile
constexpr int FWAVES = 8;  // wavefronts per workgroup

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64 * FWAVES) void k_curv_fused(
    const float *__restrict__ P, const uint16_t *__restrict__ w1t_g, const uint16_t *__restrict__ w2t_g,
    const double *__restrict__ c, int nx, int ny, int nz, const int32_t *__restrict__ list, int nm, double kappa_lo,
    double *__restrict__ kappa, uint8_t *__restrict__ status, int32_t *__restrict__ hf_list,
    int32_t *__restrict__ hf_count) {
  __shared__ __attribute__((aligned(16))) uint16_t W1s[NH][XP];
  __shared__ __attribute__((aligned(16))) uint16_t W2s[NH][HP];
  __shared__ __attribute__((aligned(16))) uint16_t Xh[FWAVES][FT][XP];
  __shared__ __attribute__((aligned(16))) uint16_t Xl[FWAVES][FT][XP];
  __shared__ __attribute__((aligned(16))) uint16_t H1[FWAVES][FT][HP];
  __shared__ float b1s[NH], b2s[NH], w3s[NH];
  __shared__ float yb[FWAVES][FT];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < NH * NIN; i += 64 * FWAVES) W1s[i / NIN][i % NIN] = w1t_g[i];
  for (int i = tid; i < NH * NH; i += 64 * FWAVES) W2s[i / NH][i % NH] = w2t_g[i];
  for (int i = tid; i < NH; i += 64 * FWAVES) {
    b1s[i] = P[OFF_B1 + i];
    b2s[i] = P[OFF_B2 + i];
    w3s[i] = P[OFF_W3 + i];
  }
  // padding inputs 27..31 stay zero
  for (int i = lane; i < FT * NIN; i += 64) {
    Xh[w][i / NIN][i % NIN] = 0;
    Xl[w][i / NIN][i % NIN] = 0;
  }
  const float b3 = P[OFF_B3];
  __syncthreads();
  const int lr = lane & 15, lq = lane >> 4;
  const int ntiles = (nm + FT - 1) / FT;
  for (int tile = blockIdx.x * FWAVES + w; tile < ntiles; tile += gridDim.x * FWAVES) {
    // ---- canonical stencils, one lane per cell
    const int q = tile * FT + lane;
    const bool own = lane < FT && q < nm;
    int sg = 1;
    int32_t p = 0;
    if (own) {
      p = list[q];
      double b[27];
      Canon cn;
      sg = canonical_block(c, p, nx, ny, nz, b, cn);
      canonical_scatter(b, cn, [&](int e, float v) {
        const uint16_t hi = bf16_bits(v);
        Xh[w][lane][e] = hi;
        Xl[w][lane][e] = bf16_bits(v - bf16_val(hi));
      });
    } else if (lane < FT) {
      for (int e = 0; e < 27; ++e) {
        Xh[w][lane][e] = 0;
        Xl[w][lane][e] = 0;
      }
    }
    wave_sync();
    // ---- layer 1: 32 rows x 128 columns
#pragma unroll
    for (int mt = 0; mt < FT / 16; ++mt)
#pragma unroll
      for (int nt = 0; nt < NH / 16; ++nt) {
        const bf16x8 wf = frag(&W1s[16 * nt + lr][8 * lq]);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(frag(&Xh[w][16 * mt + lr][8 * lq]), wf, acc);
        acc = mfma(frag(&Xl[w][16 * mt + lr][8 * lq]), wf, acc);
        const int col = 16 * nt + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float z = acc[r] + b1s[col];
          H1[w][16 * mt + 4 * lq + r][col] = bf16_bits(z > 0.0f ? z : 0.0f);
        }
      }
    wave_sync();
    // ---- layer 2 and the layer-3 partial products, summed per 32 columns as k_mlp_fwd does
    float yq[4][FT / 16][4];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int mt = 0; mt < FT / 16; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) yq[g][mt][r] = 0.0f;
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int jn = 0; jn < 2; ++jn) {
        const int nt = 2 * g + jn;
        const int col = 16 * nt + lr;
#pragma unroll
        for (int mt = 0; mt < FT / 16; ++mt) {
          f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kk = 0; kk < NH; kk += 32)
            acc = mfma(frag(&H1[w][16 * mt + lr][kk + 8 * lq]), frag(&W2s[16 * nt + lr][kk + 8 * lq]), acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float z = acc[r] + b2s[col];
            const float h = z > 0.0f ? z : 0.0f;
            yq[g][mt][r] = yq[g][mt][r] + h * w3s[col];
          }
        }
      }
    float ysum[FT / 16][4];
#pragma unroll
    for (int mt = 0; mt < FT / 16; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float part[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          float v = yq[g][mt][r];
          v = row16_sum(v);
          part[g] = v;
        }
        ysum[mt][r] = (((part[0] + part[1]) + part[2]) + part[3]) + b3;
      }
    if (lr == 0) {
#pragma unroll
      for (int mt = 0; mt < FT / 16; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) yb[w][16 * mt + 4 * lq + r] = ysum[mt][r];
    }
    wave_sync();
    // ---- kappa, status, fallback list
    bool flag = false;
    if (own) {
      const double kn = (double)sg * (double)yb[w][lane];
      kappa[p] = kn;
      status[p] = 8;
      flag = fabs(kn) < kappa_lo;
    }
    const uint64_t mask = __ballot(flag);
    if (mask) {
      int base = 0;
      if (lane == 0) base = atomicAdd(hf_count, (int)__popcll(mask));
      base = __shfl(base, 0, 64);
      if (flag) hf_list[base + __popcll(mask & ((1ull << lane) - 1))] = p;
    }
    wave_sync();  // the next tile overwrites this wavefront's LDS slice
  }
}

// Network outputs (and optionally activation records) of given inputs
// x[m][27], by the tile scheme of k_curv_fused: each wavefront takes tiles of
// FT samples on its own, their inputs read as one contiguous block, no block
// barrier after the weights are staged. The matrix-core sequences and the
// order of every sum are those of k_mlp_fwd, so the outputs and records are
// bit-identical to it.
__global__ __launch_bounds__(64 * FWAVES) void k_mlp_infer(const float *__restrict__ P,
                                                           const uint16_t *__restrict__ w1t_g,
                                                           const uint16_t *__restrict__ w2t_g, int m,
                                                           const float *__restrict__ x, float *__restrict__ y,
                                                           uint8_t *__restrict__ acts) {
  __shared__ __attribute__((aligned(16))) uint16_t W1s[NH][XP];
  __shared__ __attribute__((aligned(16))) uint16_t W2s[NH][HP];
  __shared__ __attribute__((aligned(16))) uint16_t Xh[FWAVES][FT][XP];
  __shared__ __attribute__((aligned(16))) uint16_t Xl[FWAVES][FT][XP];
  __shared__ __attribute__((aligned(16))) uint16_t H1[FWAVES][FT][HP];
  __shared__ float b1s[NH], b2s[NH], w3s[NH];
  __shared__ float yb[FWAVES][FT];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int i = tid; i < NH * NIN; i += 64 * FWAVES) W1s[i / NIN][i % NIN] = w1t_g[i];
  for (int i = tid; i < NH * NH; i += 64 * FWAVES) W2s[i / NH][i % NH] = w2t_g[i];
  for (int i = tid; i < NH; i += 64 * FWAVES) {
    b1s[i] = P[OFF_B1 + i];
    b2s[i] = P[OFF_B2 + i];
    w3s[i] = P[OFF_W3 + i];
  }
  // padding inputs 27..31 stay zero
  for (int i = lane; i < FT * NIN; i += 64) {
    Xh[w][i / NIN][i % NIN] = 0;
    Xl[w][i / NIN][i % NIN] = 0;
  }
  const float b3 = P[OFF_B3];
  __syncthreads();
  const int lr = lane & 15, lq = lane >> 4;
  const int ntiles = (m + FT - 1) / FT;
  // A tile's inputs are FT x 27 consecutive values, NV per lane; the next
  // tile's are loaded while the current one is computed.
  constexpr int NV = (FT * 27 + 63) / 64;
  float xv[NV];
  auto load_inputs = [&](int t) {
    const int s0 = t * FT;
    const int nvals = ((m - s0 < FT) ? m - s0 : FT) * 27;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int i = lane + 64 * q;
      xv[q] = (i < nvals) ? x[(int64_t)s0 * 27 + i] : 0.0f;
    }
  };
  const int tstride = gridDim.x * FWAVES;
  if (blockIdx.x * FWAVES + w < ntiles) load_inputs(blockIdx.x * FWAVES + w);
  for (int tile = blockIdx.x * FWAVES + w; tile < ntiles; tile += tstride) {
    const int s0 = tile * FT;
    // ---- the tile's inputs, split into hi + lo
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int i = lane + 64 * q;
      if (i < FT * 27) {
        const int sr = i / 27, k = i - 27 * sr;
        const uint16_t hi = bf16_bits(xv[q]);
        Xh[w][sr][k] = hi;
        Xl[w][sr][k] = bf16_bits(xv[q] - bf16_val(hi));
      }
    }
    wave_sync();
    if (tile + tstride < ntiles) load_inputs(tile + tstride);
    // ---- layer 1: FT rows x 128 columns
#pragma unroll
    for (int mt = 0; mt < FT / 16; ++mt)
#pragma unroll
      for (int nt = 0; nt < NH / 16; ++nt) {
        const bf16x8 wf = frag(&W1s[16 * nt + lr][8 * lq]);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma(frag(&Xh[w][16 * mt + lr][8 * lq]), wf, acc);
        acc = mfma(frag(&Xl[w][16 * mt + lr][8 * lq]), wf, acc);
        const int col = 16 * nt + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * mt + 4 * lq + r;
          const float z = acc[r] + b1s[col];
          const uint16_t h = bf16_bits(z > 0.0f ? z : 0.0f);
          H1[w][row][col] = h;
          if (acts && s0 + row < m) act_h1(acts, s0 + row, ACT_BYTES)[col] = h;
        }
      }
    wave_sync();
    // ---- layer 2 and the layer-3 partial products, summed per 32 columns as k_mlp_fwd does
    float yq[4][FT / 16][4];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int mt = 0; mt < FT / 16; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) yq[g][mt][r] = 0.0f;
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int jn = 0; jn < 2; ++jn) {
        const int nt = 2 * g + jn;
        const int col = 16 * nt + lr;
#pragma unroll
        for (int mt = 0; mt < FT / 16; ++mt) {
          f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kk = 0; kk < NH; kk += 32)
            acc = mfma(frag(&H1[w][16 * mt + lr][kk + 8 * lq]), frag(&W2s[16 * nt + lr][kk + 8 * lq]), acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * mt + 4 * lq + r;
            const float z = acc[r] + b2s[col];
            const float h = z > 0.0f ? z : 0.0f;
            if (acts && s0 + row < m) act_h2(acts, s0 + row, ACT_BYTES)[col] = h;
            yq[g][mt][r] = yq[g][mt][r] + h * w3s[col];
          }
        }
      }
#pragma unroll
    for (int mt = 0; mt < FT / 16; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float part[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          float v = yq[g][mt][r];
          v = row16_sum(v);
          part[g] = v;
        }
        if (lr == 0) yb[w][16 * mt + 4 * lq + r] = (((part[0] + part[1]) + part[2]) + part[3]) + b3;
      }
    wave_sync();
    if (lane < FT && s0 + lane < m) y[s0 + lane] = yb[w][lane];
    wave_sync();  // the next tile overwrites this wavefront's LDS slice
  }
}

}  // namespace

static int mlp_prepare(vofmt_ctx *ctx, const float *params, uint16_t **w, hipStream_t stream) {
  uint16_t *buf = (uint16_t *)scratch(ctx, SLOT_MLP_W, sizeof(uint16_t) * (NIN * NH + 2 * NH * NH));
  if (!buf) return VOFMT_E_NOMEM;
  w[0] = buf;                       // W1^T
  w[1] = buf + NIN * NH;            // W2^T
  w[2] = buf + NIN * NH + NH * NH;  // W2
  hipLaunchKernelGGL(k_mlp_prep, dim3(ceil_div(NH * NH, 256)), dim3(256), 0, stream, params, w[0], w[1], w[2]);
  return hip_check(ctx, hipGetLastError(), "k_mlp_prep");
}

static int fwd_grid(vofmt_ctx *ctx, int ntiles) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1)
    cus = 256;
  const int g = 2 * cus;  // two 70 KB-LDS workgroups fit one compute unit
  return ntiles < g ? ntiles : g;
}

extern "C" int vofmt_mlp_forward(vofmt_ctx *ctx, const float *params, int32_t m, const float *x, float *y,
                                 uint8_t *acts, hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (m < 0 || !params || (m > 0 && (!x || !y)))
    return set_err(ctx, VOFMT_E_ARG, "vofmt_mlp_forward: bad arguments");
  if (m == 0) return VOFMT_OK;
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  uint16_t *w[3];
  int rc = mlp_prepare(ctx, params, w, stream);
  if (rc) return rc;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1)
    cus = 256;
  const int ftiles = (m + FT - 1) / FT;
  const int fgrid = ftiles < cus * FWAVES ? (ftiles + FWAVES - 1) / FWAVES : cus;
  const int rec = prof_begin(ctx, "k_mlp_infer", stream);
  hipLaunchKernelGGL(k_mlp_infer, dim3(fgrid), dim3(64 * FWAVES), 0, stream, params, w[0], w[1], m, x, y, acts);
  prof_end(ctx, rec, stream);
  return hip_check(ctx, hipGetLastError(), "k_mlp_infer");
}

extern "C" int vofmt_mlp_train_step(vofmt_ctx *ctx, float *params, float *adam_m, float *adam_v, int32_t step,
                                    float lr, int32_t m, const float *x, const float *y_target, float *grads,
                                    uint8_t *trace, float *loss_host, hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (m < 1 || step < 1 || !params || !adam_m || !adam_v || !x || !y_target || !loss_host || !(lr >= 0.0f))
    return set_err(ctx, VOFMT_E_ARG, "vofmt_mlp_train_step: bad arguments");
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  uint16_t *w[3];
  int rc = mlp_prepare(ctx, params, w, stream);
  if (rc) return rc;
  const int ntiles = (m + TILE - 1) / TILE;
  uint8_t *acts = (uint8_t *)scratch(ctx, SLOT_MLP_ACTS, (size_t)ACT_BYTES * (size_t)m);
  float *gbuf = (float *)scratch(ctx, SLOT_MLP_G, sizeof(float) * ((size_t)m + (size_t)ntiles + 4));
  float *partial = (float *)scratch(ctx, SLOT_MLP_PART, sizeof(float) * (size_t)ntiles * NPARAMS);
  float *hl = (float *)host_scratch(ctx, sizeof(float) * 4);
  if (!acts || !gbuf || !partial || !hl) return VOFMT_E_NOMEM;
  float *loss_part = gbuf + m;
  float *loss_out = gbuf + m + ntiles;
  int rec = prof_begin(ctx, "k_mlp_fwd(train)", stream);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(fwd_grid(ctx, ntiles)), dim3(256), 0, stream, params, w[0], w[1], m, x,
                     (float *)nullptr, acts, y_target, gbuf, loss_part);
  prof_end(ctx, rec, stream);
  rec = prof_begin(ctx, "k_mlp_bwd", stream);
  hipLaunchKernelGGL(k_mlp_bwd, dim3(ntiles), dim3(256), 0, stream, params, w[2], m, x, acts, gbuf, partial, trace);
  prof_end(ctx, rec, stream);
  rec = prof_begin(ctx, "k_mlp_adam", stream);
  hipLaunchKernelGGL(k_mlp_adam, dim3(ceil_div(NPARAMS, 256)), dim3(256), 0, stream, params, adam_m, adam_v, partial,
                     ntiles, step, lr, grads, loss_part, loss_out, m);
  prof_end(ctx, rec, stream);
  VOFMT_HIP(ctx, hipGetLastError());
  VOFMT_HIP(ctx, hipMemcpyAsync(hl, loss_out, sizeof(float), hipMemcpyDeviceToHost, stream));
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  *loss_host = hl[0];
  return VOFMT_OK;
}

int list_grid(vofmt_ctx *ctx);

// Canonical stencils of the mixed cells (0 < c < 1) of one field, in
// increasing cell order. Writes at most `capacity` entries; *count_host gets
// the number of mixed cells (synchronises). xs: [capacity][27] FP32.
extern "C" int vofmt_mlp_stencils(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, const double *c,
                                  int32_t capacity, float *xs, int32_t *cell, int8_t *sign, int32_t *count_host,
                                  hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nx < 1 || ny < 1 || nz < 1 || !c || !count_host || capacity < 0)
    return set_err(ctx, VOFMT_E_ARG, "vofmt_mlp_stencils: bad arguments");
  const int64_t n3 = (int64_t)nx * ny * nz;
  if (n3 >= INT32_MAX) return set_err(ctx, VOFMT_E_ARG, "vofmt_mlp_stencils: too many cells");
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t nb = ceil_div(n3, compact::kBlock);
  const int64_t ntiles = compact::list_tiles(n3);
  int32_t *bc = (int32_t *)scratch(ctx, SLOT_MISC, sizeof(int32_t) * (size_t)nb);
  int32_t *tot = (int32_t *)scratch(ctx, SLOT_MISC2, sizeof(int32_t) * (size_t)(ntiles + 1));
  int32_t *list = (int32_t *)scratch(ctx, SLOT_CURV_LIST, sizeof(int32_t) * (size_t)n3);
  int32_t *hc = (int32_t *)host_scratch(ctx, sizeof(int32_t) * 2);
  if (!bc || !tot || !list || !hc) return VOFMT_E_NOMEM;
  compact::launch_ordered_list(c, n3, bc, tot, list, (double *)nullptr, (uint8_t *)nullptr, stream);
  VOFMT_HIP(ctx, hipGetLastError());
  VOFMT_HIP(ctx, hipMemcpyAsync(hc, tot + ntiles, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  const int total = hc[0];
  *count_host = total;
  if (total > capacity)
    return set_err(ctx, VOFMT_E_ARG, "vofmt_mlp_stencils: %d mixed cells, capacity %d", total, capacity);
  if (total == 0) return VOFMT_OK;
  if (!xs || !cell || !sign) return set_err(ctx, VOFMT_E_ARG, "vofmt_mlp_stencils: null output");
  VOFMT_HIP(ctx, hipMemcpyAsync(cell, list, sizeof(int32_t) * (size_t)total, hipMemcpyDeviceToDevice, stream));
  hipLaunchKernelGGL(k_stencil_list, dim3(ceil_div(total, 256)), dim3(256), 0, stream, c, nx, ny, nz, list, total, xs,
                     sign);
  return hip_check(ctx, hipGetLastError(), "vofmt_mlp_stencils kernels");
}

extern "C" int vofmt_curvature_mlp(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, const double *c,
                                   const float *params, double kappa_lo, double *kappa, uint8_t *status,
                                   int32_t *nmixed_host, hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nx < 1 || ny < 1 || nz < 1 || !c || !params || !kappa || !status || !(kappa_lo >= 0.0))
    return set_err(ctx, VOFMT_E_ARG, "vofmt_curvature_mlp: bad arguments");
  const int64_t n3 = (int64_t)nx * ny * nz;
  if (n3 >= INT32_MAX) return set_err(ctx, VOFMT_E_ARG, "vofmt_curvature_mlp: too many cells");
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t lt = compact::list_tiles(n3);
  int32_t *list = (int32_t *)scratch(ctx, SLOT_CURV_LIST, sizeof(int32_t) * (size_t)n3);
  int32_t *bc = (int32_t *)scratch(ctx, SLOT_MISC, sizeof(int32_t) * (size_t)ceil_div(n3, compact::kBlock));
  int32_t *tot = (int32_t *)scratch(ctx, SLOT_CURV_COUNT, sizeof(int32_t) * (size_t)(lt + 2));
  int32_t *hc = (int32_t *)host_scratch(ctx, sizeof(int32_t) * 2);
  if (!list || !bc || !tot || !hc) return VOFMT_E_NOMEM;
  int32_t *hf_count = tot + lt + 1;
  VOFMT_HIP(ctx, hipMemsetAsync(hf_count, 0, sizeof(int32_t), stream));
  int rec = prof_begin(ctx, "mixed_list", stream);
  compact::launch_ordered_list(c, n3, bc, tot, list, kappa, status, stream);
  prof_end(ctx, rec, stream);
  VOFMT_HIP(ctx, hipGetLastError());
  VOFMT_HIP(ctx, hipMemcpyAsync(hc, tot + lt, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  const int nm = hc[0];
  if (nmixed_host) *nmixed_host = nm;
  if (nm == 0) return VOFMT_OK;
  int32_t *hf_list = (int32_t *)scratch(ctx, SLOT_CURV_HF, sizeof(int32_t) * (size_t)nm);
  if (!hf_list) return VOFMT_E_NOMEM;
  uint16_t *w[3];
  int rc = mlp_prepare(ctx, params, w, stream);
  if (rc) return rc;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1)
    cus = 256;
  const int ftiles = (nm + FT - 1) / FT;
  const int fgrid = ftiles < cus * FWAVES ? (ftiles + FWAVES - 1) / FWAVES : cus;
  rec = prof_begin(ctx, "k_curv_fused", stream);
  hipLaunchKernelGGL(k_curv_fused, dim3(fgrid), dim3(64 * FWAVES), 0, stream, params, w[0], w[1], c, nx, ny, nz, list,
                     nm, kappa_lo, kappa, status, hf_list, hf_count);
  prof_end(ctx, rec, stream);
  rec = prof_begin(ctx, "k_curv_fallback", stream);
  hipLaunchKernelGGL(k_curv_fallback, dim3(list_grid(ctx)), dim3(256), 0, stream, c, nx, ny, nz, hf_list, hf_count,
                     kappa, status);
  prof_end(ctx, rec, stream);
  return hip_check(ctx, hipGetLastError(), "curvature_mlp kernels");
}
