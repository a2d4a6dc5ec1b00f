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
// bits). The FP32 biases enter the forward products' accumulation (b1 as
// three BF16 parts summing to it, b2 as the initial accumulator). The last
// layer (128 -> 1) is an FP32 dot product of the unrounded second-layer
// activations with the FP32 W3. Loss and Adam in FP32. ReLU'(z) is
// (activation > 0). Batch reductions go through partial sums, each over a
// contiguous range of tiles in order, added in a fixed order, so every result
// is reproducible bit for bit.
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

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int NIN = 32, NH = 128;
constexpr int OFF_W1 = 0, OFF_B1 = NIN * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NH, NPARAMS = OFF_B3 + 4;
static_assert(NPARAMS == VOFMT_MLP_NPARAMS, "parameter layout");

constexpr int TILE = 64;  // samples per tile of the backward pass
constexpr int HP = 136;  // LDS row pitches (bf16 elements), padded against bank conflicts
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

// BF16 copies of the weights for one call: W1 and W2 in the order of the
// forward pass's operand fragments (w1f [kk][half][lane][8], with b1 as
// hi + mid + lo on the padding inputs 27..29; w2f [nt][kk][lane][8]), and W2
// row-major [128][128] for the backward product.
__global__ void k_mlp_prep(const float *__restrict__ P, uint16_t *__restrict__ w1f, uint16_t *__restrict__ w2f,
                           uint16_t *__restrict__ w2n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NIN * NH) {
    const int f = i >> 3, e = i & 7, ln = f & 63, half = (f >> 6) & 1, kk = f >> 7;
    const int lr = ln & 15, lq = ln >> 4;
    const int u = 32 * kk + 8 * (lr >> 2) + 4 * half + (lr & 3);  // hidden unit of product row lr
    const int k = 8 * lq + e;
    uint16_t v = 0;
    if (k < 27) {
      v = bf16_bits(P[OFF_W1 + k * NH + u]);
    } else if (k < 30) {
      const float b = P[OFF_B1 + u];
      const uint16_t hi = bf16_bits(b);
      const float r1 = b - bf16_val(hi);
      const uint16_t mid = bf16_bits(r1);
      const float r2 = r1 - bf16_val(mid);
      v = k == 27 ? hi : (k == 28 ? mid : bf16_bits(r2));
    }
    w1f[i] = v;
  }
  if (i < NH * NH) {
    const int f = i >> 3, e = i & 7, ln = f & 63, kk = (f >> 6) & 3, nt = f >> 8;
    const int lr = ln & 15, lq = ln >> 4;
    w2f[i] = bf16_bits(P[OFF_W2 + (32 * kk + 8 * lq + e) * NH + 16 * nt + lr]);
    w2n[i] = bf16_bits(P[OFF_W2 + i]);
  }
}

__device__ __forceinline__ uint16_t *act_h1(uint8_t *rec, int64_t s, int stride) {
  return reinterpret_cast<uint16_t *>(rec + s * stride);
}
__device__ __forceinline__ float *act_h2(uint8_t *rec, int64_t s, int stride) {
  return reinterpret_cast<float *>(rec + s * stride + 256);
}

// ------------------------------------------------------------ forward pass
//
// A wavefront evaluates the network on a tile of WT = 64 samples by itself
// (no workgroup barrier after the weights are staged), both matrix-core
// layers chained in registers:
// - layer 1 is computed transposed, Z1^T = W1^T X^T, in product tiles of 16
//   hidden units x 16 samples whose rows are assigned to units so that lane
//   (lr, lq) of the tile (kk, half) receives units 32kk + 8lq + 4half + r
//   (r = 0..3) of sample lr: after both halves the lane holds, rounded to
//   BF16, exactly its B operand of layer 2's product over the K block kk;
// - layer 2 is computed transposed as well, Z2^T = W2^T H1^T, which leaves
//   units 16nt + 4lq + r of sample lr in lane (lr, lq): the last layer is a
//   dot product within the lane, then a sum over the four lane groups.
// b1 enters layer 1's product through the padding inputs 27..29, which hold
// the value one, with weights hi, mid, lo: three BF16 numbers whose sum is b1
// (exactly, for |b1| above 2^-100); b2 is the initial accumulator of layer 2.
// The weights sit in LDS in the order of the operand fragments, 16 bytes per
// lane at consecutive addresses.
constexpr int WT = 64;        // samples per wavefront tile
constexpr int WMT = WT / 16;  // 16-sample product tiles per wavefront tile
constexpr int L1P = 2;        // sample tiles per pass of layer 1 (bounds the live X operands)
constexpr int NW1F = 4 * 2 * 64, NW2F = 8 * 4 * 64;  // operand fragments of W1 and W2
static_assert(WT == TILE, "the loss of a forward tile is the loss of a backward tile");

typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

struct NetLds {
  bf16x8 w1f[NW1F];  // [kk][half][lane]
  bf16x8 w2f[NW2F];  // [nt][kk][lane]
  float b2[NH], w3[NH];
};

__device__ __forceinline__ void stage_net(NetLds &L, const float *__restrict__ P, const uint4 *__restrict__ w1f_g,
                                          const uint4 *__restrict__ w2f_g, int tid, int nthreads) {
  uint4 *d1 = reinterpret_cast<uint4 *>(L.w1f);
  uint4 *d2 = reinterpret_cast<uint4 *>(L.w2f);
  for (int i = tid; i < NW1F; i += nthreads) d1[i] = w1f_g[i];
  for (int i = tid; i < NW2F; i += nthreads) d2[i] = w2f_g[i];
  for (int i = tid; i < NH; i += nthreads) {
    L.b2[i] = P[OFF_B2 + i];
    L.w3[i] = P[OFF_W3 + i];
  }
}

typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

// (a, b) rounded to BF16 (nearest even) in one packed conversion, a in the low half.
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

// relu(a), relu(b) as BF16, packed: the rounding first, then a signed 16-bit
// maximum with zero, which clears exactly the values with the sign bit set --
// the same bits as rounding relu(a), relu(b).
__device__ __forceinline__ uint32_t relu_pack(float a, float b) {
  typedef __attribute__((ext_vector_type(2))) short s16x2;
  s16x2 v = __builtin_bit_cast(s16x2, pack_bf16(a, b));
  v = __builtin_elementwise_max(v, (s16x2){0, 0});
  return __builtin_bit_cast(uint32_t, v);
}

// Buffer resource over [base, base + bytes) (raw addressing, bounds checked
// by the hardware): a vector access beyond it reads zero and writes nothing.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void *base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, bytes, 0x00020000);
}

// relu(z) = (z > 0 ? z : 0) for every z but NaN, in one instruction: a
// signed 32-bit maximum with zero clears exactly the values with the sign
// bit set.
__device__ __forceinline__ float relu(float z) { return __int_as_float(max(__float_as_int(z), 0)); }

// The layer-1 operand of a 16-sample tile from eight input values of the
// lane (inputs 8lq .. 8lq+7 of sample lr), split into hi + lo, two values at
// a time: hi = bf16(v), lo = bf16(v - hi).
__device__ __forceinline__ void split_frag(const float (&v)[8], bf16x8 &h, bf16x8 &l) {
  u32x4 hw, lw;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const uint32_t hp = pack_bf16(v[2 * p], v[2 * p + 1]);
    hw[p] = hp;
    lw[p] = pack_bf16(v[2 * p] - __uint_as_float(hp << 16), v[2 * p + 1] - __uint_as_float(hp & 0xffff0000u));
  }
  h = __builtin_bit_cast(bf16x8, hw);
  l = __builtin_bit_cast(bf16x8, lw);
}

// The network on one wavefront tile. xfrag(mt, xh, xl) supplies the layer-1
// operands of sample tile mt; h1out(mt, kk, bits) and h2out(mt, nt, h) see
// the activations (units 32kk + 8lq .. +7 and 16nt + 4lq .. +3 of sample
// 16mt + lr). Returns in y[mt] the output of sample 16mt + lr, in every lane
// group.
template <class XF, class H1Out, class H2Out>
__device__ __forceinline__ void net_tile(const NetLds &L, int lane, float b3, XF xfrag, H1Out h1out, H2Out h2out,
                                         float (&y)[WMT]) {
  const int lq = lane >> 4;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  u32x4 h1[WMT][4];
#pragma unroll
  for (int mp = 0; mp < WMT; mp += L1P) {
    bf16x8 xh[L1P], xl[L1P];
#pragma unroll
    for (int j = 0; j < L1P; ++j) xfrag(mp + j, xh[j], xl[j]);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const bf16x8 a = L.w1f[(2 * kk + half) * 64 + lane];
#pragma unroll
        for (int j = 0; j < L1P; ++j) {
          f32x4 acc = mfma(a, xh[j], zero);
          acc = mfma(a, xl[j], acc);
          h1[mp + j][kk][2 * half] = relu_pack(acc[0], acc[1]);
          h1[mp + j][kk][2 * half + 1] = relu_pack(acc[2], acc[3]);
        }
      }
  }
#pragma unroll
  for (int mt = 0; mt < WMT; ++mt)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) h1out(mt, kk, h1[mt][kk]);
  float yq[WMT];
#pragma unroll
  for (int mt = 0; mt < WMT; ++mt) yq[mt] = 0.0f;
#pragma unroll
  for (int nt = 0; nt < 8; ++nt) {
    const f32x4 b2 = *reinterpret_cast<const f32x4 *>(&L.b2[16 * nt + 4 * lq]);
    const f32x4 w3 = *reinterpret_cast<const f32x4 *>(&L.w3[16 * nt + 4 * lq]);
    bf16x8 a[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) a[kk] = L.w2f[(4 * nt + kk) * 64 + lane];
#pragma unroll
    for (int mt = 0; mt < WMT; ++mt) {
      f32x4 acc = b2;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc = mfma(a[kk], __builtin_bit_cast(bf16x8, h1[mt][kk]), acc);
      f32x4 h;
#pragma unroll
      for (int r = 0; r < 4; ++r) h[r] = relu(acc[r]);
      h2out(mt, nt, h);
#pragma unroll
      for (int r = 0; r < 4; ++r) yq[mt] = fmaf(h[r], w3[r], yq[mt]);
    }
  }
#pragma unroll
  for (int mt = 0; mt < WMT; ++mt) {
    float v = yq[mt];
    v = v + __shfl_xor(v, 16);
    v = v + __shfl_xor(v, 32);
    y[mt] = v + b3;
  }
}

// y[lq]: the output of the lane's own sample 16lq + lr = lane.
__device__ __forceinline__ float own_output(const float (&y)[WMT], int lq) {
  float v = y[0];
  v = lq == 1 ? y[1] : v;
  v = lq == 2 ? y[2] : v;
  v = lq == 3 ? y[3] : v;
  return v;
}

// Forward pass over x[m][27], persistent: wavefront tiles of WT samples.
// acts (nullable): the activation records. With a target (training): also
// the upstream gradient g = dL/dy of every sample and the loss of every tile.
template <bool kTrain, bool kActs>
__device__ __forceinline__ void mlp_tiles(const NetLds &L, const float *__restrict__ P, int m,
                                          const float *__restrict__ x, float *__restrict__ y,
                                          uint8_t *__restrict__ acts, const float *__restrict__ tgt,
                                          float *__restrict__ g_out, float *__restrict__ loss_part, int waves) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: tile indices and buffer bases stay scalar
  const int lr = lane & 15, lq = lane >> 4;
  const float b3 = P[OFF_B3];
  const int ntiles = (m + WT - 1) / WT;
  const int xoff = (lr * 27 + 8 * lq) * 4;                  // byte offset of the lane's inputs in a row tile
  const uint32_t keep = lq < 3 ? 0xffffffffu : 0u;          // inputs 8lq + 3 .. 8lq + 7 exist
  const uint32_t one = lq == 3 ? __float_as_uint(1.0f) : 0u;  // else 27..29 are one
  for (int tile = blockIdx.x * waves + w; tile < ntiles; tile += gridDim.x * waves) {
    // the weight fragments are read from LDS tile by tile: kept out of the
    // loop they would need 160 registers
    __asm__ volatile("" ::: "memory");
    const int s0 = tile * WT;
    // the tile's rows of x and of the records: rows past m read zero and are not written
    const int rows = m - s0 < WT ? m - s0 : WT;
    const __amdgpu_buffer_rsrc_t xr = buffer_of(x + (int64_t)s0 * 27, rows * 27 * 4);
    const __amdgpu_buffer_rsrc_t ar = buffer_of(kActs ? acts + (int64_t)s0 * ACT_BYTES : acts, kActs ? rows * ACT_BYTES : 0);
    // inputs 8lq + e of sample row 16mt + lr, all loaded (inputs 27..31 read the
    // next row or zero); the lanes of group 3 then put one on 27..29, zero on 30..31
    auto xfrag = [&](int mt, bf16x8 &xh, bf16x8 &xl) {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t xv = __builtin_amdgcn_raw_buffer_load_b32(xr, xoff + (16 * mt * 27 + e) * 4, 0, 0);
        v[e] = __uint_as_float(e < 3 ? xv : ((xv & keep) | (e < 6 ? one : 0u)));
      }
      split_frag(v, xh, xl);
    };
    auto h1out = [&](int mt, int kk, u32x4 bits) {
      if (kActs) __builtin_amdgcn_raw_buffer_store_b128(bits, ar, (16 * mt + lr) * ACT_BYTES + (32 * kk + 8 * lq) * 2, 0, 0);
    };
    auto h2out = [&](int mt, int nt, f32x4 h) {
      if (kActs)
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, h), ar,
                                               (16 * mt + lr) * ACT_BYTES + 256 + (16 * nt + 4 * lq) * 4, 0, 0);
    };
    float yv[WMT];
    net_tile(L, lane, b3, xfrag, h1out, h2out, yv);
    const float yy = own_output(yv, lq);
    const int s = s0 + lane;
    if (y && s < m) y[s] = yy;
    if (kTrain) {
      float lv = 0.0f;
      if (s < m) {
        const float t = tgt[s];
        const float a = fabsf(t) > 0.05f ? fabsf(t) : 0.05f;
        const float wgt = 1.0f / (a * a);
        const float d = yy - t;
        lv = (d * d) * wgt;
        g_out[s] = ((2.0f * d) * wgt) / (float)m;
      }
      // butterfly over the wavefront: every lane ends with the same sum
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) lv = lv + __shfl_xor(lv, off);
      if (lane == 0) loss_part[tile] = lv;
    }
  }
}

constexpr int IWAVES = 8;  // wavefronts per workgroup of the forward kernels

template <bool kActs>
__global__ __launch_bounds__(64 * IWAVES) __attribute__((amdgpu_waves_per_eu(4))) void k_mlp_infer(const float *__restrict__ P,
                                                           const uint4 *__restrict__ w1f_g,
                                                           const uint4 *__restrict__ w2f_g, int m,
                                                           const float *__restrict__ x, float *__restrict__ y,
                                                           uint8_t *__restrict__ acts) {
  __shared__ NetLds L;
  stage_net(L, P, w1f_g, w2f_g, threadIdx.x, 64 * IWAVES);
  __syncthreads();
  mlp_tiles<false, kActs>(L, P, m, x, y, acts, nullptr, nullptr, nullptr, IWAVES);
}

__global__ __launch_bounds__(64 * IWAVES) __attribute__((amdgpu_waves_per_eu(4))) void k_mlp_fwd(const float *__restrict__ P, const uint4 *__restrict__ w1f_g,
                                                         const uint4 *__restrict__ w2f_g, int m,
                                                         const float *__restrict__ x, uint8_t *__restrict__ acts,
                                                         const float *__restrict__ tgt, float *__restrict__ g_out,
                                                         float *__restrict__ loss_part) {
  __shared__ NetLds L;
  stage_net(L, P, w1f_g, w2f_g, threadIdx.x, 64 * IWAVES);
  __syncthreads();
  mlp_tiles<true, true>(L, P, m, x, nullptr, acts, tgt, g_out, loss_part, IWAVES);
}

// Backward pass, persistent: workgroup g takes the 64-sample tiles
// [g T, (g+1) T) in order and accumulates its partial gradient of every
// parameter across them -- the weight gradients in the matrix cores'
// accumulators, the bias and W3 gradients as FP32 sums in fixed orders (per
// thread over the samples it handles, then over the threads) -- then writes
// it once (the partials are added later in a fixed order). trace
// (nullable): the training records of the samples.
__global__ __launch_bounds__(256) void k_mlp_bwd(const float *__restrict__ P, const uint16_t *__restrict__ w2n_g,
                                                 int m, const float *__restrict__ x, uint8_t *__restrict__ acts,
                                                 const float *__restrict__ g, float *__restrict__ partial,
                                                 uint8_t *__restrict__ trace, int tiles_per_group) {
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
  const int ntiles = (m + TILE - 1) / TILE;
  const int t0 = blockIdx.x * tiles_per_group;
  const int t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  float *part = partial + (int64_t)blockIdx.x * NPARAMS;
  if (tid < NH) w3s[tid] = P[OFF_W3 + tid];
  // accumulators over the workgroup's tiles: dW2 rows 16mt.., columns of wave w; dW1 likewise
  f32x4 accW2[2][8], accW1[2][2];
#pragma unroll
  for (int jn = 0; jn < 2; ++jn) {
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) accW2[jn][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) accW1[jn][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  // dW3 and db2 of unit tid % 128 over the samples of parity tid / 128; db1 of the lane's
  // units 16 (2w + jn) + lr over its rows 4lq + r of every 16-row tile; db3 (thread 0)
  float a3 = 0.0f, a2 = 0.0f, a1[2] = {0.0f, 0.0f}, ab3 = 0.0f;
  for (int tile = t0; tile < t1; ++tile) {
    const int s0 = tile * TILE;
    __syncthreads();  // the previous tile's LDS data is no longer read
    if (tid < TILE) gs[tid] = (s0 + tid < m) ? g[s0 + tid] : 0.0f;
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
      a3 = a3 + gs[s] * h2;
      a2 = a2 + bf16_val(b);
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
          a1[jn] = a1[jn] + bf16_val(b);
          if (trace && s0 + row < m)
            reinterpret_cast<uint16_t *>(trace + (int64_t)(s0 + row) * TRACE_BYTES + 1024)[col] = b;
        }
      }
    }
    __syncthreads();
    // dW2 += H1^T . dZ2 (128 x 128, K = 64 samples)
#pragma unroll
    for (int jn = 0; jn < 2; ++jn) {
      const int nt = 2 * w + jn;
#pragma unroll
      for (int mt = 0; mt < 8; ++mt)
#pragma unroll
        for (int kk = 0; kk < TILE; kk += 32)
          accW2[jn][mt] =
              mfma(frag(&H1T[16 * mt + lr][kk + 8 * lq]), frag(&D2T[16 * nt + lr][kk + 8 * lq]), accW2[jn][mt]);
    }
    // dW1 += X^T . dZ1 (32 x 128, K = 64 samples), X as hi + lo
#pragma unroll
    for (int jn = 0; jn < 2; ++jn) {
      const int nt = 2 * w + jn;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int kk = 0; kk < TILE; kk += 32) {
          const bf16x8 d1 = frag(&D1T[16 * nt + lr][kk + 8 * lq]);
          accW1[jn][mt] = mfma(frag(&XTh[16 * mt + lr][kk + 8 * lq]), d1, accW1[jn][mt]);
          accW1[jn][mt] = mfma(frag(&XTl[16 * mt + lr][kk + 8 * lq]), d1, accW1[jn][mt]);
        }
    }
    if (tid == 0)
      for (int s = 0; s < TILE; ++s) ab3 = ab3 + gs[s];
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
  // the workgroup's partial gradient
#pragma unroll
  for (int jn = 0; jn < 2; ++jn) {
    const int col = 16 * (2 * w + jn) + lr;
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) part[OFF_W2 + (16 * mt + 4 * lq + r) * NH + col] = accW2[jn][mt][r];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) part[OFF_W1 + (16 * mt + 4 * lq + r) * NH + col] = accW1[jn][mt][r];
  }
  // the per-thread sums combined in a fixed order (the tiles' LDS arrays are free now)
  __syncthreads();
  float *red = reinterpret_cast<float *>(&D2[0][0]);  // [2][128] dW3, [2][128] db2, [4][128] db1
  red[tid] = a3;
  red[256 + tid] = a2;
#pragma unroll
  for (int jn = 0; jn < 2; ++jn) red[512 + lq * NH + 16 * (2 * w + jn) + lr] = a1[jn];
  __syncthreads();
  if (tid < NH) {
    part[OFF_W3 + tid] = red[tid] + red[NH + tid];
    part[OFF_B2 + tid] = red[256 + tid] + red[256 + NH + tid];
    part[OFF_B1 + tid] = ((red[512 + tid] + red[512 + NH + tid]) + red[512 + 2 * NH + tid]) + red[512 + 3 * NH + tid];
  } else if (tid == NH) {
    part[OFF_B3 + 1] = 0.0f;
    part[OFF_B3 + 2] = 0.0f;
    part[OFF_B3 + 3] = 0.0f;
  }
  if (tid == 0) part[OFF_B3] = ab3;
}

// Gradient = fixed-order sum of the workgroup partials; Adam on the FP32 masters.
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ P, float *__restrict__ Mo,
                                                  float *__restrict__ Vo, const float *__restrict__ partial, int nparts,
                                                  int ntiles, int step, float lrate, float *__restrict__ grads,
                                                  const float *__restrict__ loss_part, float *__restrict__ loss_out,
                                                  int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NPARAMS) {
    float gsum = 0.0f;
    for (int t = 0; t < nparts; ++t) gsum = gsum + partial[(int64_t)t * NPARAMS + i];
    if (grads) grads[i] = gsum;
    const float mm = 0.9f * Mo[i] + 0.1f * gsum;
    const float vv = 0.999f * Vo[i] + 0.001f * (gsum * gsum);
    Mo[i] = mm;
    Vo[i] = vv;
    // bias corrections 1 - beta^step, in FP64 so that small steps lose nothing
    const float c1 = (float)(1.0 - pow(0.9, (double)step)), c2 = (float)(1.0 - pow(0.999, (double)step));
    P[i] = P[i] - lrate * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
  }
  // the loss: tile losses summed per thread of block 0 (stride 256), then a fixed tree
  if (blockIdx.x == 0) {
    __shared__ float lsum[256];
    float l = 0.0f;
    for (int t = threadIdx.x; t < ntiles; t += 256) l = l + loss_part[t];
    lsum[threadIdx.x] = l;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
      if ((int)threadIdx.x < h) lsum[threadIdx.x] = lsum[threadIdx.x] + lsum[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) loss_out[0] = lsum[0] / (float)m;
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
  bool two;        // the block holds two interfaces (see canonical_of_block)
};

// The 3x3x3 block around cell p (below 2^31, so 32-bit index arithmetic).
__device__ __forceinline__ void load_block(const double *__restrict__ c, uint32_t p, int nx, int ny, int nz,
                                           double *b) {
  const uint32_t row = p / (uint32_t)nx;
  const int i = (int)(p - row * (uint32_t)nx);
  const int k = (int)(row / (uint32_t)ny);
  const int j = (int)(row - (uint32_t)k * (uint32_t)ny);
  const int xs[3] = {wrap_dec(i, nx), i, wrap_inc(i, nx)};
  const int ys[3] = {wrap_dec(j, ny), j, wrap_inc(j, ny)};
  const int zs[3] = {wrap_dec(k, nz), k, wrap_inc(k, nz)};
#pragma unroll
  for (int az = 0; az < 3; ++az)
#pragma unroll
    for (int ay = 0; ay < 3; ++ay)
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) b[ax + 3 * ay + 9 * az] = c[(int64_t)(zs[az] * ny + ys[ay]) * nx + xs[ax]];
}

// The block (complemented when its centre exceeds 1/2) is handed on as
// FP32 values xf; the FP64 block itself is only needed for the normal.
__device__ __forceinline__ int canonical_of_block(double *b, float *xf, Canon &cn) {
  const int sign = (b[13] > 0.5) ? -1 : 1;
  // the complement 1 - b as one fused multiply-add (the same rounding as the subtraction)
  const double sf = sign < 0 ? -1.0 : 1.0, sa = sign < 0 ? 1.0 : 0.0;
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    b[q] = fma(sf, b[q], sa);
    xf[q] = (float)b[q];
  }
  double m0, m1, m2;
  int sigma_low;
  plic::myc_normal_sigma(b, m0, m1, m2, sigma_low);
  auto mv = [&](int a) { return a == 0 ? m0 : (a == 1 ? m1 : m2); };
  // two interfaces: along the first height-function axis (largest |m_d|, ties
  // to the lower axis) the centred-columns orientation disagrees with the
  // height functions' (full end low when m_d >= 0)
  {
    const double a0 = fabs(m0), a1 = fabs(m1), a2 = fabs(m2);
    const int ds = (a0 >= a1 && a0 >= a2) ? 0 : (a1 >= a2 ? 1 : 2);
    cn.two = (((sigma_low >> ds) & 1) != 0) != (mv(ds) >= 0.0);
  }
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

__device__ __forceinline__ int canonical_block(const double *__restrict__ c, uint32_t p, int nx, int ny, int nz,
                                               float *xf, Canon &cn) {
  double b[27];
  load_block(c, p, nx, ny, nz, b);
  return canonical_of_block(b, xf, cn);
}

// Entry a = (a0, a1, a2) of the block (offsets -1..1 along x, y, z) lands at
// canonical offsets q_k = d_k * a[o_k]: index (q0+1) + 3(q1+1) + 9(q2+1)
// = 13 + a0 S0 + a1 S1 + a2 S2, where source axis o_k has the stride
// S[o_k] = d_k 3^k.
template <class Put>
__device__ __forceinline__ void canonical_scatter(const float *xf, const Canon &cn, Put put) {
  auto stride = [&](int j) { return cn.o0 == j ? cn.d0 : (cn.o1 == j ? 3 * cn.d1 : 9 * cn.d2); };
  const int S0 = stride(0), S1 = stride(1), S2 = stride(2);
#pragma unroll
  for (int a2 = -1; a2 <= 1; ++a2)
#pragma unroll
    for (int a1 = -1; a1 <= 1; ++a1)
#pragma unroll
      for (int a0 = -1; a0 <= 1; ++a0)
        put(13 + a0 * S0 + a1 * S1 + a2 * S2, xf[(a0 + 1) + 3 * (a1 + 1) + 9 * (a2 + 1)]);
}

// Canonical stencils of the listed cells: xs[q], sign[q] for cell list[q].
__global__ __launch_bounds__(256) void k_stencil_list(const double *__restrict__ c, int nx, int ny, int nz,
                                                      const int32_t *__restrict__ list, int n, float *__restrict__ xs,
                                                      int8_t *__restrict__ sgn) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int64_t p = list[q];
  float xf[27];
  Canon cn;
  const int sg = canonical_block(c, (uint32_t)p, nx, ny, nz, xf, cn);
  float *row = xs + (int64_t)q * 27;
  canonical_scatter(xf, cn, [&](int e, float v) { row[e] = v; });
  sgn[q] = (int8_t)sg;
}

// Height functions on the fallback cells: their value where valid (status
// 1..3), else the network's value stays (status 4 + 8). The list is in
// regions of region_cells entries, region g holding counts[g] cells; `sub`
// workgroups share a region.
__global__ __launch_bounds__(256) void k_curv_fallback(const double *__restrict__ c, int nx, int ny, int nz,
                                                       const int32_t *__restrict__ hf_list,
                                                       const int32_t *__restrict__ counts, int64_t region_cells,
                                                       int sub, double *__restrict__ kappa,
                                                       uint8_t *__restrict__ status) {
  const int g = blockIdx.x / sub, part = blockIdx.x % sub;
  const int n = counts[g];
  const int32_t *lst = hf_list + (int64_t)g * region_cells;
  for (int q = part * blockDim.x + threadIdx.x; q < n; q += sub * blockDim.x) {
    const int64_t p = lst[q];
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

// Learned curvature of the listed interface cells in one pass (persistent):
// each wavefront takes tiles of WT cells on its own -- stencil gather and
// canonicalisation (one lane per cell) into its LDS slice of layer-1
// operands, then the network tile of the forward pass -- and writes
// kappa = sign * y with status 8, appending cells with |kappa| < kappa_lo or
// two interfaces in their block to the fallback list. The network arithmetic is that of the forward kernels,
// so y is bit-identical to vofmt_mlp_forward on the same stencils.
constexpr int FWAVES = 12;  // wavefronts per workgroup (LDS: 41 KB of weights + 9 KB per wavefront)

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int XSP = 36;  // row pitch (floats) of the stencil rows in LDS: 16-byte rows, conflict-free reads

__global__ __launch_bounds__(64 * FWAVES) void k_curv_fused(
    const float *__restrict__ P, const uint4 *__restrict__ w1f_g, const uint4 *__restrict__ w2f_g,
    const double *__restrict__ c, int nx, int ny, int nz, const int32_t *__restrict__ list, int nm, double kappa_lo,
    double *__restrict__ kappa, uint8_t *__restrict__ status, int32_t *__restrict__ hf_list,
    int32_t *__restrict__ hf_counts, int tiles_per_group) {
  __shared__ NetLds L;
  __shared__ int nflag;  // cells of the workgroup's tiles appended to its region of the fallback list
  // the canonical stencils of the wavefront's tile as FP32 rows [cell][input]
  __shared__ __attribute__((aligned(16))) float XS[FWAVES][WT][XSP];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  stage_net(L, P, w1f_g, w2f_g, tid, 64 * FWAVES);
  // inputs 27..29 are one, the rest of the padding zero (rows are written from 0 to 26 only)
  for (int i = lane; i < WT * XSP; i += 64) {
    const int col = i % XSP;
    XS[w][i / XSP][col] = (col >= 27 && col < 30) ? 1.0f : 0.0f;
  }
  const float b3 = P[OFF_B3];
  if (tid == 0) nflag = 0;
  __syncthreads();
  const int lr = lane & 15, lq = lane >> 4;
  float *xrow = XS[w][lane];
  // the workgroup's tiles: one contiguous range, whose cells bound its region of the list
  const int ntiles = (nm + WT - 1) / WT;
  const int t0 = blockIdx.x * tiles_per_group;
  const int t1 = t0 + tiles_per_group < ntiles ? t0 + tiles_per_group : ntiles;
  int32_t *region = hf_list + (int64_t)t0 * WT;
  for (int tile = t0 + w; tile < t1; tile += FWAVES) {
    // ---- canonical stencils, one lane per cell, into the lane's row
    const int q = tile * WT + lane;
    const bool own = q < nm;
    int sg = 1;
    int32_t p = 0;
    bool two = false;
    if (own) {
      p = list[q];
      float xf[27];
      Canon cn;
      sg = canonical_block(c, (uint32_t)p, nx, ny, nz, xf, cn);
      two = cn.two;
      canonical_scatter(xf, cn, [&](int k, float v) { xrow[k] = v; });
    } else {
      for (int k = 0; k < 27; ++k) xrow[k] = 0.0f;
    }
    wave_sync();
    // ---- the network: inputs 8lq .. 8lq+7 of cell 16mt + lr, split into hi + lo
    auto xfrag = [&](int mt, bf16x8 &xh, bf16x8 &xl) {
      const f32x4 *src = reinterpret_cast<const f32x4 *>(&XS[w][16 * mt + lr][8 * lq]);
      const f32x4 u = src[0], t = src[1];
      const float v[8] = {u[0], u[1], u[2], u[3], t[0], t[1], t[2], t[3]};
      split_frag(v, xh, xl);
    };
    auto none1 = [](int, int, u32x4) {};
    auto none2 = [](int, int, f32x4) {};
    float yv[WMT];
    net_tile(L, lane, b3, xfrag, none1, none2, yv);
    // ---- kappa, status, fallback list
    bool flag = false;
    if (own) {
      const double kn = (double)sg * (double)own_output(yv, lq);
      kappa[p] = kn;
      status[p] = 8;
      flag = two || fabs(kn) < kappa_lo;
    }
    const uint64_t mask = __ballot(flag);
    if (mask) {
      int base = 0;
      if (lane == 0) base = atomicAdd(&nflag, (int)__popcll(mask));
      base = __shfl(base, 0, 64);
      if (flag) region[base + __popcll(mask & ((1ull << lane) - 1))] = p;
    }
    wave_sync();  // the next tile overwrites this wavefront's rows
  }
  __syncthreads();
  if (tid == 0) hf_counts[blockIdx.x] = nflag;
}

}  // namespace

static int mlp_prepare(vofmt_ctx *ctx, const float *params, uint16_t **w, hipStream_t stream) {
  uint16_t *buf = (uint16_t *)scratch(ctx, SLOT_MLP_W, sizeof(uint16_t) * (NIN * NH + 2 * NH * NH));
  if (!buf) return VOFMT_E_NOMEM;
  w[0] = buf;                       // W1 fragments
  w[1] = buf + NIN * NH;            // W2 fragments
  w[2] = buf + NIN * NH + NH * NH;  // W2
  hipLaunchKernelGGL(k_mlp_prep, dim3(ceil_div(NH * NH, 256)), dim3(256), 0, stream, params, w[0], w[1], w[2]);
  return hip_check(ctx, hipGetLastError(), "k_mlp_prep");
}

// Workgroups of a persistent kernel: as many as fit the device at once, at
// most one per `waves` work tiles.
template <class K>
static int persistent_grid(vofmt_ctx *ctx, K kernel, int waves, int64_t tiles) {
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64 * waves, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const int64_t need = (tiles + waves - 1) / waves;
  const int64_t g = (int64_t)cus * per_cu;
  return (int)(need < g ? need : g);
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
  const int tiles = (m + WT - 1) / WT;
  const int rec = prof_begin(ctx, "k_mlp_infer", stream);
  if (acts)
    hipLaunchKernelGGL(k_mlp_infer<true>, dim3(persistent_grid(ctx, k_mlp_infer<true>, IWAVES, tiles)),
                       dim3(64 * IWAVES), 0, stream, params, (const uint4 *)w[0], (const uint4 *)w[1], m, x, y, acts);
  else
    hipLaunchKernelGGL(k_mlp_infer<false>, dim3(persistent_grid(ctx, k_mlp_infer<false>, IWAVES, tiles)),
                       dim3(64 * IWAVES), 0, stream, params, (const uint4 *)w[0], (const uint4 *)w[1], m, x, y, acts);
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
  // backward: one workgroup per compute unit at most, each over a contiguous range of tiles
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1)
    cus = 256;
  int groups = ntiles < cus ? ntiles : cus;
  const int per_group = (ntiles + groups - 1) / groups;
  groups = (ntiles + per_group - 1) / per_group;
  uint8_t *acts = (uint8_t *)scratch(ctx, SLOT_MLP_ACTS, (size_t)ACT_BYTES * (size_t)m);
  float *gbuf = (float *)scratch(ctx, SLOT_MLP_G, sizeof(float) * ((size_t)m + (size_t)ntiles + 4));
  float *partial = (float *)scratch(ctx, SLOT_MLP_PART, sizeof(float) * (size_t)groups * NPARAMS);
  float *hl = (float *)host_scratch(ctx, sizeof(float) * 4);
  if (!acts || !gbuf || !partial || !hl) return VOFMT_E_NOMEM;
  float *loss_part = gbuf + m;
  float *loss_out = gbuf + m + ntiles;
  int rec = prof_begin(ctx, "k_mlp_fwd(train)", stream);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(persistent_grid(ctx, k_mlp_fwd, IWAVES, ntiles)), dim3(64 * IWAVES), 0, stream,
                     params, (const uint4 *)w[0], (const uint4 *)w[1], m, x, acts, y_target, gbuf, loss_part);
  prof_end(ctx, rec, stream);
  rec = prof_begin(ctx, "k_mlp_bwd", stream);
  hipLaunchKernelGGL(k_mlp_bwd, dim3(groups), dim3(256), 0, stream, params, w[2], m, x, acts, gbuf, partial, trace,
                     per_group);
  prof_end(ctx, rec, stream);
  rec = prof_begin(ctx, "k_mlp_adam", stream);
  hipLaunchKernelGGL(k_mlp_adam, dim3(ceil_div(NPARAMS, 256)), dim3(256), 0, stream, params, adam_m, adam_v, partial,
                     groups, ntiles, step, lr, grads, loss_part, loss_out, m);
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
  uint64_t *bits = (uint64_t *)scratch(ctx, SLOT_LIST_BITS, sizeof(uint64_t) * (size_t)ceil_div(n3, 64));
  if (!bc || !tot || !list || !hc || !bits) return VOFMT_E_NOMEM;
  compact::launch_ordered_list(c, n3, bc, tot, list, (double *)nullptr, (uint8_t *)nullptr, bits, stream);
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
  const int fgrid_max = persistent_grid(ctx, k_curv_fused, FWAVES, INT32_MAX);
  int32_t *tot = (int32_t *)scratch(ctx, SLOT_CURV_COUNT, sizeof(int32_t) * (size_t)(lt + 1 + fgrid_max));
  int32_t *hc = (int32_t *)host_scratch(ctx, sizeof(int32_t) * 2);
  uint64_t *bits = (uint64_t *)scratch(ctx, SLOT_LIST_BITS, sizeof(uint64_t) * (size_t)ceil_div(n3, 64));
  if (!list || !bc || !tot || !hc || !bits) return VOFMT_E_NOMEM;
  int32_t *hf_counts = tot + lt + 1;  // fallback cells per workgroup of the fused kernel
  int rec = prof_begin(ctx, "mixed_list", stream);
  compact::launch_ordered_list(c, n3, bc, tot, list, kappa, status, bits, stream);
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
  // every workgroup takes an equal contiguous range of tiles
  const int ntiles = (nm + WT - 1) / WT;
  int fgrid = ntiles < fgrid_max ? ntiles : fgrid_max;
  const int per_group = (ntiles + fgrid - 1) / fgrid;
  fgrid = (ntiles + per_group - 1) / per_group;
  rec = prof_begin(ctx, "k_curv_fused", stream);
  hipLaunchKernelGGL(k_curv_fused, dim3(fgrid), dim3(64 * FWAVES), 0, stream, params, (const uint4 *)w[0],
                     (const uint4 *)w[1], c, nx, ny, nz, list, nm, kappa_lo, kappa, status, hf_list, hf_counts,
                     per_group);
  prof_end(ctx, rec, stream);
  rec = prof_begin(ctx, "k_curv_fallback", stream);
  constexpr int kSub = 8;  // workgroups per region
  hipLaunchKernelGGL(k_curv_fallback, dim3(fgrid * kSub), dim3(256), 0, stream, c, nx, ny, nz, hf_list, hf_counts,
                     (int64_t)per_group * WT, kSub, kappa, status);
  prof_end(ctx, rec, stream);
  return hip_check(ctx, hipGetLastError(), "curvature_mlp kernels");
}
