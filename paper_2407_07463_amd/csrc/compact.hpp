// Lists of the interface (mixed) cells of one field in increasing cell order:
// block counts (with one bit per cell), a tiled scan, then a second pass that
// writes the list from the bits. No
// atomics, so the order is fixed. A cell is an interface cell when its value
// lies more than 1e-12 inside (0, 1); round-off residues of pure cells are not.
#pragma once

#include "common.hpp"

namespace compact {
namespace {  // each translation unit gets its own kernels

constexpr int kBlock = 256;
constexpr int kTile = 1024;  // entries per scan tile

constexpr double kResidue = 1e-12;
__device__ __forceinline__ bool is_mixed(double v) { return v > kResidue && v < 1.0 - kResidue; }

// The mixed-cell list takes kPer cells per thread: block b covers cells
// [b kCells, (b + 1) kCells) as kPer coalesced sub-chunks of kBlock cells
// (sub-chunk k at b kCells + k kBlock), whose values are all loaded before
// the first is used. Far fewer, longer-lived workgroups than one per
// kBlock cells.
constexpr int kPer = 8;
constexpr int64_t kCells = (int64_t)kBlock * kPer;

// Mixed cells per block of kCells cells, and the mixed-cell bits: word
// p / 64 of `bits` for the 64 cells p of a wavefront's sub-chunk (64-aligned).
__global__ __launch_bounds__(kBlock) void k_block_counts(const double *__restrict__ c, int64_t n3,
                                                         int32_t *__restrict__ bc, uint64_t *__restrict__ bits) {
  const int64_t p0 = (int64_t)blockIdx.x * kCells + threadIdx.x;
  double v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) v[k] = (p0 + k * kBlock < n3) ? c[p0 + k * kBlock] : 0.0;
  int n = 0;  // wavefront-uniform
  const int64_t pw0 = p0 - (threadIdx.x & 63);  // the wavefront's first cell of sub-chunk 0
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const uint64_t mk = __ballot(p0 + k * kBlock < n3 && is_mixed(v[k]));
    n += (int)__popcll(mk);
    const int64_t pw = pw0 + k * kBlock;
    if ((threadIdx.x & 63) == 0 && pw < n3) bits[pw >> 6] = mk;
  }
  __shared__ int wc[kBlock / 64];
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += wc[w];
    bc[blockIdx.x] = t;
  }
}

// Exclusive scan of one tile of kTile entries in place; the tile total goes to tot[tile].
// Batches of arrays along blockIdx.y: array b starts at v + b * vstride, its totals at
// tot + b * tstride.
__global__ __launch_bounds__(kTile) void k_scan_tile(int32_t *__restrict__ v, int64_t n, int32_t *__restrict__ tot,
                                                     int64_t vstride, int64_t tstride) {
  v += blockIdx.y * vstride;
  tot += blockIdx.y * tstride;
  __shared__ int32_t s[kTile];
  const int64_t i = (int64_t)blockIdx.x * kTile + threadIdx.x;
  const int32_t x = (i < n) ? v[i] : 0;
  s[threadIdx.x] = x;
  __syncthreads();
  for (int off = 1; off < kTile; off <<= 1) {
    const int32_t add = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  if (i < n) v[i] = s[threadIdx.x] - x;
  if (threadIdx.x == kTile - 1) tot[blockIdx.x] = s[kTile - 1];
}

// Exclusive scan of the tile totals (one workgroup, any length); the grand
// total goes to tot[ntiles]. Batches along blockIdx.y as in k_scan_tile.
__global__ __launch_bounds__(kTile) void k_scan_totals(int32_t *__restrict__ tot, int64_t ntiles, int64_t tstride) {
  tot += blockIdx.y * tstride;
  __shared__ int32_t s[kTile];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < ntiles; base += kTile) {
    const int64_t i = base + threadIdx.x;
    const int32_t x = (i < ntiles) ? tot[i] : 0;
    s[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < kTile; off <<= 1) {
      const int32_t add = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < ntiles) tot[i] = carry + s[threadIdx.x] - x;
    __syncthreads();
    if (threadIdx.x == 0) carry += s[kTile - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[ntiles] = carry;
}

// Ordered list: block b writes its mixed cells from bc[b] + tot[b / kTile],
// sub-chunk by sub-chunk, wavefront by wavefront, from the bits of the
// counting pass (the field is not read again). With kappa/status given,
// also writes NaN / 0 into every cell that is not mixed.
__global__ __launch_bounds__(kBlock) void k_write_ordered(const uint64_t *__restrict__ bits, int64_t n3,
                                                          const int32_t *__restrict__ bc,
                                                          const int32_t *__restrict__ tot, int32_t *__restrict__ list,
                                                          double *__restrict__ kappa, uint8_t *__restrict__ status) {
  const int64_t p0 = (int64_t)blockIdx.x * kCells + threadIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t pw0 = p0 - lane;
  uint64_t wd[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) wd[k] = (pw0 + k * kBlock < n3) ? bits[(pw0 + k * kBlock) >> 6] : 0ull;
  __shared__ int wc[kPer][kBlock / 64];
  uint64_t mk[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int64_t p = p0 + k * kBlock;
    const bool inside = p < n3;
    const bool mixed = inside && ((wd[k] >> lane) & 1ull);
    if (inside && !mixed && kappa) {
      kappa[p] = __builtin_nan("");
      status[p] = 0;
    }
    mk[k] = __ballot(mixed);
    if (lane == 0) wc[k][w] = (int)__popcll(mk[k]);
  }
  __syncthreads();
  int run = bc[blockIdx.x] + tot[blockIdx.x / kTile];  // entries of the cells before sub-chunk k
  const uint64_t below = (1ull << lane) - 1;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    int idx = run;
    for (int j = 0; j < w; ++j) idx += wc[k][j];
    if ((mk[k] >> lane) & 1ull) list[idx + (int)__popcll(mk[k] & below)] = (int32_t)(p0 + k * kBlock);
    for (int j = 0; j < kBlock / 64; ++j) run += wc[k][j];
  }
}

// The ordered list of the mixed cells of c into `list` (capacity n3), its
// length into tot[ntiles] on the device. bc: ceil(n3 / kBlock) ints of
// scratch; tot: ntiles + 1 ints, ntiles = ceil(bc length / kTile); bits:
// ceil(n3 / 64) words of scratch.
inline void launch_ordered_list(const double *c, int64_t n3, int32_t *bc, int32_t *tot, int32_t *list, double *kappa,
                                uint8_t *status, uint64_t *bits, hipStream_t stream) {
  const int64_t nb = (n3 + kCells - 1) / kCells;
  const int64_t ntiles = (nb + kTile - 1) / kTile;
  hipLaunchKernelGGL(k_block_counts, dim3((unsigned)nb), dim3(kBlock), 0, stream, c, n3, bc, bits);
  hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)ntiles), dim3(kTile), 0, stream, bc, nb, tot, (int64_t)0, (int64_t)0);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kTile), 0, stream, tot, ntiles, (int64_t)0);
  hipLaunchKernelGGL(k_write_ordered, dim3((unsigned)nb), dim3(kBlock), 0, stream, bits, n3, bc, tot, list, kappa,
                     status);
}

// Scan tiles of the mixed-cell list of n3 cells (its length is at tot[list_tiles(n3)]).
inline int64_t list_tiles(int64_t n3) { return ((n3 + kCells - 1) / kCells + kTile - 1) / kTile; }
// Scan tiles of a predicate list of n cells (one block count per kBlock cells).
inline int64_t list_tiles_if(int64_t n) { return ((n + kBlock - 1) / kBlock + kTile - 1) / kTile; }

// Ordered lists of the cells p < n of a predicate whose counting pass stores
// it as one bit per cell (one 64-bit word per wavefront of cells) and one
// count per kBlock cells: the writing pass reads the bits.
// One wavefront per block of kBlock cells (its kBlock / 64 words), four
// blocks per workgroup: word j's set bits are written in round j, after the
// block's offset and the bits of its earlier words.
__global__ __launch_bounds__(kBlock) void k_write_ordered_bits(int64_t n, const uint64_t *__restrict__ bits,
                                                               const int32_t *__restrict__ bc,
                                                               const int32_t *__restrict__ tot,
                                                               int32_t *__restrict__ list) {
  constexpr int kWords = kBlock / 64;
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);  // this wavefront's block
  const int64_t nb = (n + kBlock - 1) / kBlock;
  if (b >= nb) return;  // whole wavefront
  const int64_t c0 = b * kBlock;
  uint64_t wm[kWords];
#pragma unroll
  for (int j = 0; j < kWords; ++j) wm[j] = (c0 + 64 * j < n) ? bits[(c0 >> 6) + j] : 0ull;
  int idx = bc[b] + tot[b / kTile];
  const uint64_t below = (1ull << lane) - 1;
#pragma unroll
  for (int j = 0; j < kWords; ++j) {
    if ((wm[j] >> lane) & 1ull) list[idx + (int)__popcll(wm[j] & below)] = (int32_t)(c0 + 64 * j + lane);
    idx += (int)__popcll(wm[j]);
  }
}

}  // namespace
}  // namespace compact
