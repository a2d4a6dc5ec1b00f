// Drop labelling and drop moments.
//
// Labelling implements the tag.h step of section "The no-coalescence.h
// algorithm" (one value per region bounded by interfaces), read as the
// 6-connected periodic components of {c > c_eps}, numbered 1..K in
// increasing order of their smallest linear index.
//
// GPU scheme (union-find with atomicMin hooking, Komura/Playne-style); every
// kernel runs one wavefront per 64-cell row segment, so the lanes of a run of
// occupied cells sit side by side in one wavefront:
//   1. init:    parent[p] = start of p's run of occupied cells inside its
//               segment (one ballot per wavefront), -1 if empty;
//   2. merge:   one union per run of cells occupied in both this row and the
//               +y (or +z) row — the cells of a run already share a parent —
//               and one at the segment's first cell with its -x neighbour
//               (periodic); a union always hooks the larger root under the
//               smaller one, so every component ends rooted at its smallest
//               linear index whatever the order of the unions;
//   3. flatten: parent[start] = root(start) for every run start (the other
//               cells keep pointing at their start);
//   4. rank:    roots are counted per block with ballots, block counts are
//               scanned, and each root gets 1 + (number of roots before it);
//   5. final:   label[p] = rank of the root of p's run, read by the run's
//               start lane and passed to the run by a lane shuffle.
// The result is bit-identical to a sequential flood fill seeded in linear
// order.
#include "common.hpp"
#include "compact.hpp"

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int find_root(const int32_t *__restrict__ P, int32_t a) {
  int32_t b = P[a];
  while (b != a) {
    a = b;
    b = P[a];
  }
  return a;
}

// Root search with path halving: every node passed gets its grandparent as
// parent. Only nodes that are no longer roots are written, and always with
// an element of the same component of smaller index, so a concurrent hook
// is never undone for good: a hook that lands on a node that stopped being
// a root is retried by its union on the node's parent (see unite).
__device__ __forceinline__ int find_root_halving(int32_t *P, int32_t a) {
  int32_t b = P[a];
  while (b != a) {
    const int32_t g = P[b];
    if (g != b) P[a] = g;
    a = b;
    b = g;
  }
  return a;
}

// The parent array is read while other threads hook roots; volatile-free
// reads are fine: a stale parent still points to an element of the same
// component with a smaller-or-equal index, and the hooking loop retries
// until it installs the link on a true root.
__device__ __forceinline__ void unite(int32_t *P, int32_t a, int32_t b) {
  while (true) {
    a = find_root_halving(P, a);
    b = find_root_halving(P, b);
    if (a == b) return;
    if (a > b) {
      int32_t t = a;
      a = b;
      b = t;
    }
    // hook root b (larger) under a (smaller)
    int32_t old = atomicMin(&P[b], a);
    if (old == b) return;
    b = old;
  }
}

// Each wavefront walks kSegs consecutive 64-cell row segments (linear order
// of the cells is the order of (segment, lane)), so a workgroup covers
// 4 * kSegs segments.
constexpr int kSegs = 8;

// Row segment `sgi` (all segments of the field in linear order):
// row = z * ny + y, x = 64 * seg + lane.
struct Segment {
  int64_t row;
  int seg, y, z;
};
__device__ __forceinline__ Segment segment_of(int64_t sgi, int words, int ny) {
  Segment s;
  s.row = sgi / words;  // wavefront-uniform: scalar arithmetic
  s.seg = (int)(sgi - s.row * words);
  s.y = (int)(s.row % ny);
  s.z = (int)(s.row / ny);
  return s;
}
__device__ __forceinline__ int64_t first_segment() {
  return (((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6) * kSegs;
}

__global__ __launch_bounds__(kBlock) void k_label_init(const double *__restrict__ c, double c_eps,
                                                       int32_t *__restrict__ P, int nx, int ny, int nz, int words) {
  const int lane = threadIdx.x & 63;
  const int64_t nseg = (int64_t)ny * nz * words, s0 = first_segment();
  for (int64_t sgi = s0; sgi < s0 + kSegs && sgi < nseg; ++sgi) {  // wave-uniform
    const Segment sg = segment_of(sgi, words, ny);
    const int x = sg.seg * 64 + lane;
    const bool live = x < nx;
    const int64_t p = sg.row * nx + x;
    const bool occ = live && (c[p] > c_eps);
    const uint64_t m = __ballot(occ);
    if (!live) continue;
    if (!occ) {
      P[p] = -1;
      continue;
    }
    // start of the run of set bits that contains `lane`
    const uint64_t below = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1);
    const uint64_t zeros = ~m & below;  // empty cells at or below this lane
    const int start = zeros ? (64 - __clzll(zeros)) : 0;  // one past the highest empty lane below
    P[p] = (int32_t)(sg.row * nx + sg.seg * 64 + start);
  }
}

// Lane of the first cell of the run of set bits of m that contains `lane`.
__device__ __forceinline__ int run_start_lane(uint64_t m, int lane) {
  const uint64_t upto = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1);
  const uint64_t zeros = ~m & upto;
  return zeros ? (64 - __clzll(zeros)) : 0;
}

// Unions are made between run starts only (the union at the first cell of an
// overlap goes to the starts of the two runs), so the root searches, which
// shorten the paths they walk, only ever rewrite run starts: every other
// occupied cell keeps pointing at its own run's start.
__global__ __launch_bounds__(kBlock) void k_label_merge(int32_t *P, int nx, int ny, int nz, int words) {
  const int lane = threadIdx.x & 63;
  const int64_t nseg = (int64_t)ny * nz * words, s0 = first_segment();
  for (int64_t sgi = s0; sgi < s0 + kSegs && sgi < nseg; ++sgi) {  // wave-uniform
    const Segment sg = segment_of(sgi, words, ny);
    const int x = sg.seg * 64 + lane;
    const bool live = x < nx;
    const int64_t p = sg.row * nx + x;
    const bool occ = live && P[p] >= 0;
    const uint64_t mo = __ballot(occ);
    if (mo == 0) continue;  // wave-uniform
    const int64_t seg0 = sg.row * nx + sg.seg * 64;
    // -x: the segment's first cell (a run start) and its left neighbour (the
    // previous segment's last cell, or x = nx-1 through the periodic
    // boundary), represented by its parent, which is a run start
    if (lane == 0 && occ) {
      const int64_t q = sg.row * nx + (x == 0 ? nx - 1 : x - 1);
      if (q != p) {
        const int32_t pq = P[q];
        if (pq >= 0) unite(P, (int32_t)p, pq);
      }
    }
    // +y and +z: the first cell of every run occupied in both rows
    const int yp = (sg.y == ny - 1) ? 0 : sg.y + 1;
    const int zp = (sg.z == nz - 1) ? 0 : sg.z + 1;
    const int64_t rowy = (int64_t)sg.z * ny + yp, rowz = (int64_t)zp * ny + sg.y;
    const int64_t qy = rowy * nx + x, qz = rowz * nx + x;
    const bool oy = live && P[qy] >= 0;
    const bool oz = live && P[qz] >= 0;
    const uint64_t my = __ballot(oy), mz = __ballot(oz);
    const uint64_t by = mo & my, bz = mo & mz;
    const uint64_t sy = by & ~(by << 1), sz = bz & ~(bz << 1);
    const int32_t sp = (int32_t)(seg0 + run_start_lane(mo, lane));
    if (((sy >> lane) & 1ull) && qy != p)
      unite(P, sp, (int32_t)(rowy * nx + sg.seg * 64 + run_start_lane(my, lane)));
    if (((sz >> lane) & 1ull) && qz != p)
      unite(P, sp, (int32_t)(rowz * nx + sg.seg * 64 + run_start_lane(mz, lane)));
  }
}

// Run starts: parent = root; roots counted per block (the layout of
// k_label_rank).
__global__ __launch_bounds__(kBlock) void k_label_flatten(int32_t *P, int nx, int ny, int nz, int words,
                                                          uint32_t *__restrict__ blockcount) {
  const int lane = threadIdx.x & 63;
  const int64_t nseg = (int64_t)ny * nz * words, s0 = first_segment();
  uint32_t nroot = 0;  // wave-uniform
  for (int64_t sgi = s0; sgi < s0 + kSegs && sgi < nseg; ++sgi) {
    const Segment sg = segment_of(sgi, words, ny);
    const int x = sg.seg * 64 + lane;
    const bool live = x < nx;
    const int64_t p = sg.row * nx + x;
    const int32_t v = live ? P[p] : -1;
    const uint64_t mo = __ballot(v >= 0);
    const uint64_t starts = mo & ~(mo << 1);
    bool root = false;
    if ((starts >> lane) & 1ull) {
      const int32_t r = find_root(P, (int32_t)p);
      root = (r == p);
      if (r != v) P[p] = r;
    }
    nroot += (uint32_t)__popcll(__ballot(root));
  }
  __shared__ uint32_t wcount[kBlock / 64];
  if (lane == 0) wcount[threadIdx.x >> 6] = nroot;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int w = 0; w < kBlock / 64; ++w) s += wcount[w];
    blockcount[blockIdx.x] = s;
  }
}

// The total of the tiled scan into *total.
__global__ void k_copy_total(const int32_t *__restrict__ tot, int64_t ntiles, int32_t *__restrict__ total) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *total = tot[ntiles];
}

// Rank every root: rootlab[p] = 1 + number of roots before p; rootpos[rank] = p.
// blockoff: per-block exclusive offsets within tiles of compact::kTile
// blocks, tileoff: exclusive offsets of the tiles.
__global__ __launch_bounds__(kBlock) void k_label_rank(const int32_t *__restrict__ P, int nx, int ny, int nz,
                                                       int words, const int32_t *__restrict__ blockoff,
                                                       const int32_t *__restrict__ tileoff,
                                                       int32_t *__restrict__ rootlab, int32_t *__restrict__ rootpos) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t nseg = (int64_t)ny * nz * words, s0 = first_segment();
  // roots of each wavefront, then the offset of this wavefront in the block
  uint32_t nroot = 0;
  for (int64_t sgi = s0; sgi < s0 + kSegs && sgi < nseg; ++sgi) {
    const Segment sg = segment_of(sgi, words, ny);
    const int x = sg.seg * 64 + lane;
    const int64_t p = sg.row * nx + x;
    nroot += (uint32_t)__popcll(__ballot((x < nx) && (P[p] == p)));
  }
  __shared__ uint32_t wcount[kBlock / 64];
  if (lane == 0) wcount[w] = nroot;
  __syncthreads();
  uint32_t before = (uint32_t)(blockoff[blockIdx.x] + tileoff[blockIdx.x / compact::kTile]);
  for (int k = 0; k < w; ++k) before += wcount[k];
  for (int64_t sgi = s0; sgi < s0 + kSegs && sgi < nseg; ++sgi) {
    const Segment sg = segment_of(sgi, words, ny);
    const int x = sg.seg * 64 + lane;
    const int64_t p = sg.row * nx + x;
    const bool root = (x < nx) && (P[p] == p);
    const uint64_t m = __ballot(root);
    if (root) {
      const uint32_t r = before + (uint32_t)__popcll(m & ((1ull << lane) - 1));
      rootlab[p] = (int32_t)r + 1;
      if (rootpos) rootpos[r] = (int32_t)p;
    }
    before += (uint32_t)__popcll(m);
  }
}

// label[p] = rank of the root of p's run (0 if empty), in place.
__global__ __launch_bounds__(kBlock) void k_label_final(int32_t *__restrict__ P, int nx, int ny, int nz, int words,
                                                        const int32_t *__restrict__ rootlab) {
  const int lane = threadIdx.x & 63;
  const int64_t nseg = (int64_t)ny * nz * words, s0 = first_segment();
  for (int64_t sgi = s0; sgi < s0 + kSegs && sgi < nseg; ++sgi) {  // wave-uniform
    const Segment sg = segment_of(sgi, words, ny);
    const int x = sg.seg * 64 + lane;
    const bool live = x < nx;
    const int64_t p = sg.row * nx + x;
    const int64_t seg0 = sg.row * nx + sg.seg * 64;
    const int32_t v = live ? P[p] : -1;
    const uint64_t mo = __ballot(v >= 0);
    const uint64_t starts = mo & ~(mo << 1);
    // a start holds its root; the others point at their start (in this segment)
    int32_t lab = 0;
    if ((starts >> lane) & 1ull) lab = rootlab[v];
    const int src = (v >= 0) ? (int)((((starts >> lane) & 1ull) ? p : (int64_t)v) - seg0) : lane;
    const int32_t got = __shfl(lab, src, 64);
    if (live) P[p] = (v >= 0) ? got : 0;
  }
}

// ------------------------------------------------------------------ moments

// Offsets of p from the drop's first cell p0, wrapped into [-n/2, n/2).
__device__ __forceinline__ int wrapped_delta(int a, int a0, int n) {
  int d = a - a0;
  if (d < 0) d += n;
  if (2 * d >= n) d -= n;
  return d;
}

// Per-drop bounding box of the offsets (integer atomics: order-independent).
// Wavefront-wide minimum / maximum over the lanes in `mask` (others pass the
// neutral value in).
__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Per-drop reductions (first cell, bounding box) go through a small hash
// table in LDS per workgroup: a workgroup sweeps kChunk consecutive cells,
// the lanes of a wavefront holding the same drop are combined first, each
// such group updates the drop's LDS record with LDS atomics, and at the end
// the workgroup applies one set of global atomics per drop it met. Global
// atomics on one address from many workgroups are serialised; this makes
// them about kChunk / (cells of a drop's row run) times fewer. A drop that
// finds the table full goes to the global atomics directly. Integer min/max
// are order-independent, so the result does not depend on scheduling.
constexpr int kChunk = 8192;   // cells per workgroup (32 per thread)
constexpr int kTable = 64;     // LDS records per workgroup (power of two)
static_assert(kTable == 64 && kChunk % kBlock == 0, "table_slot hashes to 6 bits");

__device__ __forceinline__ int table_slot(int32_t *key, int32_t l) {
  const uint32_t h = ((uint32_t)l * 2654435761u) >> 26;  // 6 bits: kTable = 64
  for (int k = 0; k < kTable; ++k) {
    const int s = (int)((h + k) & (kTable - 1));
    const int32_t prev = atomicCAS(&key[s], 0, l);
    if (prev == 0 || prev == l) return s;
  }
  return -1;
}

// Bounding box of every drop as offsets from its first cell (periodic).
__global__ __launch_bounds__(kBlock) void k_drop_bbox(const int32_t *__restrict__ lab, int64_t n3, int nx, int ny, int nz,
                                                      FastDiv fnx, FastDiv fny, int32_t K,
                                                      const int32_t *__restrict__ rootpos,
                                                      int32_t *__restrict__ box) {
  __shared__ int32_t key[kTable];
  __shared__ int32_t rec[kTable][6];
  for (int i = threadIdx.x; i < kTable; i += kBlock) {
    key[i] = 0;
    for (int a = 0; a < 3; ++a) {
      rec[i][2 * a] = INT32_MAX;
      rec[i][2 * a + 1] = INT32_MIN;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t c0 = (int64_t)blockIdx.x * kChunk;
  for (int it = 0; it < kChunk / kBlock; ++it) {
    const int64_t p = c0 + (int64_t)it * kBlock + threadIdx.x;
    const int32_t l = (p < n3) ? lab[p] : 0;
    const bool valid = l > 0 && l <= K;
    int d[3] = {0, 0, 0};
    if (valid) {
      const uint32_t p0 = (uint32_t)rootpos[l - 1];
      // cell -> (x, y, z) by multiply-shift division (cells < 2^31)
      const uint32_t r = fast_div((uint32_t)p, fnx), r0 = fast_div(p0, fnx);
      const uint32_t zz = fast_div(r, fny), zz0 = fast_div(r0, fny);
      const int x = (int)((uint32_t)p - r * (uint32_t)nx), y = (int)(r - zz * (uint32_t)ny), z = (int)zz;
      const int x0 = (int)(p0 - r0 * (uint32_t)nx), y0 = (int)(r0 - zz0 * (uint32_t)ny), z0 = (int)zz0;
      d[0] = wrapped_delta(x, x0, nx);
      d[1] = wrapped_delta(y, y0, ny);
      d[2] = wrapped_delta(z, z0, nz);
    }
    uint64_t todo = __ballot(valid);
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int32_t lv = __shfl(l, leader, 64);
      const bool mine = valid && l == lv;
      const uint64_t same = __ballot(mine);
      int mn[3], mx[3];
      for (int a = 0; a < 3; ++a) {
        mn[a] = wave_min(mine ? d[a] : INT32_MAX);
        mx[a] = wave_max(mine ? d[a] : INT32_MIN);
      }
      if (lane == leader) {
        const int s = table_slot(key, lv);
        if (s >= 0) {
          for (int a = 0; a < 3; ++a) {
            atomicMin(&rec[s][2 * a], mn[a]);
            atomicMax(&rec[s][2 * a + 1], mx[a]);
          }
        } else {
          int32_t *b = box + 6 * (int64_t)(lv - 1);
          for (int a = 0; a < 3; ++a) {
            atomicMin(&b[2 * a], mn[a]);
            atomicMax(&b[2 * a + 1], mx[a]);
          }
        }
      }
      todo &= ~same;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kTable; i += kBlock) {
    const int32_t lv = key[i];
    if (lv == 0) continue;
    int32_t *b = box + 6 * (int64_t)(lv - 1);
    for (int a = 0; a < 3; ++a) {
      atomicMin(&b[2 * a], rec[i][2 * a]);
      atomicMax(&b[2 * a + 1], rec[i][2 * a + 1]);
    }
  }
}

__global__ void k_first_init(int32_t *first, int64_t K) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) first[i] = INT32_MAX;
}

// First (smallest linear index) cell of every drop; the lowest lane of a
// wavefront holding a drop has the wavefront's smallest cell of that drop.
__global__ __launch_bounds__(kBlock) void k_first_min(const int32_t *__restrict__ lab, int64_t n3, int32_t K,
                                                      int32_t *__restrict__ first) {
  __shared__ int32_t key[kTable];
  __shared__ int32_t rec[kTable];
  for (int i = threadIdx.x; i < kTable; i += kBlock) {
    key[i] = 0;
    rec[i] = INT32_MAX;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t c0 = (int64_t)blockIdx.x * kChunk;
  for (int it = 0; it < kChunk / kBlock; ++it) {
    const int64_t p = c0 + (int64_t)it * kBlock + threadIdx.x;
    const int32_t l = (p < n3) ? lab[p] : 0;
    const bool valid = l > 0 && l <= K;
    uint64_t todo = __ballot(valid);
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int32_t lv = __shfl(l, leader, 64);
      const uint64_t same = __ballot(valid && l == lv);
      if (lane == leader) {
        const int s = table_slot(key, lv);
        if (s >= 0) atomicMin(&rec[s], (int32_t)p);
        else atomicMin(&first[lv - 1], (int32_t)p);
      }
      todo &= ~same;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kTable; i += kBlock)
    if (key[i] != 0) atomicMin(&first[key[i] - 1], rec[i]);
}

__global__ void k_box_init(int32_t *box, int64_t K) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 6 * K) return;
  box[i] = (i & 1) ? INT32_MIN : INT32_MAX;
}

// kSumSplit workgroups per drop sum c and c*offset over consecutive parts of
// the drop's bounding box (per-thread strided partial sums, then a fixed
// tree); k_drop_finish adds the parts of each drop in order. The result is
// reproducible bit for bit.
constexpr int kSumSplit = 8;
__global__ __launch_bounds__(kBlock) void k_drop_sums(const double *__restrict__ c, const int32_t *__restrict__ lab,
                                                      int nx, int ny, int nz, const int32_t *__restrict__ rootpos,
                                                      const int32_t *__restrict__ box, double *__restrict__ part,
                                                      int32_t *__restrict__ extent_err) {
  const int l = blockIdx.x / kSumSplit + 1, sl = blockIdx.x % kSumSplit;
  const int32_t p0 = rootpos[l - 1];
  const int32_t *b = box + 6 * (int64_t)(l - 1);
  if (p0 == INT32_MAX || b[0] > b[1]) {  // label without cells: inconsistent input
    if (threadIdx.x == 0) atomicOr(extent_err, 2);
    return;
  }
  const int x0 = p0 % nx, y0 = (p0 / nx) % ny, z0 = p0 / (nx * ny);
  const int lx = b[0], ly = b[2], lz = b[4];
  const int ex = b[1] - b[0] + 1, ey = b[3] - b[2] + 1, ez = b[5] - b[4] + 1;
  // a drop spans less than half the box along each axis: its box has < 2^31 cells
  const int nbox = ex * ey * ez;
  const int q0 = (int)((int64_t)nbox * sl / kSumSplit), q1 = (int)((int64_t)nbox * (sl + 1) / kSumSplit);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int q = q0 + (int)threadIdx.x; q < q1; q += kBlock) {
    const int dx = q % ex + lx;
    const int dy = (q / ex) % ey + ly;
    const int dz = q / (ex * ey) + lz;
    // offsets lie in [-n/2, n/2): one period at most
    int x = x0 + dx, y = y0 + dy, z = z0 + dz;
    x += (x < 0) ? nx : ((x >= nx) ? -nx : 0);
    y += (y < 0) ? ny : ((y >= ny) ? -ny : 0);
    z += (z < 0) ? nz : ((z >= nz) ? -nz : 0);
    const int64_t p = ((int64_t)z * ny + y) * nx + x;
    if (lab[p] != l) continue;
    const double v = c[p];
    s0 += v;
    s1 += v * (double)dx;
    s2 += v * (double)dy;
    s3 += v * (double)dz;
  }
  __shared__ double red[4][kBlock];
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  red[2][threadIdx.x] = s2;
  red[3][threadIdx.x] = s3;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[((int64_t)(l - 1) * kSumSplit + sl) * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// Volume and periodic centroid of every drop from its kSumSplit parts.
__global__ void k_drop_finish(int32_t K, int nx, int ny, int nz, const int32_t *__restrict__ rootpos,
                              const int32_t *__restrict__ box, const double *__restrict__ part,
                              double *__restrict__ vol, double *__restrict__ xyz, int32_t *__restrict__ extent_err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const int32_t p0 = rootpos[i];
  const int32_t *b = box + 6 * i;
  if (p0 == INT32_MAX || b[0] > b[1]) return;  // reported by k_drop_sums
  double S[4] = {0.0, 0.0, 0.0, 0.0};
  for (int sl = 0; sl < kSumSplit; ++sl)
    for (int k = 0; k < 4; ++k) S[k] += part[(i * kSumSplit + sl) * 4 + k];
  const double V = S[0];
  vol[i] = V;
  const int n[3] = {nx, ny, nz};
  const int r[3] = {p0 % nx, (p0 / nx) % ny, p0 / (nx * ny)};
  for (int a = 0; a < 3; ++a) {
    double x = ((double)r[a] + 0.5) + S[1 + a] / V;
    if (x >= (double)n[a]) x -= (double)n[a];
    if (x < 0.0) x += (double)n[a];
    xyz[3 * i + a] = x;
    if (2 * (b[2 * a + 1] - b[2 * a]) >= n[a]) atomicOr(extent_err, 1);
  }
}

}  // namespace

// Workgroups of the labelling kernels: kSegs row segments per wavefront.
static inline int64_t label_blocks(int nx, int ny, int nz) {
  const int64_t words = (nx + 63) / 64;
  const int64_t per = (int64_t)(kBlock / 64) * kSegs;
  return ((int64_t)ny * nz * words + per - 1) / per;
}

// Label one tracer field into `lab`. Returns K via *k_dev (device int32).
// Scratch: block counts (label_blocks entries), tile offsets
// (label_blocks / compact::kTile + 2 entries), rootlab (n3 int32).
static int label_one(vofmt_ctx *ctx, int nx, int ny, int nz, const double *c, double c_eps, int32_t *lab,
                     uint32_t *blockcount, int32_t *tileoff, int32_t *rootlab, int32_t *k_dev, hipStream_t stream) {
  const int words = (int)ceil_div(nx, 64);
  const unsigned nb = (unsigned)label_blocks(nx, ny, nz);  // every kernel: kSegs row segments per wavefront
  const unsigned nb_init = nb;
  hipLaunchKernelGGL(k_label_init, dim3(nb_init), dim3(kBlock), 0, stream, c, c_eps, lab, nx, ny, nz, words);
  hipLaunchKernelGGL(k_label_merge, dim3(nb), dim3(kBlock), 0, stream, lab, nx, ny, nz, words);
  hipLaunchKernelGGL(k_label_flatten, dim3(nb), dim3(kBlock), 0, stream, lab, nx, ny, nz, words, blockcount);
  static_assert(kBlock == compact::kBlock, "block counts and the tiled scan share the block size");
  const int64_t ntiles = (nb + compact::kTile - 1) / compact::kTile;
  int32_t *bc = (int32_t *)blockcount;
  hipLaunchKernelGGL(compact::k_scan_tile, dim3((unsigned)ntiles), dim3(compact::kTile), 0, stream, bc, (int64_t)nb,
                     tileoff);
  hipLaunchKernelGGL(compact::k_scan_totals, dim3(1), dim3(compact::kTile), 0, stream, tileoff, ntiles);
  hipLaunchKernelGGL(k_copy_total, dim3(1), dim3(64), 0, stream, tileoff, ntiles, k_dev);
  hipLaunchKernelGGL(k_label_rank, dim3(nb), dim3(kBlock), 0, stream, lab, nx, ny, nz, words, bc, tileoff, rootlab,
                     (int32_t *)nullptr);
  hipLaunchKernelGGL(k_label_final, dim3(nb), dim3(kBlock), 0, stream, lab, nx, ny, nz, words, rootlab);
  return hip_check(ctx, hipGetLastError(), "label kernels");
}

extern "C" int vofmt_label_drops(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers,
                                 const double *c, double c_eps, int32_t *labels, int32_t *ndrops_host,
                                 hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nx < 1 || ny < 1 || nz < 1 || ntracers < 0 || !(c_eps >= 0.0))
    return set_err(ctx, VOFMT_E_ARG, "vofmt_label_drops: bad sizes or c_eps");
  if (ntracers == 0) return VOFMT_OK;
  if (!c || !labels || !ndrops_host) return set_err(ctx, VOFMT_E_ARG, "vofmt_label_drops: null pointer");
  const int64_t n3 = (int64_t)nx * ny * nz;
  if (n3 >= INT32_MAX) return set_err(ctx, VOFMT_E_ARG, "vofmt_label_drops: more than 2^31-1 cells per field");
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t nb = label_blocks(nx, ny, nz);
  uint32_t *blockcount = (uint32_t *)scratch(ctx, SLOT_LABEL_A, sizeof(uint32_t) * (size_t)nb);
  int32_t *rootlab = (int32_t *)scratch(ctx, SLOT_LABEL_B, sizeof(int32_t) * (size_t)n3);
  int32_t *kdev = (int32_t *)scratch(ctx, SLOT_MISC, sizeof(int32_t) * (size_t)ntracers);
  int32_t *tileoff = (int32_t *)scratch(ctx, SLOT_MISC3, sizeof(int32_t) * (size_t)(nb / compact::kTile + 2));
  int32_t *kh = (int32_t *)host_scratch(ctx, sizeof(int32_t) * (size_t)ntracers);
  if (!blockcount || !rootlab || !kdev || !tileoff || !kh) return VOFMT_E_NOMEM;
  for (int t = 0; t < ntracers; ++t) {
    int rc = label_one(ctx, nx, ny, nz, c + (int64_t)t * n3, c_eps, labels + (int64_t)t * n3, blockcount, tileoff,
                       rootlab, kdev + t, stream);
    if (rc) return rc;
  }
  VOFMT_HIP(ctx, hipMemcpyAsync(kh, kdev, sizeof(int32_t) * ntracers, hipMemcpyDeviceToHost, stream));
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  for (int t = 0; t < ntracers; ++t) ndrops_host[t] = kh[t];
  return VOFMT_OK;
}

extern "C" int vofmt_drop_moments(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers,
                                  const double *c, const int32_t *labels, const int32_t *ndrops_host, double *vol,
                                  double *xyz, hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nx < 1 || ny < 1 || nz < 1 || ntracers < 0) return set_err(ctx, VOFMT_E_ARG, "vofmt_drop_moments: bad sizes");
  if (ntracers == 0) return VOFMT_OK;
  if (!c || !labels || !ndrops_host) return set_err(ctx, VOFMT_E_ARG, "vofmt_drop_moments: null pointer");
  int64_t D = 0;
  for (int t = 0; t < ntracers; ++t) {
    if (ndrops_host[t] < 0) return set_err(ctx, VOFMT_E_ARG, "vofmt_drop_moments: negative drop count");
    D += ndrops_host[t];
  }
  if (D == 0) return VOFMT_OK;
  if (!vol || !xyz) return set_err(ctx, VOFMT_E_ARG, "vofmt_drop_moments: null output");
  const int64_t n3 = (int64_t)nx * ny * nz;
  if (n3 >= INT32_MAX) return set_err(ctx, VOFMT_E_ARG, "vofmt_drop_moments: more than 2^31-1 cells per field");
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  int64_t kmax = 0;
  for (int t = 0; t < ntracers; ++t) kmax = ndrops_host[t] > kmax ? ndrops_host[t] : kmax;
  int32_t *rootpos = (int32_t *)scratch(ctx, SLOT_LABEL_C, sizeof(int32_t) * (size_t)(kmax + 1));
  int32_t *box = (int32_t *)scratch(ctx, SLOT_MISC2, sizeof(int32_t) * 6 * (size_t)(kmax + 1));
  int32_t *flags = (int32_t *)scratch(ctx, SLOT_MISC, sizeof(int32_t) * 2);
  double *part = (double *)scratch(ctx, SLOT_LABEL_A, sizeof(double) * 4 * kSumSplit * (size_t)(kmax + 1));
  int32_t *fh = (int32_t *)host_scratch(ctx, sizeof(int32_t) * 2);
  if (!rootpos || !box || !flags || !part || !fh) return VOFMT_E_NOMEM;
  VOFMT_HIP(ctx, hipMemsetAsync(flags, 0, sizeof(int32_t) * 2, stream));
  const FastDiv fnx = make_fastdiv((uint32_t)nx), fny = make_fastdiv((uint32_t)ny);
  const unsigned nbc = ceil_div(n3, kChunk);  // workgroups of the per-drop reductions
  int64_t off = 0;
  for (int t = 0; t < ntracers; ++t) {
    const int32_t K = ndrops_host[t];
    if (K == 0) continue;
    const int32_t *lab = labels + (int64_t)t * n3;
    hipLaunchKernelGGL(k_first_init, dim3(ceil_div(K, 256)), dim3(256), 0, stream, rootpos, (int64_t)K);
    hipLaunchKernelGGL(k_first_min, dim3(nbc), dim3(kBlock), 0, stream, lab, n3, K, rootpos);
    hipLaunchKernelGGL(k_box_init, dim3(ceil_div(6 * (int64_t)K, 256)), dim3(256), 0, stream, box, (int64_t)K);
    hipLaunchKernelGGL(k_drop_bbox, dim3(nbc), dim3(kBlock), 0, stream, lab, n3, nx, ny, nz, fnx, fny, K, rootpos,
                       box);
    hipLaunchKernelGGL(k_drop_sums, dim3((unsigned)(K * kSumSplit)), dim3(kBlock), 0, stream, c + (int64_t)t * n3, lab,
                       nx, ny, nz, rootpos, box, part, flags);
    hipLaunchKernelGGL(k_drop_finish, dim3(ceil_div(K, 256)), dim3(256), 0, stream, K, nx, ny, nz, rootpos, box, part,
                       vol + off, xyz + 3 * off, flags);
    VOFMT_HIP(ctx, hipGetLastError());
    off += K;
  }
  VOFMT_HIP(ctx, hipMemcpyAsync(fh, flags, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, stream));
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  if (fh[0] & 2) return set_err(ctx, VOFMT_E_ARG, "vofmt_drop_moments: labels do not match ndrops_host");
  if (fh[0]) return set_err(ctx, VOFMT_E_EXTENT, "vofmt_drop_moments: a drop spans half the box or more");
  return VOFMT_OK;
}
