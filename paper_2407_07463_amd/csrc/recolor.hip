// Reassignment of drops in near contact to other tracers: Steps 1-4 of
// section "The no-coalescence.h algorithm".
//
// Reading: drops are the (tracer, label) pairs; two distinct drops are
// neighbours when occupied cells of each lie at a periodic offset o with
// |o|^2 < (1 + gap)^2 (o = 0 included across tracers); neighbours in the
// same tracer conflict; drops are visited in ascending (tracer, label) and a
// drop whose current tracer is held by an earlier neighbour moves to the
// smallest tracer none of its neighbours holds, or to a new one.
//
// GPU scheme:
//   1. own[p]: global id of the only drop occupying cell p, -1 if none,
//      -2 if several (drops of different tracers overlapping);
//   2. every occupied cell scans the offsets of the ball and sets the bit of
//      each neighbouring drop in a D x D adjacency bitmap (atomicOr; the
//      bitmap is symmetric and its content independent of thread order);
//   3. the bitmap is turned into sorted neighbour lists (CSR);
//   4. one wavefront runs the greedy pass: tracers of all drops in LDS,
//      neighbour lists streamed through LDS in chunks, one ballot per drop
//      for the conflict test and an OR-reduction for the tracers in use;
//   5. the host reads back the tracer count (capacity check), then every
//      cell clears its moved-out values and adds them to the new fields.
//
// Stencil mode (vofmt_recolor_tracers_stencil): the neighbour relation of
// step 2 is the paper's criterion read literally. Within a tracer, two drops
// are neighbours when an empty cell (label 0) has one of them and the other
// at opposite offsets +o, -o of the 5x5x5 stencil (Steps 1-3): one wavefront
// per 64-cell row segment tests the 62 opposite pairs on occupancy bits of
// the 25 neighbouring rows and loads labels only for candidate pairs. Across
// tracers, drops are neighbours ("in contact", Step 4) when cells of the two
// lie within 4 cells along every axis (the stencil's reach), found by the
// scan of step 2 over the half 9x9x9 cube, pairs within one tracer skipped.
#include <cstdlib>
#include <cstring>

#include "common.hpp"
#include "compact.hpp"

namespace {

constexpr int kBlock = 256;
constexpr int kMaxTracers = 64;    // tracers are bits of a 64-bit mask
constexpr int kMaxDrops = 32768;   // the adjacency bitmap is D^2 bits
constexpr int kChunk = 4096;       // neighbour ids staged in LDS per chunk

struct TracerOffsets {
  int32_t off[kMaxTracers + 1];  // first global drop id of each tracer
};

__global__ __launch_bounds__(kBlock) void k_owner(const int32_t *__restrict__ lab, int64_t n3, int ntr,
                                                  TracerOffsets to, int32_t *__restrict__ own) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n3) return;
  int32_t o = -1;
  for (int t = 0; t < ntr; ++t) {
    const int32_t l = lab[(int64_t)t * n3 + p];
    if (l > 0 && to.off[t] + l <= to.off[t + 1]) o = (o == -1) ? to.off[t] + l - 1 : -2;
  }
  own[p] = o;
}

// The same for 4 consecutive cells per thread with 16-byte label loads
// (labels 16-byte aligned and n3 a multiple of 4).
__global__ __launch_bounds__(kBlock) void k_owner4(const int4 *__restrict__ lab, int64_t n4, int ntr,
                                                   TracerOffsets to, int4 *__restrict__ own) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n4) return;
  int32_t o[4] = {-1, -1, -1, -1};
  for (int t = 0; t < ntr; ++t) {
    const int4 l4 = lab[(int64_t)t * n4 + i];
    const int32_t l[4] = {l4.x, l4.y, l4.z, l4.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (l[k] > 0 && to.off[t] + l[k] <= to.off[t + 1]) o[k] = (o[k] == -1) ? to.off[t] + l[k] - 1 : -2;
  }
  own[i] = make_int4(o[0], o[1], o[2], o[3]);
}

// v in (-n, 2n): one conditional add or subtract instead of a modulo
__device__ __forceinline__ int wrap_near(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ void set_edge(uint32_t *adj, int64_t words, int32_t a, int32_t b) {
  uint32_t *w = adj + (int64_t)a * words + (b >> 5);
  const uint32_t bit = 1u << (b & 31);
  if (!(*w & bit)) atomicOr(w, bit);
}

// Calls f(id) for every drop occupying cell p (for cells shared by several drops).
template <class F>
__device__ __forceinline__ void for_drops_at(const int32_t *__restrict__ lab, int64_t n3, int ntr,
                                             const TracerOffsets &to, int64_t p, F f) {
  for (int t = 0; t < ntr; ++t) {
    const int32_t l = lab[(int64_t)t * n3 + p];
    if (l > 0 && to.off[t] + l <= to.off[t + 1]) f(to.off[t] + l - 1);
  }
}

__device__ __forceinline__ void edges_of(const int32_t *__restrict__ own, const int32_t *__restrict__ lab, int nx,
                                         int ny, int nz, int ntr, const TracerOffsets &to,
                                         const int4 *__restrict__ offs, int noffs, int small_offsets,
                                         uint32_t *__restrict__ adj, int64_t words, int64_t n3, const FastDiv &fnx,
                                         const FastDiv &fny, const int32_t *__restrict__ cross_T0, int64_t p) {
  // cross_T0 != null: only drops of different tracers (initial tracer per drop) are related
  auto set_edge = [&](uint32_t *adj_, int64_t words_, int32_t u, int32_t v) {
    if (cross_T0 != nullptr && cross_T0[u] == cross_T0[v]) return;
    ::set_edge(adj_, words_, u, v);
  };
  const int32_t a = own[p];
  const uint32_t r = fast_div((uint32_t)p, fnx), zz = fast_div(r, fny);  // cells < 2^31
  const int x = (int)((uint32_t)p - r * (uint32_t)nx), y = (int)(r - zz * (uint32_t)ny), z = (int)zz;
  if (a == -2) {
    // drops sharing this very cell are neighbours (offset 0 across tracers)
    for_drops_at(lab, n3, ntr, to, p, [&](int32_t u) {
      for_drops_at(lab, n3, ntr, to, p, [&](int32_t v) {
        if (u != v) set_edge(adj, words, u, v);
      });
    });
  }
  // The owners of kBatch offsets are loaded together (past the last offset
  // every lane loads its own cell and ignores it); a drop just paired with
  // this cell's drop is not paired again (a boundary cell sees a neighbouring
  // drop through many offsets).
  constexpr int kBatch = 8;
  int32_t last_b = -1;
  for (int k0 = 0; k0 < noffs; k0 += kBatch) {
    int32_t bs[kBatch];
    int64_t qs[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int k = k0 + j < noffs ? k0 + j : 0;
      const int4 o = offs[k];
      const int64_t q = small_offsets ? ((int64_t)wrap_near(z + o.z, nz) * ny + wrap_near(y + o.y, ny)) * nx +
                                            wrap_near(x + o.x, nx)
                                      : ((int64_t)wrap_any(z + o.z, nz) * ny + wrap_any(y + o.y, ny)) * nx +
                                            wrap_any(x + o.x, nx);
      qs[j] = (k0 + j < noffs) ? q : p;
      bs[j] = own[qs[j]];
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      if (k0 + j >= noffs) break;
      const int64_t q = qs[j];
      const int32_t b = bs[j];
      if (b == -1) continue;
      if (a >= 0 && b >= 0) {
        if (a != b && b != last_b) {
          set_edge(adj, words, a, b);
          last_b = b;
        }
        continue;
      }
      // a shared cell on either side: every drop of p with every drop of q
      auto with_q = [&](int32_t u) {
        if (b >= 0) {
          if (u != b) set_edge(adj, words, u, b);
        } else {
          for_drops_at(lab, n3, ntr, to, q, [&](int32_t v) {
            if (u != v) set_edge(adj, words, u, v);
          });
        }
      };
      if (a >= 0) with_q(a);
      else for_drops_at(lab, n3, ntr, to, p, with_q);
    }
  }
}


// Cells that can find a pair: shared cells, and cells of one drop with a
// six-neighbour not owned by that drop. An interior cell finds no pair that
// a boundary cell of its drop does not: a lattice path from it towards any
// other drop's cell, one axis step at a time, only gets closer and leaves the
// drop through a boundary cell.
// The owner array (-1 empty, -2 shared, else the drop) of every cell gives
// the predicate: a shared cell, or a cell of one drop with a six-neighbour
// not owned by it. Block counts (kBlock cells) and one bit per cell, for
// compact::k_write_ordered_bits: lane l of a wavefront holds cell p (64
// consecutive cells), its x neighbours come from the lanes beside it, and
// only a row's end cells and the wavefront's edge lanes load theirs. The y
// and z neighbours are loaded for cells of one drop only.
__global__ __launch_bounds__(kBlock) void k_pair_source_counts(const int32_t *__restrict__ own, int nx, int ny,
                                                               int nz, FastDiv fnx, FastDiv fny, int64_t n,
                                                               int32_t *__restrict__ bc, uint64_t *__restrict__ bits) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool in = p < n;
  const int64_t pc = in ? p : n - 1;  // (a lane past the end shadows the last cell)
  const int32_t a = own[pc];
  const uint32_t r = fast_div((uint32_t)pc, fnx), zz = fast_div(r, fny);
  const int x = (int)((uint32_t)pc - r * (uint32_t)nx), y = (int)(r - zz * (uint32_t)ny), z = (int)zz;
  const int64_t row = (int64_t)r * nx;
  // x neighbours: from the lanes beside, unless across the wavefront's edge or the row's end
  int32_t am = __shfl_up(a, 1, 64), ap = __shfl_down(a, 1, 64);
  const bool load_m = lane == 0 || x == 0, load_p = lane == 63 || x == nx - 1;
  if (a >= 0 && load_m) am = own[row + wrap_dec(x, nx)];
  if (a >= 0 && load_p) ap = own[row + wrap_inc(x, nx)];
  bool hit = false;
  if (a == -2) {
    hit = true;
  } else if (a >= 0) {
    const int64_t plane = (int64_t)ny * nx, zr = (int64_t)z * plane;
    const int32_t ym = own[zr + (int64_t)wrap_dec(y, ny) * nx + x], yp = own[zr + (int64_t)wrap_inc(y, ny) * nx + x];
    const int32_t zm = own[(int64_t)wrap_dec(z, nz) * plane + (int64_t)y * nx + x];
    const int32_t zp = own[(int64_t)wrap_inc(z, nz) * plane + (int64_t)y * nx + x];
    hit = !(am == a && ap == a && ym == a && yp == a && zm == a && zp == a);
  }
  hit = hit && in;
  __shared__ int wc[kBlock / 64];
  const uint64_t mask = __ballot(hit);
  if (lane == 0) {
    wc[threadIdx.x >> 6] = (int)__popcll(mask);
    if (in) bits[p >> 6] = mask;  // (a wavefront wholly past n has no word)
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += wc[w];
    bc[blockIdx.x] = t;
  }
}

// Near-contact pairs seen from the listed cells (persistent grid).
__global__ __launch_bounds__(kBlock) void k_edges(const int32_t *__restrict__ own, const int32_t *__restrict__ lab,
                                                  int nx, int ny, int nz, int ntr, TracerOffsets to,
                                                  const int4 *__restrict__ offs, int noffs, int small_offsets,
                                                  const int32_t *__restrict__ list, const int32_t *__restrict__ count,
                                                  uint32_t *__restrict__ adj, int64_t words, FastDiv fnx,
                                                  FastDiv fny, const int32_t *__restrict__ cross_T0) {
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int nlist = *count;
  for (int qi = blockIdx.x * kBlock + threadIdx.x; qi < nlist; qi += gridDim.x * kBlock) {
    const int64_t p = list[qi];
    edges_of(own, lab, nx, ny, nz, ntr, to, offs, noffs, small_offsets, adj, words, n3, fnx, fny, cross_T0, p);
  }
}

// Occupancy of every 64-cell row segment of every tracer: bit l of word
// occ[t][z][y][w] is (label > 0) of cell x = 64 w + l (0 beyond the row).
__global__ __launch_bounds__(kBlock) void k_occ_words(const int32_t *__restrict__ lab, int nx, int64_t rows,
                                                      int words, uint64_t *__restrict__ occ) {
  const int64_t seg = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t nseg = rows * words;
  if (seg >= nseg) return;  // whole wavefront
  const int64_t row = seg / words;
  const int w = (int)(seg - row * words);
  const int x = 64 * w + lane;
  const bool occ_ = x < nx && lab[row * nx + x] > 0;
  const uint64_t b = __ballot(occ_);
  if (lane == 0) occ[seg] = b;
}

// Bit m of v (m < 16) to bit 4m.
__device__ __forceinline__ uint64_t spread4(uint64_t v) {
  v &= 0xFFFFull;
  v = (v | (v << 24)) & 0x000000FF000000FFull;
  v = (v | (v << 12)) & 0x000F000F000F000Full;
  v = (v | (v << 6)) & 0x0303030303030303ull;
  v = (v | (v << 3)) & 0x1111111111111111ull;
  return v;
}

// The same words when rows hold a multiple of 256 cells: one wavefront per
// four segments of a row, each lane loading four labels at once (cells
// 4l .. 4l+3 of the 256); ballot k holds component k of every lane, and the
// word of segment j interleaves 16 bits of each ballot.
__global__ __launch_bounds__(kBlock) void k_occ_words4(const int4 *__restrict__ lab4, int64_t ngroups,
                                                       uint64_t *__restrict__ occ) {
  const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (g >= ngroups) return;  // whole wavefront
  const int4 v = lab4[g * 64 + lane];  // segments 4g .. 4g+3 are cells 256g .. 256g+255 of the fields
  const uint64_t b0 = __ballot(v.x > 0), b1 = __ballot(v.y > 0), b2 = __ballot(v.z > 0), b3 = __ballot(v.w > 0);
  if (lane < 4) {
    const int sh = 16 * lane;
    occ[4 * g + lane] = spread4(b0 >> sh) | (spread4(b1 >> sh) << 1) | (spread4(b2 >> sh) << 2) |
                        (spread4(b3 >> sh) << 3);
  }
}

// Bits of cells xs, xs+1, ..., xs+63 (periodic in x, xs any integer) of one
// row of occupancy words. Windows inside the row take two aligned words; the
// rest (the row's ends, rows shorter than 64 cells) assemble the bits piece by
// piece.
__device__ __forceinline__ uint64_t row_window(const uint64_t *__restrict__ rw, int nx, int xs) {
  if (xs >= 0 && xs + 64 <= nx) {
    const int w = xs >> 6, b = xs & 63;
    return b == 0 ? rw[w] : ((rw[w] >> b) | (rw[w + 1] << (64 - b)));
  }
  int x = wrap_any(xs, nx);
  uint64_t res = 0;
  int got = 0;
  while (got < 64) {
    const int b = x & 63;
    int take = 64 - b;
    if (take > nx - x) take = nx - x;
    if (take > 64 - got) take = 64 - got;
    uint64_t chunk = rw[x >> 6] >> b;
    if (take < 64) chunk &= (1ull << take) - 1ull;
    res |= chunk << got;
    got += take;
    x += take;
    if (x == nx) x = 0;
  }
  return res;
}

// One of each opposite pair of offsets o of the 5x5x5 stencil (o > 0 in
// (z, y, x) order): 62 pairs, as (ox, oy, oz) in -2..2.
struct StencilPairs {
  int8_t o[62][3];
};
static StencilPairs make_stencil_pairs() {
  StencilPairs sp{};
  int k = 0;
  for (int oz = -2; oz <= 2; ++oz)
    for (int oy = -2; oy <= 2; ++oy)
      for (int ox = -2; ox <= 2; ++ox)
        if (oz > 0 || (oz == 0 && (oy > 0 || (oy == 0 && ox > 0)))) {
          sp.o[k][0] = (int8_t)ox;
          sp.o[k][1] = (int8_t)oy;
          sp.o[k][2] = (int8_t)oz;
          ++k;
        }
  return sp;
}

// Steps 1-3 within tracer t for the 64 cells of one row segment. Lane k < 62
// takes the opposite pair k of the stencil, offsets +o and -o, and forms over
// the segment's cells at once, from three 64-bit windows of occupancy bits,
// the cells whose centre is empty (label 0) and whose cells at +o and -o are
// both occupied; for each such cell it loads the two labels and records the
// two drops as neighbours when they differ (Step 3). Every pair is tested for
// every cell, as in the definition; a lane's bit operations replace 64
// per-cell tests.
constexpr int kStencilSegs = 16;  // segments per wavefront of k_stencil_edges (1: 5.32 ms, 4: 4.92, 8: 4.76, 16: 4.64 at 512^3 x 8)
__global__ __launch_bounds__(kBlock) void k_stencil_edges(const int32_t *__restrict__ lab,
                                                          const uint64_t *__restrict__ occ, int nx, int ny, int nz,
                                                          int ntr, int words, TracerOffsets to, StencilPairs sp,
                                                          uint32_t *__restrict__ adj, int64_t awords, FastDiv fw,
                                                          FastDiv frows, FastDiv fny) {
  const int lane = threadIdx.x & 63;
  const int64_t rows = (int64_t)nz * ny;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  for (int ks = 0; ks < kStencilSegs; ++ks) {  // consecutive segments of one wavefront
  const int64_t seg = wave * kStencilSegs + ks;
  if (seg >= (int64_t)ntr * rows * words) return;  // whole wavefront
  // (t, z, y) row of all tracers and word w: segment counts stay below 2^31,
  // so the divisions are 32-bit multiply-shifts
  const uint32_t tr = fast_div((uint32_t)seg, fw);
  const int w = (int)((uint32_t)seg - tr * (uint32_t)words);
  const uint32_t t32 = fast_div(tr, frows);
  const int t = (int)t32;
  const int64_t r = (int64_t)(tr - t32 * (uint32_t)rows);
  const uint32_t z32 = fast_div((uint32_t)r, fny);
  const int z = (int)z32, y = (int)((uint32_t)r - z32 * (uint32_t)ny);
  const uint64_t *occ_t = occ + (int64_t)t * rows * words;
  const int x0 = 64 * w;
  // offsets reach 2 cells: one conditional wrap when the axis has 3 cells or more
  auto wrap2 = [](int v, int n) { return n >= 3 ? (v < 0 ? v + n : (v >= n ? v - n : v)) : wrap_any(v, n); };
  const int nvalid = nx - x0 < 64 ? nx - x0 : 64;
  const uint64_t valid = nvalid == 64 ? ~0ull : ((1ull << nvalid) - 1ull);
  const uint64_t empty = ~occ_t[r * words + w] & valid;  // bit i: cell x0 + i has no drop of tracer t
  uint64_t cand = 0;
  int ox = 0, oy = 0, oz = 0;
  if (lane < 62) {
    ox = sp.o[lane][0];
    oy = sp.o[lane][1];
    oz = sp.o[lane][2];
    const uint64_t *rp = occ_t + ((int64_t)wrap2(z + oz, nz) * ny + wrap2(y + oy, ny)) * words;
    const uint64_t *rm = occ_t + ((int64_t)wrap2(z - oz, nz) * ny + wrap2(y - oy, ny)) * words;
    // bit i: cell x0 + i + ox of the row at +o, cell x0 + i - ox of the row at -o
    cand = row_window(rp, nx, x0 + ox) & row_window(rm, nx, x0 - ox) & empty;
  }
  if (__ballot(cand != 0ull) == 0ull) continue;  // no pair around any empty cell of the segment
  const int64_t rowp = ((int64_t)t * nz + wrap2(z + oz, nz)) * ny + wrap2(y + oy, ny);
  const int64_t rowm = ((int64_t)t * nz + wrap2(z - oz, nz)) * ny + wrap2(y - oy, ny);
  const int64_t qc = (((int64_t)t * nz + z) * ny + y) * nx + x0;  // a cell of the segment (x0 < nx)
  // The labels of up to kBatch cells are loaded together (every lane loads,
  // from the segment's first cell when it has no cell left, and selects
  // afterwards); a pair of drops just recorded by this lane is not recorded
  // again (the cells of a gap between two drops mostly see the same pair).
  constexpr int kBatch = 8;
  int32_t last_a = 0, last_b = 0;
  while (cand) {
    int32_t la[kBatch], lb[kBatch];
    bool has[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      has[u] = cand != 0ull;
      const int i = has[u] ? __ffsll((unsigned long long)cand) - 1 : 0;
      cand &= cand - 1;
      const int x = x0 + i;
      const int64_t qp = rowp * nx + wrap2(x + ox, nx), qm = rowm * nx + wrap2(x - ox, nx);
      la[u] = lab[has[u] ? qp : qc];
      lb[u] = lab[has[u] ? qm : qc];
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int32_t a = la[u], b = lb[u];
      if (has[u] && a != b && a > 0 && b > 0 && to.off[t] + a <= to.off[t + 1] && to.off[t] + b <= to.off[t + 1] &&
          !(a == last_a && b == last_b)) {
        const int32_t ga = to.off[t] + a - 1, gb = to.off[t] + b - 1;
        set_edge(adj, awords, ga, gb);
        set_edge(adj, awords, gb, ga);
        last_a = a;
        last_b = b;
      }
    }
  }
  }
}

// Occupancy of the other tracers: word (row, w) of others[t] is the OR of
// that word of occ[u] over every tracer u != t (prefix ORs going up, suffix
// ORs coming down). nseg1: words per tracer.
__global__ __launch_bounds__(kBlock) void k_other_tracers(const uint64_t *__restrict__ occ, int64_t nseg1, int ntr,
                                                          uint64_t *__restrict__ others) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nseg1) return;
  uint64_t acc = 0;
  for (int t = 0; t < ntr; ++t) {
    others[(int64_t)t * nseg1 + i] = acc;
    acc |= occ[(int64_t)t * nseg1 + i];
  }
  acc = 0;
  for (int t = ntr - 1; t >= 0; --t) {
    others[(int64_t)t * nseg1 + i] |= acc;
    acc |= occ[(int64_t)t * nseg1 + i];
  }
}

// Stencil mode, contacts across tracers (persistent grid over the listed
// cells): the pairs k_edges finds with the half cube max|o_a| <= 4, where
// only drops of different tracers are related. A listed cell p of a single
// drop a, of tracer t, takes the cube row by row: a 9-bit window of others[t]
// (cells x-4 .. x+4 of the row; x+1 .. x+4 in its own row) marks the cells
// that hold a drop of another tracer, and only their owners are loaded. A
// cell with no other tracer can pair a with no drop of another tracer, so the
// edges are those of the full scan. Shared cells take the full scan.
__global__ __launch_bounds__(kBlock) void k_edges_cross(const int32_t *__restrict__ own,
                                                        const int32_t *__restrict__ lab, const uint64_t *__restrict__ others,
                                                        int nx, int ny, int nz, int ntr, int xw, TracerOffsets to,
                                                        const int4 *__restrict__ offs, int noffs, int small_offsets,
                                                        const int32_t *__restrict__ list,
                                                        const int32_t *__restrict__ count, uint32_t *__restrict__ adj,
                                                        int64_t words, FastDiv fnx, FastDiv fny,
                                                        const int32_t *__restrict__ T0) {
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int64_t nseg1 = (int64_t)nz * ny * xw;
  const int nlist = *count;
  for (int qi = blockIdx.x * kBlock + threadIdx.x; qi < nlist; qi += gridDim.x * kBlock) {
    const int64_t p = list[qi];
    const int32_t a = own[p];
    if (a < 0) {  // a shared cell
      edges_of(own, lab, nx, ny, nz, ntr, to, offs, noffs, small_offsets, adj, words, n3, fnx, fny, T0, p);
      continue;
    }
    const uint32_t r = fast_div((uint32_t)p, fnx), zz = fast_div(r, fny);  // cells < 2^31
    const int x = (int)((uint32_t)p - r * (uint32_t)nx), y = (int)(r - zz * (uint32_t)ny), z = (int)zz;
    const int ta = T0[a];
    const uint64_t *ot = others + (int64_t)ta * nseg1;
    int32_t last_b = -1;
    auto visit = [&](int64_t q) {
      const int32_t b = own[q];
      if (b == -1 || b == last_b) return;
      if (b >= 0) {
        if (T0[b] != ta) {
          set_edge(adj, words, a, b);
          last_b = b;
        }
      } else {
        for_drops_at(lab, n3, ntr, to, q, [&](int32_t v) {
          if (T0[v] != ta) set_edge(adj, words, a, v);
        });
      }
    };
    // the 40 rows of the half cube: (dz, dy) = (0, 1..4) and (1..4, -4..4)
    for (int dz = 0; dz <= 4; ++dz)
      for (int dy = (dz == 0 ? 1 : -4); dy <= 4; ++dy) {
        const int64_t row = (int64_t)wrap_any(z + dz, nz) * ny + wrap_any(y + dy, ny);
        uint64_t m = row_window(ot + row * xw, nx, x - 4) & 0x1FFull;
        while (m) {
          const int i = __ffsll((unsigned long long)m) - 1;
          m &= m - 1;
          visit(row * nx + wrap_any(x - 4 + i, nx));
        }
      }
    // the cell's own row: x+1 .. x+4
    {
      const int64_t row = (int64_t)z * ny + y;
      uint64_t m = row_window(ot + row * xw, nx, x + 1) & 0xFull;
      while (m) {
        const int i = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        visit(row * nx + wrap_any(x + 1 + i, nx));
      }
    }
  }
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Degree of every drop (symmetrise first: a bit set in either direction).
__global__ __launch_bounds__(kBlock) void k_degree(uint32_t *__restrict__ adj, int32_t D, int64_t words,
                                                   int32_t *__restrict__ deg) {
  const int32_t g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= D) return;
  int s = 0;
  for (int64_t w = 0; w < words; ++w) s += __popc(adj[(int64_t)g * words + w]);
  deg[g] = s;
}

__global__ __launch_bounds__(kBlock) void k_symmetrise(uint32_t *adj, int32_t D, int64_t words) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= (int64_t)D * D) return;
  const int32_t a = (int32_t)(i / D), b = (int32_t)(i % D);
  if (a >= b) return;
  const bool ab = (adj[(int64_t)a * words + (b >> 5)] >> (b & 31)) & 1u;
  const bool ba = (adj[(int64_t)b * words + (a >> 5)] >> (a & 31)) & 1u;
  if (ab && !ba) atomicOr(&adj[(int64_t)b * words + (a >> 5)], 1u << (a & 31));
  if (ba && !ab) atomicOr(&adj[(int64_t)a * words + (b >> 5)], 1u << (b & 31));
}

// Exclusive scan of D degrees (single workgroup) into rowptr[0..D].
__global__ __launch_bounds__(1024) void k_scan_deg(const int32_t *__restrict__ deg, int32_t D,
                                                   int32_t *__restrict__ rowptr) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = ((int64_t)D + 1023) / 1024;
  const int64_t lo = t * per, hi = (lo + per < D) ? lo + per : D;
  int64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += deg[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t add = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int64_t run = (t == 0) ? 0 : part[t - 1];
  for (int64_t i = lo; i < hi; ++i) {
    rowptr[i] = (int32_t)run;
    run += deg[i];
  }
  if (t == 1023) rowptr[D] = (int32_t)part[1023];
}

__global__ __launch_bounds__(kBlock) void k_csr_fill(const uint32_t *__restrict__ adj, int32_t D, int64_t words,
                                                     const int32_t *__restrict__ rowptr, int32_t *__restrict__ nbr) {
  const int32_t g = blockIdx.x * kBlock + threadIdx.x;
  if (g >= D) return;
  int32_t e = rowptr[g];
  for (int64_t w = 0; w < words; ++w) {
    uint32_t bits = adj[(int64_t)g * words + w];
    while (bits) {
      const int b = __ffs(bits) - 1;
      bits &= bits - 1;
      nbr[e++] = (int32_t)(w * 32 + b);
    }
  }
}

// The greedy pass, one wavefront. T0: initial tracer per drop. Outputs
// new_tracer, and res[0] = tracers after, res[1] = moved drops, res[2] = 1 on
// capacity overflow (then new_tracer is meaningless and nothing is moved).
__global__ __launch_bounds__(64) void k_greedy(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ nbr,
                                               const int32_t *__restrict__ T0, int32_t D, int ntr, int max_tracers,
                                               int32_t *__restrict__ new_tracer, int32_t *__restrict__ res) {
  __shared__ int8_t T[kMaxDrops];
  __shared__ int32_t stage[kChunk];
  const int lane = threadIdx.x;
  for (int32_t g = lane; g < D; g += 64) T[g] = (int8_t)T0[g];
  __syncthreads();
  int N = ntr;
  int32_t moved = 0;
  int overflow = 0;
  int32_t base = 0;  // first neighbour index staged
  int32_t staged_end = 0;
  for (int32_t g = 0; g < D && !overflow; ++g) {
    const int32_t e0 = rowptr[g], e1 = rowptr[g + 1];
    const int tg = T[g];
    bool conflict = false;
    uint64_t used = 0;
    for (int32_t e = e0; e < e1; e += 64) {
      // make sure [e, min(e+64, e1)) is staged
      if (e + 64 > staged_end && staged_end < e1) {
        __syncthreads();
        base = e;
        staged_end = (base + kChunk < rowptr[D]) ? base + kChunk : rowptr[D];
        for (int32_t k = lane; k < staged_end - base; k += 64) stage[k] = nbr[base + k];
        __syncthreads();
      }
      const int32_t idx = e + lane;
      bool c = false;
      uint64_t u = 0;
      if (idx < e1) {
        const int32_t h = stage[idx - base];
        const int th = T[h];
        c = (h < g) && (th == tg);
        u = 1ull << th;
      }
      conflict = conflict || (__ballot(c) != 0ull);
      // OR-reduction of the tracer masks across the wavefront
#pragma unroll
      for (int s = 32; s > 0; s >>= 1) u |= __shfl_xor(u, s, 64);
      used |= u;
    }
    if (!conflict) continue;
    uint64_t avail = ~used & ~(1ull << tg);
    if (N < 64) avail &= (1ull << N) - 1;
    int n;
    if (avail) {
      n = __ffsll((unsigned long long)avail) - 1;
    } else {
      if (N + 1 > max_tracers) {
        overflow = 1;
        break;
      }
      n = N++;
    }
    __syncthreads();
    if (lane == 0) T[g] = (int8_t)n;
    ++moved;
    __syncthreads();
  }
  __syncthreads();
  for (int32_t g = lane; g < D; g += 64) new_tracer[g] = T[g];
  if (lane == 0) {
    res[0] = N;
    res[1] = moved;
    res[2] = overflow;
  }
}

// The same greedy pass decided in rounds by one workgroup. A drop's decision
// reads the final tracers of its earlier neighbours and the initial tracers
// of its later ones (a later neighbour cannot be decided before it), and the
// number of tracers in use, which changes only when a drop needs a new
// tracer. With no new tracer, a drop can be decided as soon as all its
// earlier neighbours are, and the result is the sequential pass's: each round
// decides every such drop (the smallest undecided drop always is one, so the
// rounds end), then applies the decisions. If some drop needs a new tracer,
// res[3] = 1 and the caller runs the sequential pass instead.
__global__ __launch_bounds__(1024) void k_greedy_rounds(const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ nbr,
                                                        const int32_t *__restrict__ T0, int32_t D, int ntr,
                                                        int32_t *__restrict__ new_tracer, int32_t *__restrict__ res) {
  __shared__ int8_t T[kMaxDrops];
  __shared__ int8_t dec[kMaxDrops];  // this round's decisions, -1 for none
  __shared__ uint32_t done[kMaxDrops / 32];
  __shared__ int s_changed, s_moved, s_new;
  const int tid = threadIdx.x;
  for (int32_t g = tid; g < D; g += 1024) {
    T[g] = (int8_t)T0[g];
    dec[g] = -1;
  }
  for (int32_t i = tid; i < kMaxDrops / 32; i += 1024) done[i] = 0u;
  if (tid == 0) {
    s_moved = 0;
    s_new = 0;
  }
  const uint64_t inuse = (ntr < 64) ? ((1ull << ntr) - 1) : ~0ull;
  while (true) {
    __syncthreads();
    if (tid == 0) s_changed = 0;
    __syncthreads();
    for (int32_t g = tid; g < D; g += 1024) {
      if ((done[g >> 5] >> (g & 31)) & 1u) continue;
      const int tg = T[g];
      bool ready = true, conflict = false;
      uint64_t used = 0;
      for (int32_t e = rowptr[g]; e < rowptr[g + 1]; ++e) {
        const int32_t h = nbr[e];
        if (h < g && !((done[h >> 5] >> (h & 31)) & 1u)) {
          ready = false;
          break;
        }
        const int th = T[h];
        conflict = conflict || (h < g && th == tg);
        used |= 1ull << th;
      }
      if (!ready) continue;
      int n = tg;
      if (conflict) {
        const uint64_t avail = ~used & ~(1ull << tg) & inuse;
        if (avail) n = __ffsll((unsigned long long)avail) - 1;
        else s_new = 1;
        atomicAdd(&s_moved, 1);
      }
      dec[g] = (int8_t)n;
      s_changed = 1;
    }
    __syncthreads();
    if (!s_changed || s_new) break;  // uniform: read after the barrier
    for (int32_t g = tid; g < D; g += 1024)
      if (dec[g] >= 0) {
        T[g] = dec[g];
        dec[g] = -1;
        atomicOr(&done[g >> 5], 1u << (g & 31));
      }
  }
  for (int32_t g = tid; g < D; g += 1024) new_tracer[g] = T[g];
  if (tid == 0) {
    res[0] = ntr;
    res[1] = s_moved;
    res[2] = 0;
    res[3] = s_new;
  }
}

__global__ void k_initial_tracers(int32_t *T0, int32_t D, int ntr, TracerOffsets to) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= D) return;
  int t = 0;
  while (t + 1 < ntr && to.off[t + 1] <= g) ++t;
  T0[g] = t;
}

// Move the cells of every moved drop: first clear every moved-out value of
// the cell, then add each to its new field.
// Moves the cells of every drop whose tracer changes: the old field is
// cleared first, then the values are added to the new fields. A cell owned by
// one drop (own >= 0, tracer T0[own]) needs only the owner array; cells
// shared by several drops read every tracer's labels.
__global__ __launch_bounds__(kBlock) void k_move(double *__restrict__ c, const int32_t *__restrict__ lab, int64_t n3,
                                                 int ntr, TracerOffsets to, const int32_t *__restrict__ own,
                                                 const int32_t *__restrict__ T0, const int32_t *__restrict__ newt) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= n3) return;
  const int32_t o = own[p];
  if (o == -1) return;
  if (o >= 0) {
    const int t = T0[o], n = newt[o];
    if (n == t) return;
    double *src = c + (int64_t)t * n3 + p, *dst = c + (int64_t)n * n3 + p;
    const double v = *src;
    *src = 0.0;
    *dst = *dst + v;
    return;
  }
  int cnt = 0;
  for (int t = 0; t < ntr; ++t) {
    const int32_t l = lab[(int64_t)t * n3 + p];
    if (l > 0 && to.off[t] + l <= to.off[t + 1] && newt[to.off[t] + l - 1] != t) ++cnt;
  }
  if (cnt == 0) return;
  double vals[kMaxTracers];
  int dst[kMaxTracers];
  int k = 0;
  for (int t = 0; t < ntr; ++t) {
    const int32_t l = lab[(int64_t)t * n3 + p];
    if (l <= 0 || to.off[t] + l > to.off[t + 1]) continue;
    const int n = newt[to.off[t] + l - 1];
    if (n == t) continue;
    vals[k] = c[(int64_t)t * n3 + p];
    dst[k] = n;
    c[(int64_t)t * n3 + p] = 0.0;
    ++k;
  }
  for (int u = 0; u < k; ++u) {
    double *q = c + (int64_t)dst[u] * n3 + p;
    *q = *q + vals[u];
  }
}

// Sum of the retired tracers' fields for the compaction: workgroup b sums
// cells [b*chunk, (b+1)*chunk) of the concatenation of the retired fields
// (strided per thread, then a fixed tree); k_sum_parts adds the parts in
// order. Reproducible bit for bit.
constexpr int kSumBlock = 256;
__global__ __launch_bounds__(kSumBlock) void k_sum_retired(const double *__restrict__ c, const int32_t *__restrict__ which,
                                                          int nret, int64_t n3, int64_t chunk,
                                                          double *__restrict__ part) {
  const int64_t total = (int64_t)nret * n3;
  const int64_t q0 = (int64_t)blockIdx.x * chunk;
  const int64_t q1 = q0 + chunk < total ? q0 + chunk : total;
  double acc = 0.0;
  int64_t r = (q0 + threadIdx.x) / n3, rend = (r + 1) * n3;  // field of q, and where it ends
  for (int64_t q = q0 + threadIdx.x; q < q1; q += kSumBlock) {
    while (q >= rend) {  // (a field holds at least one cell: n3 >= 1)
      ++r;
      rend += n3;
    }
    acc += c[(int64_t)which[r] * n3 + (q - (rend - n3))];
  }
  __shared__ double red[kSumBlock];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kSumBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void k_sum_parts(const double *__restrict__ part, int n, double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  *out = s;
}

}  // namespace

// Both recolouring modes: stencil == 0 relates drops within the distance
// threshold gap_cells, stencil != 0 by the literal 5x5x5 criterion (gap_cells
// unused). `fn` names the entry point in error messages.
static int recolor_impl(vofmt_ctx *ctx, const char *fn, int stencil, int32_t nx, int32_t ny, int32_t nz,
                        int32_t *ntracers_host, int32_t max_tracers, double *c, const int32_t *labels,
                        const int32_t *ndrops_host, double gap_cells, int32_t *new_tracer, int32_t *nmoved_host,
                        hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (!ntracers_host || !nmoved_host || !ndrops_host) return set_err(ctx, VOFMT_E_ARG, "%s: null host pointer", fn);
  const int ntr = *ntracers_host;
  if (nx < 1 || ny < 1 || nz < 1 || ntr < 0 || ntr > max_tracers || max_tracers > kMaxTracers ||
      (!stencil && (!(gap_cells >= 0.0) || gap_cells > 64.0)))
    return set_err(ctx, VOFMT_E_ARG, "%s: bad arguments (ntracers=%d max_tracers=%d (<= %d) gap=%g)", fn, ntr,
                   max_tracers, kMaxTracers, gap_cells);
  *nmoved_host = 0;
  if (ntr == 0) return VOFMT_OK;
  if (!c || !labels) return set_err(ctx, VOFMT_E_ARG, "%s: null pointer", fn);
  TracerOffsets to;
  to.off[0] = 0;
  int64_t D = 0;
  for (int t = 0; t < ntr; ++t) {
    if (ndrops_host[t] < 0) return set_err(ctx, VOFMT_E_ARG, "%s: negative drop count", fn);
    D += ndrops_host[t];
    to.off[t + 1] = (int32_t)D;
  }
  for (int t = ntr + 1; t <= kMaxTracers; ++t) to.off[t] = (int32_t)D;
  if (D == 0) return VOFMT_OK;
  if (D > kMaxDrops) return set_err(ctx, VOFMT_E_ARG, "%s: more than %d drops", fn, kMaxDrops);
  if (!new_tracer) return set_err(ctx, VOFMT_E_ARG, "%s: null new_tracer", fn);
  const int64_t n3 = (int64_t)nx * ny * nz;
  if (n3 >= INT32_MAX) return set_err(ctx, VOFMT_E_ARG, "%s: more than 2^31-1 cells per field", fn);
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  // Offsets scanned from the listed cells, one of each opposite pair (o > 0
  // in (z, y, x) order): a pair of drops is found from one side only, and
  // k_symmetrise completes the adjacency.
  // - distance mode: the half ball |o|^2 < (1+gap)^2. Every pair is still
  //   found: the two cells of the pair at the smallest offset are both listed
  //   (a cell whose six neighbours all held its drop would have a neighbour
  //   closer to the other drop), so the listed cell from which that offset
  //   points forward finds it;
  // - stencil mode (contacts across tracers): the half cube max|o_a| <= 4.
  //   A pair of cells at the smallest (max|o_a|, sum|o_a|) is listed on both
  //   sides: an axis step from an interior cell towards the other drop
  //   lowers the sum and does not raise the maximum.
  const int R = stencil ? 4 : (int)floor(1.0 + gap_cells);
  const double lim = stencil ? 1e300 : (1.0 + gap_cells) * (1.0 + gap_cells);
  int4 *hoffs = nullptr;
  int noffs = 0;
  {
    const int side = 2 * R + 1;
    hoffs = (int4 *)malloc(sizeof(int4) * (size_t)side * side * side);
    for (int oz = -R; oz <= R; ++oz)
      for (int oy = -R; oy <= R; ++oy)
        for (int ox = -R; ox <= R; ++ox) {
          const double o2 = (double)(ox * ox + oy * oy + oz * oz);
          if (o2 == 0.0 || !(o2 < lim)) continue;
          if (!(oz > 0 || (oz == 0 && (oy > 0 || (oy == 0 && ox > 0))))) continue;
          hoffs[noffs++] = make_int4(ox, oy, oz, 0);
        }
  }
  const int64_t words = (D + 31) / 32;
  int32_t *own = (int32_t *)scratch(ctx, SLOT_LABEL_B, sizeof(int32_t) * (size_t)n3);
  uint32_t *adj = (uint32_t *)scratch(ctx, SLOT_LABEL_A, sizeof(uint32_t) * (size_t)(D * words));
  int32_t *small = (int32_t *)scratch(ctx, SLOT_LABEL_C, sizeof(int32_t) * (size_t)(4 * D + 16));
  int4 *doffs = (int4 *)scratch(ctx, SLOT_MISC2, sizeof(int4) * (size_t)(noffs > 0 ? noffs : 1));
  // pinned staging: results in the first 256 bytes, offsets after them
  int32_t *hres = (int32_t *)host_scratch(ctx, 256 + sizeof(int4) * (size_t)noffs);
  if (!own || !adj || !small || !doffs || !hres) {
    free(hoffs);
    return VOFMT_E_NOMEM;
  }
  memcpy(hres + 64, hoffs, sizeof(int4) * noffs);
  free(hoffs);
  if (noffs > 0)
    VOFMT_HIP(ctx, hipMemcpyAsync(doffs, hres + 64, sizeof(int4) * noffs, hipMemcpyHostToDevice, stream));
  const int small_offsets = (R < nx && R < ny && R < nz) ? 1 : 0;
  int32_t *deg = small, *rowptr = small + D, *T0 = small + 2 * D + 1, *res = small + 3 * D + 2;
  int32_t *nbr = nullptr;
  const unsigned nbc = ceil_div(n3, kBlock);
  if (n3 % 4 == 0 && ((uintptr_t)labels & 15) == 0)
    hipLaunchKernelGGL(k_owner4, dim3(ceil_div(n3 / 4, kBlock)), dim3(kBlock), 0, stream, (const int4 *)labels,
                       n3 / 4, ntr, to, (int4 *)own);
  else
    hipLaunchKernelGGL(k_owner, dim3(nbc), dim3(kBlock), 0, stream, labels, n3, ntr, to, own);
  hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, stream, adj, D * words, 0u);
  // initial tracer of every drop (the stencil mode's cross-tracer filter reads it)
  hipLaunchKernelGGL(k_initial_tracers, dim3(ceil_div(D, 256)), dim3(256), 0, stream, T0, (int32_t)D, ntr, to);
  uint64_t *others = nullptr;
  int xw_stencil = 0;
  if (stencil) {
    // Steps 1-3 within every tracer, on occupancy bits per row segment
    const int xw = (int)ceil_div(nx, 64);
    const int64_t rows = (int64_t)nz * ny;
    const int64_t nseg = (int64_t)ntr * rows * xw;
    uint64_t *occ = (uint64_t *)scratch(ctx, SLOT_OCC, sizeof(uint64_t) * (size_t)nseg);
    if (!occ) return VOFMT_E_NOMEM;
    const int64_t nblk = (nseg * 64 + kBlock - 1) / kBlock;
    const int64_t nblk_se = (ceil_div(nseg, kStencilSegs) * 64 + kBlock - 1) / kBlock;  // k_stencil_edges
    if (nblk > INT32_MAX || nseg >= INT32_MAX) return set_err(ctx, VOFMT_E_ARG, "%s: grid too large", fn);
    if (nx % 256 == 0 && ((uintptr_t)labels & 15) == 0) {
      const int64_t ngroups = nseg / 4;  // rows of whole 256-cell groups: segment 4g + j is cells 64(4g + j) ..
      hipLaunchKernelGGL(k_occ_words4, dim3((unsigned)((ngroups * 64 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                         stream, (const int4 *)labels, ngroups, occ);
    } else {
      hipLaunchKernelGGL(k_occ_words, dim3((unsigned)nblk), dim3(kBlock), 0, stream, labels, nx,
                         (int64_t)ntr * rows, xw, occ);
    }
    hipLaunchKernelGGL(k_stencil_edges, dim3((unsigned)nblk_se), dim3(kBlock), 0, stream, labels, occ, nx, ny, nz, ntr,
                       xw, to, make_stencil_pairs(), adj, words, make_fastdiv((uint32_t)xw),
                       make_fastdiv((uint32_t)rows), make_fastdiv((uint32_t)ny));
    // the other tracers' occupancy, for the contacts across tracers
    const int64_t nseg1 = rows * xw;
    others = (uint64_t *)scratch(ctx, SLOT_OCC_OTHERS, sizeof(uint64_t) * (size_t)nseg);
    if (!others) return VOFMT_E_NOMEM;
    hipLaunchKernelGGL(k_other_tracers, dim3(ceil_div(nseg1, kBlock)), dim3(kBlock), 0, stream, occ, nseg1, ntr,
                       others);
    xw_stencil = xw;
  }
  {
    // the cells that can see a pair, in order, then the pairs they see
    const int64_t lt = compact::list_tiles_if(n3);
    int32_t *srcs = (int32_t *)scratch(ctx, SLOT_RECOLOR_LIST, sizeof(int32_t) * (size_t)n3);
    int32_t *bc = (int32_t *)scratch(ctx, SLOT_MISC, sizeof(int32_t) * (size_t)nbc);
    int32_t *tot = (int32_t *)scratch(ctx, SLOT_CURV_COUNT, sizeof(int32_t) * (size_t)(lt + 2));
    uint64_t *pbits = (uint64_t *)scratch(ctx, SLOT_CURV_HF, sizeof(uint64_t) * (size_t)((n3 + 63) / 64));
    if (!srcs || !bc || !tot || !pbits) return VOFMT_E_NOMEM;
    {
      // the ordered list of those cells: counts and bits, the tiled scan, the list from the bits
      const int64_t nb = (n3 + kBlock - 1) / kBlock, nt = (nb + compact::kTile - 1) / compact::kTile;
      static_assert(kBlock == compact::kBlock, "block counts and the tiled scan share the block size");
      hipLaunchKernelGGL(k_pair_source_counts, dim3((unsigned)nb), dim3(kBlock), 0, stream, own, nx, ny, nz,
                         make_fastdiv((uint32_t)nx), make_fastdiv((uint32_t)ny), n3, bc, pbits);
      hipLaunchKernelGGL(compact::k_scan_tile, dim3((unsigned)nt), dim3(compact::kTile), 0, stream, bc, nb, tot,
                         (int64_t)0, (int64_t)0);
      hipLaunchKernelGGL(compact::k_scan_totals, dim3(1), dim3(compact::kTile), 0, stream, tot, nt, (int64_t)0);
      hipLaunchKernelGGL(compact::k_write_ordered_bits, dim3((unsigned)((nb + kBlock / 64 - 1) / (kBlock / 64))),
                         dim3(kBlock), 0, stream, n3, pbits, bc, tot, srcs);
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1)
      cus = 256;
    if (stencil)
      hipLaunchKernelGGL(k_edges_cross, dim3(8 * cus), dim3(kBlock), 0, stream, own, labels, others, nx, ny, nz, ntr,
                         xw_stencil, to, doffs, noffs, small_offsets, srcs, tot + lt, adj, words,
                         make_fastdiv((uint32_t)nx), make_fastdiv((uint32_t)ny), (const int32_t *)T0);
    else
      hipLaunchKernelGGL(k_edges, dim3(8 * cus), dim3(kBlock), 0, stream, own, labels, nx, ny, nz, ntr, to, doffs,
                         noffs, small_offsets, srcs, tot + lt, adj, words, make_fastdiv((uint32_t)nx),
                         make_fastdiv((uint32_t)ny), nullptr);
  }
  hipLaunchKernelGGL(k_symmetrise, dim3(ceil_div(D * D, kBlock)), dim3(kBlock), 0, stream, adj, (int32_t)D, words);
  hipLaunchKernelGGL(k_degree, dim3(ceil_div(D, kBlock)), dim3(kBlock), 0, stream, adj, (int32_t)D, words, deg);
  hipLaunchKernelGGL(k_scan_deg, dim3(1), dim3(1024), 0, stream, deg, (int32_t)D, rowptr);
  VOFMT_HIP(ctx, hipGetLastError());
  // the number of directed edges sizes the neighbour array
  VOFMT_HIP(ctx, hipMemcpyAsync(hres + 8, rowptr + D, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  const int64_t E = hres[8];
  nbr = (int32_t *)scratch(ctx, SLOT_MISC3, sizeof(int32_t) * (size_t)(E > 0 ? E : 1));
  if (!nbr) return VOFMT_E_NOMEM;
  hipLaunchKernelGGL(k_csr_fill, dim3(ceil_div(D, kBlock)), dim3(kBlock), 0, stream, adj, (int32_t)D, words, rowptr,
                     nbr);
  hipLaunchKernelGGL(k_greedy_rounds, dim3(1), dim3(1024), 0, stream, rowptr, nbr, T0, (int32_t)D, ntr, new_tracer,
                     res);
  VOFMT_HIP(ctx, hipGetLastError());
  VOFMT_HIP(ctx, hipMemcpyAsync(hres, res, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, stream));
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  if (hres[3]) {  // a drop needs a new tracer: the sequential pass
    hipLaunchKernelGGL(k_greedy, dim3(1), dim3(64), 0, stream, rowptr, nbr, T0, (int32_t)D, ntr, max_tracers,
                       new_tracer, res);
    VOFMT_HIP(ctx, hipGetLastError());
    VOFMT_HIP(ctx, hipMemcpyAsync(hres, res, sizeof(int32_t) * 3, hipMemcpyDeviceToHost, stream));
    VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  }
  const int Nnew = hres[0], moved = hres[1], overflow = hres[2];
  if (overflow) return set_err(ctx, VOFMT_E_CAPACITY, "%s: more than max_tracers=%d tracers needed", fn, max_tracers);
  if (moved > 0) {
    if (Nnew > ntr)
      hipLaunchKernelGGL(k_fill_f64, dim3(1024), dim3(256), 0, stream, c + (int64_t)ntr * n3,
                         (int64_t)(Nnew - ntr) * n3, 0.0);
    hipLaunchKernelGGL(k_move, dim3(nbc), dim3(kBlock), 0, stream, c, labels, n3, ntr, to, own, T0, new_tracer);
    VOFMT_HIP(ctx, hipGetLastError());
  }
  *ntracers_host = Nnew;
  *nmoved_host = moved;
  return VOFMT_OK;
}

extern "C" int vofmt_recolor_tracers(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t *ntracers_host,
                                     int32_t max_tracers, double *c, const int32_t *labels, const int32_t *ndrops_host,
                                     double gap_cells, int32_t *new_tracer, int32_t *nmoved_host, hipStream_t stream) {
  return recolor_impl(ctx, "vofmt_recolor_tracers", 0, nx, ny, nz, ntracers_host, max_tracers, c, labels,
                      ndrops_host, gap_cells, new_tracer, nmoved_host, stream);
}

extern "C" int vofmt_recolor_tracers_stencil(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz,
                                             int32_t *ntracers_host, int32_t max_tracers, double *c,
                                             const int32_t *labels, const int32_t *ndrops_host, int32_t *new_tracer,
                                             int32_t *nmoved_host, hipStream_t stream) {
  return recolor_impl(ctx, "vofmt_recolor_tracers_stencil", 1, nx, ny, nz, ntracers_host, max_tracers, c, labels,
                      ndrops_host, 0.0, new_tracer, nmoved_host, stream);
}

extern "C" int vofmt_compact_tracers(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t *ntracers_host,
                                     double *c, const int32_t *ndrops_host, int32_t *new_index_host,
                                     double *discarded_host, hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nx < 1 || ny < 1 || nz < 1 || !ntracers_host || *ntracers_host < 0)
    return set_err(ctx, VOFMT_E_ARG, "vofmt_compact_tracers: bad sizes");
  const int ntr = *ntracers_host;
  if (ntr > 0 && (!c || !ndrops_host || !new_index_host || !discarded_host))
    return set_err(ctx, VOFMT_E_ARG, "vofmt_compact_tracers: null pointer");
  if (discarded_host) *discarded_host = 0.0;
  if (ntr == 0) return VOFMT_OK;
  const int64_t n3 = (int64_t)nx * ny * nz;
  std::vector<int32_t> retired;
  int k = 0;
  for (int t = 0; t < ntr; ++t) {
    if (ndrops_host[t] < 0) return set_err(ctx, VOFMT_E_ARG, "vofmt_compact_tracers: negative drop count");
    if (ndrops_host[t] > 0) new_index_host[t] = k++;
    else {
      new_index_host[t] = -1;
      retired.push_back(t);
    }
  }
  if (retired.empty()) return VOFMT_OK;
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  // the discarded volume, before any field moves
  const int nret = (int)retired.size();
  const int64_t total = (int64_t)nret * n3;
  const int64_t chunk = (int64_t)kSumBlock * 64;
  const int64_t nparts = (total + chunk - 1) / chunk;
  if (nparts > INT32_MAX) return set_err(ctx, VOFMT_E_ARG, "vofmt_compact_tracers: fields too large");
  int32_t *which = (int32_t *)scratch(ctx, SLOT_MISC, sizeof(int32_t) * (size_t)nret);
  double *part = (double *)scratch(ctx, SLOT_MISC2, sizeof(double) * ((size_t)nparts + 1));
  double *hres = (double *)host_scratch(ctx, sizeof(double));
  if (!which || !part || !hres) return VOFMT_E_NOMEM;
  VOFMT_HIP(ctx, hipMemcpyAsync(which, retired.data(), sizeof(int32_t) * (size_t)nret, hipMemcpyHostToDevice,
                                stream));
  hipLaunchKernelGGL(k_sum_retired, dim3((unsigned)nparts), dim3(kSumBlock), 0, stream, c, which, nret, n3, chunk,
                     part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, stream, part, (int)nparts, part + nparts);
  VOFMT_HIP(ctx, hipGetLastError());
  VOFMT_HIP(ctx, hipMemcpyAsync(hres, part + nparts, sizeof(double), hipMemcpyDeviceToHost, stream));
  // kept fields move down in increasing order (each to a slot already read or retired)
  for (int t = 0; t < ntr; ++t) {
    const int d = new_index_host[t];
    if (d >= 0 && d != t)
      VOFMT_HIP(ctx, hipMemcpyAsync(c + (int64_t)d * n3, c + (int64_t)t * n3, sizeof(double) * (size_t)n3,
                                    hipMemcpyDeviceToDevice, stream));
  }
  hipLaunchKernelGGL(k_fill_f64, dim3(1024), dim3(256), 0, stream, c + (int64_t)k * n3, (int64_t)(ntr - k) * n3,
                     0.0);
  VOFMT_HIP(ctx, hipGetLastError());
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  *discarded_host = *hres;
  *ntracers_host = k;
  return VOFMT_OK;
}
