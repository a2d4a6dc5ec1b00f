// Drop labelling and drop moments.
//
// Labelling implements the tag.h step of section "The no-coalescence.h
// algorithm" (one value per region bounded by interfaces), read as the
// 6-connected periodic components of {c > c_eps}, numbered 1..K in
// increasing order of their smallest linear index.
//
// GPU scheme: union-find over row runs (atomicMin hooking, path halving).
// A segment is 64 consecutive cells of one x-row; a run is a maximal set of
// consecutive occupied cells inside one segment, and run r of segment g (in
// x order) has the id g * S + r, S a power of two no smaller than the most
// runs a segment can hold, so ids increase with the linear index of the
// runs' first cells. The run entries are stored slot-major (entry of id
// g * S + r at r * nseg + g): the first runs of consecutive segments, which
// almost every pass reads, are adjacent in memory.
//   1. occupancy: one ballot word per segment (bit l: cell 64 * seg + l is
//               occupied), read from c once; every run starts as its own root;
//   2. union:   each run is united with the runs it overlaps in the +y and
//               +z rows (one union per overlap, at the overlap's first
//               cell), and a segment's first cell with its -x neighbour (the
//               previous segment's last cell, or the row's last cell through
//               the periodic boundary); a union hooks the larger root under
//               the smaller, so every component ends rooted at its first
//               run, whatever the order of the unions. The unions inside
//               tiles of whole rows are made in LDS, each tile by one
//               workgroup (2a), then those across tile boundaries on the run
//               table (2b);
//   3. flatten: every run points at its root; roots counted per workgroup;
//   4. rank:    the counts are scanned and each root's entry becomes
//               -(1 + number of roots before it);
//   5. resolve: every other run's entry becomes its root's;
//   6. labels:  each cell reads its run's entry and writes the label, 0 for
//               empty cells.
// Passes 2-5 touch only the occupancy words and the run array (one entry per
// run); the cells are read once (pass 1) and written once (pass 6). The
// result is bit-identical to a sequential flood fill seeded in linear order.
// Every pass runs over all fields at once, the field in blockIdx.y.
#include "common.hpp"
#include "compact.hpp"

namespace {

constexpr int kBlock = 256;

// The run entries of one field: the entry of run id g * S + r at r * nseg + g.
struct RunTable {
  int32_t *P;
  int64_t nseg;
  int shift;  // log2 S
  __device__ __forceinline__ int32_t *at(int32_t id) const {
    return P + (int64_t)(id & ((1 << shift) - 1)) * nseg + (id >> shift);
  }
};

__device__ __forceinline__ int find_root(const RunTable &T, int32_t a) {
  int32_t b = *T.at(a);
  while (b != a) {
    a = b;
    b = *T.at(a);
  }
  return a;
}

// Root search with path halving: every node passed gets its grandparent as
// parent. Only nodes that are no longer roots are written, and always with
// an element of the same component of smaller index, so a concurrent hook
// is never undone for good: a hook that lands on a node that stopped being
// a root is retried by its union on the node's parent (see unite).
__device__ __forceinline__ int find_root_halving(const RunTable &T, int32_t a) {
  int32_t b = *T.at(a);
  while (b != a) {
    const int32_t g = *T.at(b);
    if (g != b) *T.at(a) = g;
    a = b;
    b = g;
  }
  return a;
}

// The parent array is read while other threads hook roots; volatile-free
// reads are fine: a stale parent still points to an element of the same
// component with a smaller-or-equal index, and the hooking loop retries
// until it installs the link on a true root.
__device__ __forceinline__ void unite(const RunTable &T, int32_t a, int32_t b) {
  while (true) {
    a = find_root_halving(T, a);
    b = find_root_halving(T, b);
    if (a == b) return;
    if (a > b) {
      int32_t t = a;
      a = b;
      b = t;
    }
    // hook root b (larger) under a (smaller)
    int32_t old = atomicMin(T.at(b), a);
    if (old == b) return;
    b = old;
  }
}

// Each wavefront walks kSegs consecutive 64-cell row segments (linear order
// of the cells is the order of (segment, lane)), so a workgroup covers
// 4 * kSegs segments.
constexpr int kSegs = 16;   // occupancy pass (1.58 ms at 512^3 x 8; 4: 1.78, 8: 1.65, 32: 1.68)
constexpr int kSegsW = 16;  // label-writing pass

// Row segment `sgi` (all segments of the field in linear order):
// row = z * ny + y, x = 64 * seg + lane. Segment counts stay below 2^31 (at
// most one segment per cell), so the divisions are 32-bit multiply-shifts.
struct Segment {
  int64_t row;
  int seg, y, z;
};
struct SegDiv {
  FastDiv words, ny;
};
__device__ __forceinline__ Segment segment_of(int64_t sgi, const SegDiv &dv) {
  Segment s;
  const uint32_t row = fast_div((uint32_t)sgi, dv.words);
  const uint32_t z = fast_div(row, dv.ny);
  s.row = row;
  s.seg = (int)((uint32_t)sgi - row * dv.words.d);
  s.y = (int)(row - z * dv.ny.d);
  s.z = (int)z;
  return s;
}
template <int KS>
__device__ __forceinline__ int64_t first_segment() {
  return (((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6) * KS;
}

// Index of the run of m that contains bit i (bit i set).
__device__ __forceinline__ int run_index(uint64_t m, int i) {
  const uint64_t starts = m & ~(m << 1);
  const uint64_t upto = (i == 63) ? ~0ull : ((2ull << i) - 1);
  return __popcll(starts & upto) - 1;
}

// Pass 1: occupancy words; run entries set to their own ids. The values of
// the wavefront's kSegs segments are all loaded before the first ballot, so
// their loads are in flight together; the run entries are then written
// 64 / kSegs runs of every segment at a time, lane l taking run l / kSegs of
// segment l % kSegs (adjacent entries for the first runs).
__global__ __launch_bounds__(kBlock) void k_label_occ(const double *__restrict__ c, double c_eps,
                                                      uint64_t *__restrict__ occ, RunTable T, int nx, int ny, int nz,
                                                      int words, SegDiv dv, int64_t nrun) {
  const int lane = threadIdx.x & 63;
  const int64_t nseg = (int64_t)ny * nz * words, s0 = first_segment<kSegs>();
  c += blockIdx.y * ((int64_t)nx * ny * nz);  // field blockIdx.y and its work arrays
  occ += blockIdx.y * nseg;
  T.P += blockIdx.y * nrun;
  double v[kSegs];
#pragma unroll
  for (int k = 0; k < kSegs; ++k) {
    v[k] = 0.0;  // not occupied: c_eps >= 0
    const int64_t sgi = s0 + k;
    if (sgi < nseg) {  // wave-uniform
      const Segment sg = segment_of(sgi, dv);
      const int x = sg.seg * 64 + lane;
      // read once in this call: a non-temporal load leaves the caches to
      // the run entries the later passes reuse
      if (x < nx) v[k] = __builtin_nontemporal_load(&c[sg.row * nx + x]);
    }
  }
  uint64_t mk[kSegs];
  int maxr = 0;
#pragma unroll
  for (int k = 0; k < kSegs; ++k) {
    const int64_t sgi = s0 + k;
    mk[k] = (sgi < nseg) ? __ballot(v[k] > c_eps) : 0ull;
    if (lane == 0 && sgi < nseg) occ[sgi] = mk[k];
    const int nr = __popcll(mk[k] & ~(mk[k] << 1));
    maxr = nr > maxr ? nr : maxr;
  }
  constexpr int kRuns = 64 / kSegs;  // runs per segment written per round
  const int k = lane % kSegs;
  uint64_t mm = mk[0];
#pragma unroll
  for (int kk = 1; kk < kSegs; ++kk) mm = (k == kk) ? mk[kk] : mm;
  const int nr = __popcll(mm & ~(mm << 1));
  for (int r0 = 0; r0 < maxr; r0 += kRuns) {  // wave-uniform
    const int r = r0 + lane / kSegs;
    if (r < nr) T.P[(int64_t)r * nseg + s0 + k] = (int32_t)(((s0 + k) << T.shift) + r);
  }
}

// Tiles of the local union pass: ty x tz rows of whole x-rows, at most
// TS segments, so every -x neighbour lies in the tile.
struct RowTiles {
  int ty, tz;  // rows per tile along y and z; ty = 0: no tiling (every union is global)
  int nty;     // tiles along y
};
// Root search and union inside a workgroup's LDS parent array (the same
// hooking and halving rules as on the global run table).
__device__ __forceinline__ int find_root_lds(int32_t *par, int a) {
  int b = par[a];
  while (b != a) {
    const int g = par[b];
    if (g != b) par[a] = g;
    a = b;
    b = g;
  }
  return a;
}
__device__ __forceinline__ void unite_lds(int32_t *par, int a, int b) {
  while (true) {
    a = find_root_lds(par, a);
    b = find_root_lds(par, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin(&par[b], a);
    if (old == b) return;
    b = old;
  }
}

// Pass 2a: unions inside tiles of rows, in LDS. Thread i holds local
// segments PER*i .. PER*i + PER-1 (ls = (lz * tye + ly) * words + seg), and
// the runs of the tile are numbered in (ls, run) order by a prefix sum of
// the per-segment run counts: the order of their global ids, so a local
// component's root (its smallest local number) is also its smallest global
// id. Every run then gets its local root's global id as its entry; the
// roots keep their own. A tile with more than CAP runs makes its unions on
// the global run table instead (its runs are touched by no other workgroup
// in this pass). A workgroup takes tiles blockIdx.x, + gridDim.x, ... and
// loads the next tile's occupancy words while it works on the current one.
template <int TS>
__global__ __launch_bounds__(kBlock) void k_label_local(const uint64_t *__restrict__ occ, RunTable T, int nx, int ny,
                                                        int nz, int words, RowTiles rt, int ntile, int64_t nrun) {
  static_assert(TS % kBlock == 0, "whole segments per thread");
  constexpr int PER = TS / kBlock;  // segments per thread
  constexpr int CAP = 2 * TS;       // runs per tile held in LDS (2 per segment on average)
  __shared__ uint64_t om[TS];
  __shared__ int32_t first[TS];     // local number of each segment's first run
  __shared__ int32_t par[CAP];      // parents, then the roots' global ids
  __shared__ int32_t wsum[kBlock / 64];
  const int64_t nseg = (int64_t)ny * nz * words;
  occ += blockIdx.y * nseg;
  T.P += blockIdx.y * nrun;
  const int sh = T.shift;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  struct Tile {
    int y0, z0, tye, tze, nls, rw;
  };
  auto tile_of = [&](int tl) -> Tile {
    Tile t;
    t.y0 = (tl % rt.nty) * rt.ty;
    t.z0 = (tl / rt.nty) * rt.tz;
    t.tye = min(rt.ty, ny - t.y0);
    t.tze = min(rt.tz, nz - t.z0);
    t.rw = t.tye * words;  // local segments per z-plane of the tile
    t.nls = t.tze * t.rw;
    return t;
  };
  // (lz, ly, x segment) of a local segment: the thread's first one by
  // division, the next ones by counting on
  struct Loc {
    int lz, ly, sx;
  };
  auto locate = [&](const Tile &t, int ls) -> Loc {
    const int lz = ls / t.rw, rem = ls - lz * t.rw;
    const int ly = rem / words;
    return Loc{lz, ly, rem - ly * words};
  };
  auto next = [&](const Tile &t, Loc l) -> Loc {
    if (++l.sx == words) {
      l.sx = 0;
      if (++l.ly == t.tye) {
        l.ly = 0;
        ++l.lz;
      }
    }
    return l;
  };
  auto gseg = [&](const Tile &t, const Loc &l) -> int64_t {
    return ((int64_t)(t.z0 + l.lz) * ny + (t.y0 + l.ly)) * words + l.sx;
  };
  auto load = [&](int tl, uint64_t *w) {
    const Tile t = tile_of(tl);
    Loc l = locate(t, (int)threadIdx.x * PER);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int ls = (int)threadIdx.x * PER + k;
      w[k] = (ls < t.nls) ? occ[gseg(t, l)] : 0ull;
      l = next(t, l);
    }
  };
  // the pairs of runs of the tile to unite: -x neighbour of the first cell,
  // overlaps with the +y and +z rows inside the tile (through the periodic
  // boundary when the tile spans the whole axis); f(ls, r, ls2, r2)
  auto tile_pairs = [&](const Tile &t, int ls, const Loc &lc, uint64_t m, auto &&f) {
    const int lz = lc.lz, ly = lc.ly, sgx = lc.sx;
    if (m & 1ull) {
      const int lsl = (sgx > 0) ? ls - 1 : ls + words - 1;
      const int lbit = (sgx > 0) ? 63 : (nx - 1) - 64 * (words - 1);
      if (!(lsl == ls && lbit == 0)) {
        const uint64_t ml = om[lsl];
        if ((ml >> lbit) & 1ull) f(ls, 0, lsl, run_index(ml, lbit));
      }
    }
    for (int dir = 0; dir < 2; ++dir) {
      int lsn;
      if (dir == 0) {
        if (ny == 1) continue;
        if (ly + 1 < t.tye) lsn = ls + words;
        else if (t.tye == ny) lsn = ls - (ny - 1) * words;
        else continue;
      } else {
        if (nz == 1) continue;
        if (lz + 1 < t.tze) lsn = ls + t.rw;
        else if (t.tze == nz) lsn = ls - (nz - 1) * t.rw;
        else continue;
      }
      const uint64_t mn = om[lsn];
      const uint64_t ov = m & mn;
      uint64_t firsts = ov & ~(ov << 1);
      while (firsts) {
        const int i = __ffsll((unsigned long long)firsts) - 1;
        firsts &= firsts - 1;
        f(ls, run_index(m, i), lsn, run_index(mn, i));
      }
    }
  };
  uint64_t nxt[PER];
  if ((int)blockIdx.x < ntile) load(blockIdx.x, nxt);
  for (int tl = blockIdx.x; tl < ntile; tl += gridDim.x) {  // workgroup-uniform
    const Tile t = tile_of(tl);
    Loc loc[PER];
    loc[0] = locate(t, (int)threadIdx.x * PER);
#pragma unroll
    for (int k = 1; k < PER; ++k) loc[k] = next(t, loc[k - 1]);
    uint64_t cur[PER];
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      cur[k] = nxt[k];
      om[threadIdx.x * PER + k] = cur[k];
      cnt += __popcll(cur[k] & ~(cur[k] << 1));
    }
    if (tl + (int)gridDim.x < ntile) load(tl + gridDim.x, nxt);
    // exclusive prefix sum of the run counts over the threads
    int inc = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(inc, o, 64);
      if (lane >= o) inc += v;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int off = inc - cnt, total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      const int v = wsum[w];
      off += (w < wv) ? v : 0;
      total += v;
    }
    if (total <= CAP) {  // workgroup-uniform
      {
        int o = off;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int ls = (int)threadIdx.x * PER + k;
          first[ls] = o;
          const int nr = __popcll(cur[k] & ~(cur[k] << 1));
          for (int r = 0; r < nr; ++r) par[o + r] = o + r;
          o += nr;
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int ls = (int)threadIdx.x * PER + k;
        if (ls >= t.nls || cur[k] == 0) continue;
        tile_pairs(t, ls, loc[k], cur[k], [&](int l1, int r1, int l2, int r2) {
          unite_lds(par, first[l1] + r1, first[l2] + r2);
        });
      }
      __syncthreads();
      // the roots (self parents once the unions are done) take ~(global
      // id) as parent, negative where local numbers are not (each thread
      // tests and rewrites only its own runs)
      uint32_t isroot[PER];
      {
        int o = off;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int nr = __popcll(cur[k] & ~(cur[k] << 1));
          isroot[k] = 0;
          for (int r = 0; r < nr; ++r) isroot[k] |= (par[o + r] == o + r) ? (1u << r) : 0u;
          if (isroot[k]) {
            const int64_t g = gseg(t, loc[k]);
            for (int r = 0; r < nr; ++r)
              if ((isroot[k] >> r) & 1u) par[o + r] = ~(int32_t)((g << sh) + r);
          }
          o += nr;
        }
      }
      __syncthreads();
      // ... and every other run walks up to its root and takes that id (a
      // root's entry already holds its own)
      {
        int o = off;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int nr = __popcll(cur[k] & ~(cur[k] << 1));
          if (nr > 0) {
            const int64_t g = gseg(t, loc[k]);
            for (int r = 0; r < nr; ++r) {
              if ((isroot[k] >> r) & 1u) continue;
              int v = par[o + r];
              while (v >= 0) v = par[v];
              T.P[(int64_t)r * nseg + g] = ~v;
            }
          }
          o += nr;
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int ls = (int)threadIdx.x * PER + k;
        if (ls >= t.nls || cur[k] == 0) continue;
        tile_pairs(t, ls, loc[k], cur[k], [&](int l1, int r1, int l2, int r2) {
          unite(T, (int32_t)((gseg(t, locate(t, l1)) << sh) + r1), (int32_t)((gseg(t, locate(t, l2)) << sh) + r2));
        });
      }
    }
    __syncthreads();  // om, first and par are rewritten for the next tile
  }
}

// Unions of segment sgi (row (y, z), x-segment seg, occupancy m) with its -x
// neighbour and its +y and +z rows, as selected.
__device__ __forceinline__ void segment_unions(const uint64_t *__restrict__ occ, const RunTable &T, int nx, int ny,
                                               int nz, int words, int64_t sgi, int seg, int y, int z, uint64_t m,
                                               bool do_x, bool do_y, bool do_z) {
  const int S = 1 << T.shift;
  const int32_t base = (int32_t)(sgi * S);
  // -x: the first cell (bit 0, run 0) and its left neighbour
  if (do_x && (m & 1ull)) {
    const int64_t lsg = (seg > 0) ? sgi - 1 : sgi + words - 1;
    const int lbit = (seg > 0) ? 63 : (nx - 1) - 64 * (words - 1);
    if (!(lsg == sgi && lbit == 0)) {  // a one-cell row is its own neighbour
      const uint64_t ml = (lsg == sgi) ? m : occ[lsg];
      if ((ml >> lbit) & 1ull) unite(T, base, (int32_t)(lsg * S) + run_index(ml, lbit));
    }
  }
  // +y, +z: the first cell of every overlap of a run with a run of that row
  for (int dir = 0; dir < 2; ++dir) {
    if (!(dir == 0 ? do_y : do_z)) continue;
    const int64_t nrow = (dir == 0) ? (int64_t)z * ny + ((y == ny - 1) ? 0 : y + 1)
                                    : (int64_t)((z == nz - 1) ? 0 : z + 1) * ny + y;
    const int64_t nsg = nrow * words + seg;
    const uint64_t mn = occ[nsg];
    const uint64_t ov = m & mn;
    uint64_t firsts = ov & ~(ov << 1);
    while (firsts) {
      const int i = __ffsll((unsigned long long)firsts) - 1;
      firsts &= firsts - 1;
      unite(T, base + run_index(m, i), (int32_t)(nsg * S) + run_index(mn, i));
    }
  }
}

// Pass 2 without row tiles: every segment's unions with its -x, +y and +z
// neighbours.
__global__ __launch_bounds__(kBlock) void k_label_union(const uint64_t *__restrict__ occ, RunTable T, int nx, int ny,
                                                        int nz, int words, SegDiv dv, int64_t nrun) {
  const int64_t sgi = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t nseg = (int64_t)ny * nz * words;
  occ += blockIdx.y * nseg;
  T.P += blockIdx.y * nrun;
  if (sgi >= nseg) return;
  const uint64_t m = occ[sgi];
  if (m == 0) return;
  const Segment sg = segment_of(sgi, dv);
  segment_unions(occ, T, nx, ny, nz, words, sgi, sg.seg, sg.y, sg.z, m, true, ny > 1, nz > 1);
}

// The rows whose +y or +z neighbour lies in another tile: set A, every row
// of the nzb top planes of the z tiles (their +z unions, and +y where the
// row is also the top of its y tile), then set B, the nyb top rows of the y
// tiles in the other planes (their +y unions). nzb = 0 (nyb = 0) when one
// tile spans the axis or it has one cell.
struct EdgeRows {
  int nzb, nyb;
};
static inline EdgeRows edge_rows(const RowTiles &rt, int ny, int nz) {
  EdgeRows e;
  e.nzb = (nz > 1 && nz > rt.tz) ? (int)ceil_div(nz, rt.tz) : 0;
  e.nyb = (ny > 1 && ny > rt.ty) ? (int)ceil_div(ny, rt.ty) : 0;
  return e;
}

// Pass 2b: the unions across tile boundaries, one thread per segment of the
// rows of EdgeRows.
__global__ __launch_bounds__(kBlock) void k_label_union_edges(const uint64_t *__restrict__ occ, RunTable T, int nx,
                                                              int ny, int nz, int words, RowTiles rt, EdgeRows e,
                                                              int64_t nedge, int64_t nrun) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t nseg = (int64_t)ny * nz * words;
  occ += blockIdx.y * nseg;
  T.P += blockIdx.y * nrun;
  if (i >= nedge) return;
  // (nedge <= segments < 2^31: 32-bit divisions)
  const uint32_t q = (uint32_t)i / (uint32_t)words;
  const int seg = (int)((uint32_t)i - q * (uint32_t)words);
  const uint32_t na = (uint32_t)e.nzb * (uint32_t)ny;
  int y, z;
  bool do_y, do_z;
  if (q < na) {
    const int k = (int)(q / (uint32_t)ny);
    y = (int)(q - (uint32_t)k * (uint32_t)ny);
    z = min(k * rt.tz + rt.tz - 1, nz - 1);
    do_z = true;
    do_y = e.nyb > 0 && (y % rt.ty == rt.ty - 1 || y == ny - 1);
  } else {
    const uint32_t qb = q - na;
    const int kz = (int)(qb / (uint32_t)e.nyb), ky = (int)(qb - (uint32_t)kz * (uint32_t)e.nyb);
    y = min(ky * rt.ty + rt.ty - 1, ny - 1);
    // the kz-th plane that is not the top of its z tile
    z = (e.nzb == 0) ? kz : (kz / (rt.tz - 1)) * rt.tz + kz % (rt.tz - 1);
    do_y = true;
    do_z = false;
  }
  const int64_t sgi = ((int64_t)z * ny + y) * words + seg;
  const uint64_t m = occ[sgi];
  if (m == 0) return;
  segment_unions(occ, T, nx, ny, nz, words, sgi, seg, y, z, m, false, do_y, do_z);
}

// Roots of the runs of segment sgi (thread-local loop).
__device__ __forceinline__ int count_roots(const RunTable &T, uint64_t m, int64_t sgi) {
  const int nr = __popcll(m & ~(m << 1));
  int n = 0;
  for (int r = 0; r < nr; ++r) {
    const int32_t id = (int32_t)((sgi << T.shift) + r);
    n += (*T.at(id) == id) ? 1 : 0;
  }
  return n;
}

// Passes 3-5 take kSegT segments per thread: round k of wavefront w of a
// workgroup covers the 64 consecutive segments 64 (kSegT w + k) .. + 63 of
// the workgroup's kBlock * kSegT, one per lane, so the segments of a
// workgroup are in (wavefront, round, lane) order, their linear order.
constexpr int kSegT = 4;  // (flatten + rank + resolve at 512^3 x 8: 1: 0.196 ms, 2: 0.178, 4: 0.166, 8: 0.186)
__device__ __forceinline__ int64_t pass_segment(int k) {
  return ((int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63)) * kSegT + 64 * k + (threadIdx.x & 63);
}

// Pass 3: every run points at its root; roots counted per workgroup.
__global__ __launch_bounds__(kBlock) void k_label_flatten(const uint64_t *__restrict__ occ, RunTable T, int64_t nseg,
                                                          uint32_t *__restrict__ blockcount, int64_t nrun) {
  occ += blockIdx.y * nseg;
  T.P += blockIdx.y * nrun;
  blockcount += blockIdx.y * gridDim.x;
  uint64_t m[kSegT];
#pragma unroll
  for (int k = 0; k < kSegT; ++k) m[k] = (pass_segment(k) < nseg) ? occ[pass_segment(k)] : 0ull;
  uint32_t nroot = 0;
#pragma unroll
  for (int k = 0; k < kSegT; ++k) {
    const int nr = __popcll(m[k] & ~(m[k] << 1));
    for (int r = 0; r < nr; ++r) {
      const int32_t id = (int32_t)((pass_segment(k) << T.shift) + r);
      const int32_t root = find_root(T, id);
      if (root == id) ++nroot;
      else *T.at(id) = root;
    }
  }
  for (int o = 32; o > 0; o >>= 1) nroot += __shfl_xor(nroot, o, 64);
  __shared__ uint32_t wcount[kBlock / 64];
  if ((threadIdx.x & 63) == 0) wcount[threadIdx.x >> 6] = nroot;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t sum = 0;
    for (int w = 0; w < kBlock / 64; ++w) sum += wcount[w];
    blockcount[blockIdx.x] = sum;
  }
}

// The totals of the tiled scans (one per field, tstride apart) into total[].
__global__ void k_copy_total(const int32_t *__restrict__ tot, int64_t ntiles, int64_t tstride, int nfields,
                             int32_t *__restrict__ total) {
  const int t = threadIdx.x;
  if (t < nfields) total[t] = tot[t * tstride + ntiles];
}

// Pass 4: each root's entry becomes -(1 + number of roots before it), in
// linear order: the workgroup's offset from the scanned block counts, then
// within the workgroup the roots of earlier wavefronts, earlier rounds and
// lower lanes.
__global__ __launch_bounds__(kBlock) void k_label_rank(const uint64_t *__restrict__ occ, RunTable T, int64_t nseg,
                                                       const int32_t *__restrict__ blockoff,
                                                       const int32_t *__restrict__ tileoff, int64_t nrun,
                                                       int64_t tstride) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  occ += blockIdx.y * nseg;
  T.P += blockIdx.y * nrun;
  blockoff += blockIdx.y * gridDim.x;
  tileoff += blockIdx.y * tstride;
  uint64_t m[kSegT];
#pragma unroll
  for (int k = 0; k < kSegT; ++k) m[k] = (pass_segment(k) < nseg) ? occ[pass_segment(k)] : 0ull;
  int excl[kSegT];  // roots of the wavefront before this lane's segment of round k
  int wtotal = 0;   // roots of the wavefront
#pragma unroll
  for (int k = 0; k < kSegT; ++k) {
    const int mine = m[k] ? count_roots(T, m[k], pass_segment(k)) : 0;
    int incl = mine;
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o, 64);
      if (lane >= o) incl += v;
    }
    excl[k] = wtotal + incl - mine;
    wtotal += __shfl(incl, 63, 64);
  }
  __shared__ int wtot[kBlock / 64];
  if (lane == 0) wtot[w] = wtotal;
  __syncthreads();
  int base = blockoff[blockIdx.x] + tileoff[blockIdx.x / compact::kTile];
  for (int k = 0; k < w; ++k) base += wtot[k];
#pragma unroll
  for (int k = 0; k < kSegT; ++k) {
    if (!m[k]) continue;
    int before = base + excl[k];
    const int nr = __popcll(m[k] & ~(m[k] << 1));
    for (int r = 0; r < nr; ++r) {
      const int32_t id = (int32_t)((pass_segment(k) << T.shift) + r);
      if (*T.at(id) == id) *T.at(id) = -(++before);
    }
  }
}

// Pass 5: every run that is not a root takes its root's entry (the negative
// label); roots are only read.
__global__ __launch_bounds__(kBlock) void k_label_resolve(const uint64_t *__restrict__ occ, RunTable T, int64_t nseg,
                                                          int64_t nrun) {
  occ += blockIdx.y * nseg;
  T.P += blockIdx.y * nrun;
  uint64_t m[kSegT];
#pragma unroll
  for (int k = 0; k < kSegT; ++k) m[k] = (pass_segment(k) < nseg) ? occ[pass_segment(k)] : 0ull;
#pragma unroll
  for (int k = 0; k < kSegT; ++k) {
    const int nr = __popcll(m[k] & ~(m[k] << 1));
    for (int r = 0; r < nr; ++r) {
      int32_t *e = T.at((int32_t)((pass_segment(k) << T.shift) + r));
      const int32_t v = *e;
      if (v >= 0) *e = *T.at(v);
    }
  }
}

// Pass 6: label of every cell of the field (0 for empty cells). The
// occupancy words, then the run entries of the wavefront's kSegsW segments
// are each loaded together: every lane loads (from a valid slot when it has
// no cell) and selects afterwards, since a load under a lane condition is
// compiled as a branch that waits for it.
__global__ __launch_bounds__(kBlock) void k_label_write(const uint64_t *__restrict__ occ, RunTable T,
                                                        int32_t *__restrict__ lab, int nx, int ny, int nz, int words,
                                                        SegDiv dv, int64_t nrun) {
  const int lane = threadIdx.x & 63;
  const int64_t nseg = (int64_t)ny * nz * words, s0 = first_segment<kSegsW>();
  occ += blockIdx.y * nseg;
  T.P += blockIdx.y * nrun;
  lab += blockIdx.y * ((int64_t)nx * ny * nz);
  uint64_t m[kSegsW];
  int32_t e[kSegsW];
#pragma unroll
  for (int k = 0; k < kSegsW; ++k) m[k] = (s0 + k < nseg) ? occ[s0 + k] : 0ull;
  bool on[kSegsW];
#pragma unroll
  for (int k = 0; k < kSegsW; ++k) {
    on[k] = (m[k] >> lane) & 1ull;
    const int64_t sg = (s0 + k < nseg) ? s0 + k : nseg - 1;
    e[k] = T.P[(int64_t)(on[k] ? run_index(m[k], lane) : 0) * nseg + sg];
  }
#pragma unroll
  for (int k = 0; k < kSegsW; ++k) e[k] = on[k] ? -e[k] : 0;
#pragma unroll
  for (int k = 0; k < kSegsW; ++k) {
    const int64_t sgi = s0 + k;
    if (sgi >= nseg) break;  // wave-uniform
    const Segment sg = segment_of(sgi, dv);
    const int x = sg.seg * 64 + lane;
    if (x < nx) __builtin_nontemporal_store(e[k], &lab[sg.row * nx + x]);  // streamed out
  }
}

// Pass 6 when rows hold a multiple of 256 cells: lane l of a wavefront
// writes cells 4l .. 4l+3 of each of its kGroupsW 256-cell groups (segment
// 4g + l/16, bits 4(l%16) .. +3) with one 16-byte store. The occupancy
// words and then the run entries of all the wavefront's groups are loaded
// before the first store, as in k_label_write.
constexpr int kGroupsW = 4;
typedef int32_t v4i32 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kBlock) void k_label_write4(const uint64_t *__restrict__ occ, RunTable T,
                                                         int32_t *__restrict__ lab, int64_t n3, int64_t nrun) {
  const int lane = threadIdx.x & 63;
  const int64_t nseg = T.nseg, ngroups = nseg / 4;
  const int64_t g0 = (((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6) * kGroupsW;
  occ += blockIdx.y * nseg;
  T.P += blockIdx.y * nrun;
  v4i32 *lab4 = reinterpret_cast<v4i32 *>(lab + blockIdx.y * n3);
  const int j = lane >> 4, b0 = 4 * (lane & 15);
  uint64_t m[kGroupsW];
  int64_t sg[kGroupsW];
#pragma unroll
  for (int k = 0; k < kGroupsW; ++k) {
    sg[k] = (g0 + k < ngroups) ? 4 * (g0 + k) + j : nseg - 1;
    m[k] = occ[sg[k]];
  }
  int32_t e[kGroupsW][4];
#pragma unroll
  for (int k = 0; k < kGroupsW; ++k)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool on = (m[k] >> (b0 + i)) & 1ull;
      const int32_t v = T.P[(int64_t)(on ? run_index(m[k], b0 + i) : 0) * nseg + sg[k]];
      e[k][i] = on ? -v : 0;
    }
#pragma unroll
  for (int k = 0; k < kGroupsW; ++k) {
    if (g0 + k >= ngroups) break;  // wave-uniform
    const v4i32 v = {e[k][0], e[k][1], e[k][2], e[k][3]};
    __builtin_nontemporal_store(v, &lab4[(g0 + k) * 64 + lane]);  // streamed out
  }
}

// Workgroups of the per-cell labelling passes (kSegs row segments per
// wavefront) and of the per-segment passes (one thread per segment).
static inline int64_t label_blocks(int nx, int ny, int nz, int segs_per_wave) {
  const int64_t words = (nx + 63) / 64;
  const int64_t per = (int64_t)(kBlock / 64) * segs_per_wave;
  return ((int64_t)ny * nz * words + per - 1) / per;
}
static inline int64_t segment_blocks(int nx, int ny, int nz) {
  const int64_t words = (nx + 63) / 64;
  return ((int64_t)ny * nz * words + kBlock - 1) / kBlock;
}
// Run slots per segment, log2: a segment of w cells holds at most
// (w + 1) / 2 runs; the slots are the next power of two.
static inline int run_shift(int nx) {
  const int most = ((nx < 64 ? nx : 64) + 1) / 2;
  int sh = 0;
  while ((1 << sh) < most) ++sh;
  return sh;
}

// ------------------------------------------------------------------ moments
//
// Bounding box of a drop as offsets from its first cell p0 (the reference of
// the centroid), wrapped into [-n/2, n/2) per axis. The cells of a connected
// drop project onto each periodic axis as one contiguous arc. Two frames of
// the axis are tracked: A, the coordinate a itself, and B, (a + n/2) mod n,
// whose cuts (between n-1 and 0, and between n-n/2-1 and n-n/2) lie n/2
// apart. An arc of L cells with 2 (L-1) < n contains at most one cut, so the
// frame with the smaller span holds it uncut, with span L - 1, and its
// min/max minus p0's coordinate in that frame are the wrapped offsets of the
// arc's ends. When 2 (L-1) >= n both frames span at least n/2, which is the
// extent error in either case. So one pass over the labels collects, per
// drop, the first cell and the min/max of both frames on each axis, and a
// per-drop step turns them into the box.

// Wavefront-wide minimum / maximum (every lane passes a value; lanes outside
// the set pass the neutral value).
__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Per-drop reductions go through a small hash table in LDS per workgroup: a
// workgroup sweeps kChunk consecutive cells, the lanes of a wavefront holding
// the same drop are combined first, each such group updates the drop's LDS
// record with LDS atomics, and at the end the workgroup applies one set of
// global atomics per drop it met. Global atomics on one address from many
// workgroups are serialised; this makes them about kChunk / (cells of a
// drop's row run) times fewer. A drop that finds the table full goes to the
// global atomics directly. Integer min/max are order-independent, so the
// result does not depend on scheduling.
// 32768 cells (64 rows of 512) and 16 loads in flight per thread measured
// best on 512^3 fields: fewer workgroups flush fewer records (8192 cells
// and 8 loads: moments 3.40 against 2.93 ms for 8 tracers).
constexpr int kChunk = 32768;  // cells per workgroup (128 per thread)
constexpr int kTable = 64;     // LDS records per workgroup (power of two)
constexpr int kBatch = 16;     // positions per thread whose loads are issued together
constexpr int kFrames = 12;    // per drop: axis a -> min A, max A, min B, max B at 4a
static_assert(kTable == 64 && kChunk % kBlock == 0, "table_slot hashes to 6 bits");
static_assert((kChunk / kBlock) % kBatch == 0, "whole batches per thread");

__device__ __forceinline__ int table_slot(int32_t *key, int32_t l) {
  const uint32_t h = ((uint32_t)l * 2654435761u) >> 26;  // 6 bits: kTable = 64
  for (int k = 0; k < kTable; ++k) {
    const int s = (int)((h + k) & (kTable - 1));
    const int32_t prev = atomicCAS(&key[s], 0, l);
    if (prev == 0 || prev == l) return s;
  }
  return -1;
}

__global__ void k_scan_init(int32_t *first, int32_t *frames, int64_t K) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) first[i] = INT32_MAX;
  if (i < kFrames * K) frames[i] = (i & 1) ? INT32_MIN : INT32_MAX;
}

// One drop's record (first cell, frame extents) merged into the workgroup's
// LDS table, or into the global arrays when the table is full.
__device__ __forceinline__ void merge_record(int32_t *key, int32_t *rfirst, int32_t (*rec)[kFrames],
                                             int32_t *first, int32_t *frames, int32_t l, int32_t f,
                                             const int32_t *e) {
  const int s = table_slot(key, l);
  int32_t *pf = (s >= 0) ? &rfirst[s] : &first[l - 1];
  int32_t *g = (s >= 0) ? &rec[s][0] : &frames[kFrames * (int64_t)(l - 1)];
  atomicMin(pf, f);
  for (int k = 0; k < kFrames; k += 2) {
    atomicMin(&g[k], e[k]);
    atomicMax(&g[k + 1], e[k + 1]);
  }
}

// First cell and the frame extents of every drop.
__global__ __launch_bounds__(kBlock) void k_drop_scan(const int32_t *__restrict__ lab, int64_t n3, int nx, int ny,
                                                      int nz, FastDiv fnx, FastDiv fny,
                                                      const int32_t *__restrict__ toff,
                                                      int32_t *__restrict__ first, int32_t *__restrict__ frames) {
  // field blockIdx.y: its drops are records toff[t] .. toff[t+1]-1
  const int t = blockIdx.y;
  const int32_t o = toff[t], K = toff[t + 1] - o;
  if (K == 0) return;  // (uniform over the workgroup)
  lab += (int64_t)t * n3;
  first += o;
  frames += (int64_t)kFrames * o;
  __shared__ int32_t key[kTable];
  __shared__ int32_t rfirst[kTable];
  __shared__ int32_t rec[kTable][kFrames];
  for (int i = threadIdx.x; i < kTable; i += kBlock) {
    key[i] = 0;
    rfirst[i] = INT32_MAX;
    for (int k = 0; k < kFrames; ++k) rec[i][k] = (k & 1) ? INT32_MIN : INT32_MAX;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int n[3] = {nx, ny, nz};
  const int h[3] = {nx / 2, ny / 2, nz / 2};
  const int64_t c0 = (int64_t)blockIdx.x * kChunk;
  for (int it0 = 0; it0 < kChunk / kBlock; it0 += kBatch) {
    int32_t lb[kBatch];  // the labels of kBatch positions are loaded together
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int64_t p = c0 + (int64_t)(it0 + u) * kBlock + threadIdx.x;
      lb[u] = (p < n3) ? lab[p] : 0;
    }
#pragma unroll 1
    for (int u = 0; u < kBatch; ++u) {
      const int64_t pw = c0 + (int64_t)(it0 + u) * kBlock + (threadIdx.x & ~63);  // the wavefront's first cell
      const int64_t p = pw + lane;
      const int32_t l = lb[u];
      const bool valid = l > 0 && l <= K;
      uint64_t todo = __ballot(valid);
      if (!todo) continue;  // wave-uniform
      // row of the wavefront's first and last cells (wave-uniform, scalar)
      const uint32_t pw32 = __builtin_amdgcn_readfirstlane((uint32_t)pw);
      const uint32_t rw = fast_div(pw32, fnx);
      const uint32_t rl = fast_div((uint32_t)(pw32 + 63 < n3 ? pw32 + 63 : n3 - 1), fnx);
      const bool one_row = (rw == rl);  // cell x = x of the first cell + lane
      const int xw = (int)(pw32 - rw * (uint32_t)nx);
      // coordinates of this lane's cell (needed only when the cells span two rows)
      int c[3] = {0, 0, 0};
      if (!one_row) {
        const uint32_t pc = valid ? (uint32_t)p : pw32;
        const uint32_t r = fast_div(pc, fnx), zz = fast_div(r, fny);
        c[0] = (int)(pc - r * (uint32_t)nx);
        c[1] = (int)(r - zz * (uint32_t)ny);
        c[2] = (int)zz;
      }
      while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int32_t lv = __shfl(l, leader, 64);
        const uint64_t same = __ballot(valid && l == lv);
        int e[kFrames];
        if (one_row) {
          // x: the group's lanes in increasing x; frame B cuts at x = nx - nx/2
          const int lo = leader, hi = 63 - __clzll(same);
          e[0] = xw + lo;
          e[1] = xw + hi;
          const int cut = nx - h[0] - xw;  // first lane with x >= nx - nx/2 (may be outside 0..63)
          const uint64_t above = (cut <= 0) ? ~0ull : ((cut >= 64) ? 0ull : (~0ull << cut));
          const uint64_t mhi = same & above, mlo = same & ~above;
          e[2] = mhi ? xw + (__ffsll((unsigned long long)mhi) - 1) - (nx - h[0]) : xw + lo + h[0];
          e[3] = mlo ? xw + (63 - __clzll(mlo)) + h[0] : xw + hi - (nx - h[0]);
          // y and z are those of the row
          const int zr = (int)fast_div(rw, fny), yr = (int)(rw - (uint32_t)zr * (uint32_t)ny);
          e[4] = e[5] = yr;
          e[6] = e[7] = (yr + h[1] >= ny) ? yr + h[1] - ny : yr + h[1];
          e[8] = e[9] = zr;
          e[10] = e[11] = (zr + h[2] >= nz) ? zr + h[2] - nz : zr + h[2];
        } else {
          const bool mine = valid && l == lv;
          for (int a = 0; a < 3; ++a) {
            const int vb = (c[a] + h[a] >= n[a]) ? c[a] + h[a] - n[a] : c[a] + h[a];
            e[4 * a] = wave_min(mine ? c[a] : INT32_MAX);
            e[4 * a + 1] = wave_max(mine ? c[a] : INT32_MIN);
            e[4 * a + 2] = wave_min(mine ? vb : INT32_MAX);
            e[4 * a + 3] = wave_max(mine ? vb : INT32_MIN);
          }
        }
        if (lane == leader)  // the lowest lane holds the group's first cell
          merge_record(key, rfirst, rec, first, frames, lv, (int32_t)p, e);
        todo &= ~same;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kTable; i += kBlock) {
    const int32_t lv = key[i];
    if (lv == 0) continue;
    atomicMin(&first[lv - 1], rfirst[i]);
    int32_t *g = &frames[kFrames * (int64_t)(lv - 1)];
    for (int k = 0; k < kFrames; k += 2) {
      atomicMin(&g[k], rec[i][k]);
      atomicMax(&g[k + 1], rec[i][k + 1]);
    }
  }
}

// Box of every drop from its frames: per axis, the frame with the smaller
// span, minus p0's coordinate in that frame. A label without cells keeps an
// empty box (min > max).
__global__ void k_drop_box(int32_t K, int nx, int ny, int nz, const int32_t *__restrict__ first,
                           const int32_t *__restrict__ frames, int32_t *__restrict__ box) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const int32_t p0 = first[i];
  int32_t *b = box + 6 * i;
  if (p0 == INT32_MAX) {
    for (int a = 0; a < 3; ++a) {
      b[2 * a] = INT32_MAX;
      b[2 * a + 1] = INT32_MIN;
    }
    return;
  }
  const int n[3] = {nx, ny, nz};
  const int r[3] = {p0 % nx, (p0 / nx) % ny, p0 / (nx * ny)};
  const int32_t *f = frames + kFrames * i;
  for (int a = 0; a < 3; ++a) {
    const int h = n[a] / 2;
    const int spanA = f[4 * a + 1] - f[4 * a], spanB = f[4 * a + 3] - f[4 * a + 2];
    const int rb = (r[a] + h >= n[a]) ? r[a] + h - n[a] : r[a] + h;
    const bool useA = spanA <= spanB;
    b[2 * a] = useA ? f[4 * a] - r[a] : f[4 * a + 2] - rb;
    b[2 * a + 1] = useA ? f[4 * a + 1] - r[a] : f[4 * a + 3] - rb;
  }
}

// kSumSplit workgroups per drop sum c and c*offset over consecutive parts of
// the drop's bounding box (per-thread strided partial sums, then a fixed
// tree); k_drop_finish adds the parts of each drop in order. The result is
// reproducible bit for bit.
constexpr int kSumSplit = 8;
constexpr int kSumBatch = 4;  // box cells per thread whose loads are issued together
// Box coordinates (ix, iy, iz) of a thread's cells q, q + kBlock, ...: the
// first by division, the next by adding kBlock's digits with carries (each
// digit is below its extent).
struct BoxWalk {
  int ix, iy, iz, stx, sty, stz, ex, ey;
  __device__ BoxWalk(int q, int ex_, int ey_) : ex(ex_), ey(ey_) {
    const int exy = ex_ * ey_;
    ix = q % ex_;
    iy = (q / ex_) % ey_;
    iz = q / exy;
    stx = kBlock % ex_;
    sty = (kBlock / ex_) % ey_;
    stz = kBlock / exy;
  }
  __device__ void step() {
    ix += stx;
    iy += sty;
    iz += stz;
    if (ix >= ex) {
      ix -= ex;
      ++iy;
    }
    if (iy >= ey) {
      iy -= ey;
      ++iz;
    }
  }
};
// Field of record g (toff: ntr + 1 increasing offsets) and its label.
__device__ __forceinline__ int field_of(const int32_t *__restrict__ toff, int32_t g) {
  int t = 0;
  while (toff[t + 1] <= g) ++t;
  return t;
}
__global__ __launch_bounds__(kBlock) void k_drop_sums(const double *__restrict__ c, const int32_t *__restrict__ lab,
                                                      int nx, int ny, int nz, const int32_t *__restrict__ toff,
                                                      const int32_t *__restrict__ rootpos,
                                                      const int32_t *__restrict__ box, double *__restrict__ part,
                                                      int32_t *__restrict__ extent_err) {
  const int32_t g = blockIdx.x / kSumSplit;  // record (drop of every field)
  const int sl = blockIdx.x % kSumSplit;
  const int t = field_of(toff, g);
  const int l = g - toff[t] + 1;  // its label in field t
  const int64_t n3 = (int64_t)nx * ny * nz;
  c += (int64_t)t * n3;
  lab += (int64_t)t * n3;
  const int32_t p0 = rootpos[g];
  const int32_t *b = box + 6 * (int64_t)g;
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
  const int qs = q0 + (int)threadIdx.x;
  BoxWalk bw(qs, ex, ey);
  for (int q = qs; q < q1; q += kSumBatch * kBlock) {
    // kSumBatch cells: label and value loaded together (a cell past the
    // range loads the first cell, p0, and is ignored), then summed in order
    int d[kSumBatch][3];
    int64_t pb[kSumBatch];
    bool in[kSumBatch];
#pragma unroll
    for (int u = 0; u < kSumBatch; ++u) {
      in[u] = q + u * kBlock < q1;
      d[u][0] = bw.ix + lx;
      d[u][1] = bw.iy + ly;
      d[u][2] = bw.iz + lz;
      bw.step();
      // offsets lie in [-n/2, n/2): one period at most
      int x = x0 + d[u][0], y = y0 + d[u][1], z = z0 + d[u][2];
      x += (x < 0) ? nx : ((x >= nx) ? -nx : 0);
      y += (y < 0) ? ny : ((y >= ny) ? -ny : 0);
      z += (z < 0) ? nz : ((z >= nz) ? -nz : 0);
      pb[u] = in[u] ? ((int64_t)z * ny + y) * nx + x : (int64_t)p0;
    }
    int32_t lv[kSumBatch];
    double cv[kSumBatch];
#pragma unroll
    for (int u = 0; u < kSumBatch; ++u) {
      lv[u] = lab[pb[u]];
      cv[u] = c[pb[u]];
    }
#pragma unroll
    for (int u = 0; u < kSumBatch; ++u) {
      if (!in[u] || lv[u] != l) continue;
      const double v = cv[u];
      s0 += v;
      s1 += v * (double)d[u][0];
      s2 += v * (double)d[u][1];
      s3 += v * (double)d[u][2];
    }
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
  if (threadIdx.x < 4) part[((int64_t)g * kSumSplit + sl) * 4 + threadIdx.x] = red[threadIdx.x][0];
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

// Shape sums of one drop part: with the offsets r of a cell from the centre
// of the drop's box (integer part), c, c r (3), c r r^T (6: xx, yy, zz, xy,
// xz, yz) and, given face Courant numbers, c u (3) with u the mean of the
// cell's two faces on each axis. Same partition and fixed tree as
// k_drop_sums, so the result is reproducible bit for bit.
constexpr int kShapeSums = 13;
__global__ __launch_bounds__(kBlock) void k_shape_sums(const double *__restrict__ c, const int32_t *__restrict__ lab,
                                                       const double *__restrict__ sx, const double *__restrict__ sy,
                                                       const double *__restrict__ sz, int nx, int ny, int nz,
                                                       const int32_t *__restrict__ toff,
                                                       const int32_t *__restrict__ rootpos,
                                                       const int32_t *__restrict__ box, double *__restrict__ part,
                                                       int32_t *__restrict__ extent_err) {
  const int32_t g = blockIdx.x / kSumSplit;  // record (drop of every field)
  const int sl = blockIdx.x % kSumSplit;
  const int t = field_of(toff, g);
  const int l = g - toff[t] + 1;  // its label in field t
  const int64_t n3 = (int64_t)nx * ny * nz;
  c += (int64_t)t * n3;
  lab += (int64_t)t * n3;
  const int32_t p0 = rootpos[g];
  const int32_t *b = box + 6 * (int64_t)g;
  if (p0 == INT32_MAX || b[0] > b[1]) {  // label without cells: inconsistent input
    if (threadIdx.x == 0) atomicOr(extent_err, 2);
    return;
  }
  const int x0 = p0 % nx, y0 = (p0 / nx) % ny, z0 = p0 / (nx * ny);
  const int lx = b[0], ly = b[2], lz = b[4];
  const int ex = b[1] - b[0] + 1, ey = b[3] - b[2] + 1, ez = b[5] - b[4] + 1;
  // the box centre's offset (floor of the mean of its ends)
  const int mx = (b[0] + b[1]) >> 1, my = (b[2] + b[3]) >> 1, mz = (b[4] + b[5]) >> 1;
  const int nbox = ex * ey * ez;
  const int q0 = (int)((int64_t)nbox * sl / kSumSplit), q1 = (int)((int64_t)nbox * (sl + 1) / kSumSplit);
  const bool withu = sx != nullptr;
  double acc[kShapeSums];
#pragma unroll
  for (int k = 0; k < kShapeSums; ++k) acc[k] = 0.0;
  const int qs = q0 + (int)threadIdx.x;
  BoxWalk bw(qs, ex, ey);
  for (int q = qs; q < q1; q += kBlock) {
    // one cell at a time: batching the shape sums' loads (13 accumulators)
    // measured slower
    const int dx = bw.ix + lx, dy = bw.iy + ly, dz = bw.iz + lz;
    bw.step();
    int x = x0 + dx, y = y0 + dy, z = z0 + dz;
    x += (x < 0) ? nx : ((x >= nx) ? -nx : 0);
    y += (y < 0) ? ny : ((y >= ny) ? -ny : 0);
    z += (z < 0) ? nz : ((z >= nz) ? -nz : 0);
    const int64_t p = ((int64_t)z * ny + y) * nx + x;
    if (lab[p] != l) continue;
    const double v = c[p];
    const double rx = (double)(dx - mx), ry = (double)(dy - my), rz = (double)(dz - mz);
    const double vx = v * rx, vy = v * ry, vz = v * rz;
    acc[0] += v;
    acc[1] += vx;
    acc[2] += vy;
    acc[3] += vz;
    acc[4] += vx * rx;
    acc[5] += vy * ry;
    acc[6] += vz * rz;
    acc[7] += vx * ry;
    acc[8] += vx * rz;
    acc[9] += vy * rz;
    if (withu) {
      const int xp = (x + 1 == nx) ? 0 : x + 1, yp = (y + 1 == ny) ? 0 : y + 1, zp = (z + 1 == nz) ? 0 : z + 1;
      const int64_t row = (int64_t)y * nx + (int64_t)z * ny * nx;
      acc[10] += v * (0.5 * (sx[p] + sx[row + xp]));
      acc[11] += v * (0.5 * (sy[p] + sy[(int64_t)z * ny * nx + (int64_t)yp * nx + x]));
      acc[12] += v * (0.5 * (sz[p] + sz[((int64_t)zp * ny + y) * nx + x]));
    }
  }
  __shared__ double red[kShapeSums][kBlock];
#pragma unroll
  for (int k = 0; k < kShapeSums; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < kShapeSums; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < kShapeSums)
    part[((int64_t)g * kSumSplit + sl) * kShapeSums + threadIdx.x] = red[threadIdx.x][0];
}

// Inertia tensor about the centroid, aspect ratio and mean velocity of every
// drop from its kSumSplit parts. The second moments about the centroid are
// the box-centred ones minus the centroid's share (parallel axes), plus V/12
// per axis for the cells' own extent; I = tr(J) delta - J. Eigenvalues of the
// symmetric 3x3 tensor by cyclic Jacobi rotations (Golub & Van Loan, the
// symmetric Schur decomposition), which keep every eigenvalue within a few
// ulps of the tensor's norm also for the (near-)equal pairs of round or
// axisymmetric drops, where closed forms through the characteristic
// polynomial lose half the digits.
// vol, xyz (nullable): the volume and centroid as well, the centroid as the
// first cell's centre plus the box centre's offset plus the mean offset from
// it (the moments' quantities from the shape sums).
__global__ void k_shape_finish(int32_t K, int nx, int ny, int nz, const int32_t *__restrict__ rootpos,
                               const int32_t *__restrict__ box, const double *__restrict__ part,
                               double *__restrict__ inertia, double *__restrict__ chi, double *__restrict__ vel,
                               double *__restrict__ vol, double *__restrict__ xyz, int32_t *__restrict__ extent_err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const int32_t p0 = rootpos[i];
  const int32_t *b = box + 6 * i;
  if (p0 == INT32_MAX || b[0] > b[1]) return;  // reported by k_shape_sums
  double S[kShapeSums];
  for (int k = 0; k < kShapeSums; ++k) S[k] = 0.0;
  for (int sl = 0; sl < kSumSplit; ++sl)
    for (int k = 0; k < kShapeSums; ++k) S[k] += part[(i * kSumSplit + sl) * kShapeSums + k];
  const double V = S[0];
  const double gx = S[1] / V, gy = S[2] / V, gz = S[3] / V;
  const double self = V / 12.0;
  const double Jxx = (S[4] - S[1] * gx) + self, Jyy = (S[5] - S[2] * gy) + self, Jzz = (S[6] - S[3] * gz) + self;
  const double Jxy = S[7] - S[1] * gy, Jxz = S[8] - S[1] * gz, Jyz = S[9] - S[2] * gz;
  const double Ixx = Jyy + Jzz, Iyy = Jxx + Jzz, Izz = Jxx + Jyy;
  const double Ixy = -Jxy, Ixz = -Jxz, Iyz = -Jyz;
  double *o = inertia + 6 * i;
  o[0] = Ixx;
  o[1] = Iyy;
  o[2] = Izz;
  o[3] = Ixy;
  o[4] = Ixz;
  o[5] = Iyz;
  double A[3][3] = {{Ixx, Ixy, Ixz}, {Ixy, Iyy, Iyz}, {Ixz, Iyz, Izz}};
  for (int sweep = 0; sweep < 16; ++sweep) {
    if (A[0][1] == 0.0 && A[0][2] == 0.0 && A[1][2] == 0.0) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int pp = pq == 2 ? 1 : 0, qq = pq == 0 ? 1 : 2, rr = 3 - pp - qq;
      const double apq = A[pp][qq];
      if (apq == 0.0) continue;
      const double g = 100.0 * fabs(apq);
      if (fabs(A[pp][pp]) + g == fabs(A[pp][pp]) && fabs(A[qq][qq]) + g == fabs(A[qq][qq])) {
        A[pp][qq] = A[qq][pp] = 0.0;  // negligible against both diagonal entries
        continue;
      }
      // rotation angle zeroing A[pp][qq]: t = tan, the smaller root
      const double tau = (A[qq][qq] - A[pp][pp]) / (2.0 * apq);
      const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
      const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
      A[pp][pp] -= t * apq;
      A[qq][qq] += t * apq;
      A[pp][qq] = A[qq][pp] = 0.0;
      const double arp = A[rr][pp], arq = A[rr][qq];
      A[rr][pp] = A[pp][rr] = cs * arp - sn * arq;
      A[rr][qq] = A[qq][rr] = sn * arp + cs * arq;
    }
  }
  const double lmax = fmax(A[0][0], fmax(A[1][1], A[2][2]));
  const double lmin = fmin(A[0][0], fmin(A[1][1], A[2][2]));
  chi[i] = sqrt(lmax / lmin);
  if (vel) {
    vel[3 * i] = S[10] / V;
    vel[3 * i + 1] = S[11] / V;
    vel[3 * i + 2] = S[12] / V;
  }
  const int n[3] = {nx, ny, nz};
  if (vol) {
    vol[i] = V;
    const int r[3] = {p0 % nx, (p0 / nx) % ny, p0 / (nx * ny)};
    const double g[3] = {gx, gy, gz};
    for (int a = 0; a < 3; ++a) {
      double x = (((double)r[a] + 0.5) + (double)((b[2 * a] + b[2 * a + 1]) >> 1)) + g[a];
      if (x >= (double)n[a]) x -= (double)n[a];
      if (x < 0.0) x += (double)n[a];
      xyz[3 * i + a] = x;
    }
  }
  for (int e = 0; e < 3; ++e)
    if (2 * (b[2 * e + 1] - b[2 * e]) >= n[e]) atomicOr(extent_err, 1);
}

}  // namespace

// Segments per tile of the local union pass (measured on 512^3 x 8:
// 256: 0.44 ms for passes 2a + 2b, 1024: 0.28, 2048: 0.27, 4096: 0.59 with
// one workgroup per CU).
constexpr int kTileSegs = 2048;
// Row tiles of the local union pass: as many whole rows as fit ts segments,
// tz the largest power of two up to their square root (at most nz), the rest
// along y. Rows longer than ts segments take the global unions only (ty = 0).
static inline RowTiles row_tiles(int ny, int nz, int words, int ts) {
  RowTiles rt{0, 0, 0};
  if (words > ts) return rt;
  const int rows = ts / words;
  int tz = 1;
  while ((2 * tz) * (2 * tz) <= rows) tz *= 2;
  rt.tz = tz < nz ? tz : nz;
  rt.ty = rows / rt.tz;
  if (rt.ty > ny) rt.ty = ny;
  rt.nty = (int)ceil_div(ny, rt.ty);
  return rt;
}
// The local union pass: as many workgroups per field as fill the chip once
// over all fields (each then loops over its tiles), at most one per tile.
template <int TS>
static void launch_local(vofmt_ctx *ctx, int ntile, unsigned nt, hipStream_t stream, const uint64_t *occ,
                         const RunTable &R, int nx, int ny, int nz, int words, const RowTiles &rt, int64_t nrun) {
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_label_local<TS>, kBlock, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int64_t gx = ((int64_t)cus * per_cu + nt - 1) / nt;
  if (gx > ntile) gx = ntile;
  hipLaunchKernelGGL(k_label_local<TS>, dim3((unsigned)gx, nt), dim3(kBlock), 0, stream, occ, R, nx, ny, nz, words, rt,
                     ntile, nrun);
}
// Label one tracer field into `lab`. Returns K via *k_dev (device int32).
// Scratch: occupancy words (one per segment), run array (S per segment),
// block counts (segment_blocks entries), tile offsets
// (segment_blocks / compact::kTile + 2 entries).
// All passes over the T fields at once (blockIdx.y = field), each field with
// its own work arrays.
static int label_all(vofmt_ctx *ctx, int nx, int ny, int nz, int T, const double *c, double c_eps, int32_t *lab,
                     uint64_t *occ, int32_t *runs, uint32_t *blockcount, int32_t *tileoff, int64_t tstride,
                     int32_t *k_dev, hipStream_t stream) {
  const int words = (int)ceil_div(nx, 64);
  const int64_t nseg = (int64_t)ny * nz * words;
  const RunTable R{runs, nseg, run_shift(nx)};
  const int64_t nrun = nseg << R.shift;
  const unsigned nbc = (unsigned)label_blocks(nx, ny, nz, kSegs);    // occupancy pass
  const unsigned nbw = (unsigned)label_blocks(nx, ny, nz, kSegsW);   // label-writing pass
  const unsigned nbs = (unsigned)segment_blocks(nx, ny, nz);  // per-segment passes
  const SegDiv dv{make_fastdiv((uint32_t)words), make_fastdiv((uint32_t)ny)};
  const unsigned nt = (unsigned)T;
  hipLaunchKernelGGL(k_label_occ, dim3(nbc, nt), dim3(kBlock), 0, stream, c, c_eps, occ, R, nx, ny, nz, words, dv,
                     nrun);
  const RowTiles rt = row_tiles(ny, nz, words, kTileSegs);
  if (rt.ty > 0) {
    const int ntile = (int)(rt.nty * ceil_div(nz, rt.tz));
    launch_local<kTileSegs>(ctx, ntile, nt, stream, occ, R, nx, ny, nz, words, rt, nrun);
    const EdgeRows e = edge_rows(rt, ny, nz);
    const int64_t nedge = ((int64_t)e.nzb * ny + (int64_t)e.nyb * (nz - e.nzb)) * words;
    if (nedge > 0)
      hipLaunchKernelGGL(k_label_union_edges, dim3((unsigned)ceil_div(nedge, kBlock), nt), dim3(kBlock), 0, stream, occ,
                         R, nx, ny, nz, words, rt, e, nedge, nrun);
  } else {
    hipLaunchKernelGGL(k_label_union, dim3(nbs, nt), dim3(kBlock), 0, stream, occ, R, nx, ny, nz, words, dv, nrun);
  }
  const unsigned nbg = (unsigned)ceil_div(nseg, (int64_t)kBlock * kSegT);  // passes 3-5 (<= nbs)
  hipLaunchKernelGGL(k_label_flatten, dim3(nbg, nt), dim3(kBlock), 0, stream, occ, R, nseg, blockcount, nrun);
  static_assert(kBlock == compact::kBlock, "block counts and the tiled scan share the block size");
  const int64_t ntiles = (nbg + compact::kTile - 1) / compact::kTile;
  int32_t *bc = (int32_t *)blockcount;
  hipLaunchKernelGGL(compact::k_scan_tile, dim3((unsigned)ntiles, nt), dim3(compact::kTile), 0, stream, bc,
                     (int64_t)nbg, tileoff, (int64_t)nbg, tstride);
  hipLaunchKernelGGL(compact::k_scan_totals, dim3(1, nt), dim3(compact::kTile), 0, stream, tileoff, ntiles, tstride);
  hipLaunchKernelGGL(k_copy_total, dim3(1), dim3(64 * ((T + 63) / 64)), 0, stream, tileoff, ntiles, tstride, T,
                     k_dev);
  hipLaunchKernelGGL(k_label_rank, dim3(nbg, nt), dim3(kBlock), 0, stream, occ, R, nseg, bc, tileoff, nrun, tstride);
  hipLaunchKernelGGL(k_label_resolve, dim3(nbg, nt), dim3(kBlock), 0, stream, occ, R, nseg, nrun);
  if (nx % 256 == 0 && ((uintptr_t)lab & 15) == 0) {
    const int64_t ngroups = nseg / 4;  // whole 256-cell groups: segment s is cells 64 s .. 64 s + 63
    const int64_t per = (int64_t)(kBlock / 64) * kGroupsW;
    hipLaunchKernelGGL(k_label_write4, dim3((unsigned)((ngroups + per - 1) / per), nt), dim3(kBlock), 0, stream, occ,
                       R, lab, (int64_t)nx * ny * nz, nrun);
  } else {
    hipLaunchKernelGGL(k_label_write, dim3(nbw, nt), dim3(kBlock), 0, stream, occ, R, lab, nx, ny, nz, words, dv,
                       nrun);
  }
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
  const int64_t nseg = (int64_t)ny * nz * ceil_div(nx, 64);
  const int64_t nbs = segment_blocks(nx, ny, nz);
  // run ids stay below 2^31: nseg * S <= n3 (S, a power of two, at most the segment width)
  const int64_t nrun = nseg << run_shift(nx);
  // work arrays of every field (the run array holds a slot per possible run but is only
  // touched at the runs that exist)
  const int64_t tstride = nbs / compact::kTile + 2;
  const size_t T = (size_t)ntracers;
  uint32_t *blockcount = (uint32_t *)scratch(ctx, SLOT_LABEL_A, sizeof(uint32_t) * (size_t)nbs * T);
  int32_t *runs = (int32_t *)scratch(ctx, SLOT_LABEL_B, sizeof(int32_t) * (size_t)nrun * T);
  uint64_t *occ = (uint64_t *)scratch(ctx, SLOT_LABEL_C, sizeof(uint64_t) * (size_t)nseg * T);
  int32_t *kdev = (int32_t *)scratch(ctx, SLOT_MISC, sizeof(int32_t) * T);
  int32_t *tileoff = (int32_t *)scratch(ctx, SLOT_MISC3, sizeof(int32_t) * (size_t)tstride * T);
  int32_t *kh = (int32_t *)host_scratch(ctx, sizeof(int32_t) * T);
  if (!blockcount || !runs || !occ || !kdev || !tileoff || !kh) return VOFMT_E_NOMEM;
  int rc = label_all(ctx, nx, ny, nz, ntracers, c, c_eps, labels, occ, runs, blockcount, tileoff, tstride, kdev,
                     stream);
  if (rc) return rc;
  VOFMT_HIP(ctx, hipMemcpyAsync(kh, kdev, sizeof(int32_t) * ntracers, hipMemcpyDeviceToHost, stream));
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  for (int t = 0; t < ntracers; ++t) ndrops_host[t] = kh[t];
  return VOFMT_OK;
}

// Offsets of every field's drop records (prefix sums of the drop counts)
// into device memory, staged in pinned host memory `stage` (ntr + 1 ints,
// not touched again before the call synchronises).
static hipError_t upload_offsets(const int32_t *ndrops_host, int ntr, int32_t *stage, int32_t *dev,
                                 hipStream_t stream) {
  stage[0] = 0;
  for (int t = 0; t < ntr; ++t) stage[t + 1] = stage[t] + ndrops_host[t];
  return hipMemcpyAsync(dev, stage, sizeof(int32_t) * (size_t)(ntr + 1), hipMemcpyHostToDevice, stream);
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
  // records of every field's drops, field after field (toff: their offsets)
  int32_t *rootpos = (int32_t *)scratch(ctx, SLOT_LABEL_C, sizeof(int32_t) * (size_t)(D + 1));
  int32_t *box = (int32_t *)scratch(ctx, SLOT_MISC2, sizeof(int32_t) * (6 + kFrames) * (size_t)(D + 1));
  int32_t *frames = box ? box + 6 * (D + 1) : nullptr;
  int32_t *flags = (int32_t *)scratch(ctx, SLOT_MISC, sizeof(int32_t) * (size_t)(2 + ntracers + 1));
  int32_t *toff = flags ? flags + 2 : nullptr;
  double *part = (double *)scratch(ctx, SLOT_LABEL_A, sizeof(double) * 4 * kSumSplit * (size_t)(D + 1));
  int32_t *fh = (int32_t *)host_scratch(ctx, sizeof(int32_t) * (size_t)(2 + ntracers + 1));
  if (!rootpos || !box || !flags || !part || !fh) return VOFMT_E_NOMEM;
  VOFMT_HIP(ctx, upload_offsets(ndrops_host, ntracers, fh + 2, toff, stream));
  VOFMT_HIP(ctx, hipMemsetAsync(flags, 0, sizeof(int32_t) * 2, stream));
  const FastDiv fnx = make_fastdiv((uint32_t)nx), fny = make_fastdiv((uint32_t)ny);
  const unsigned nbc = ceil_div(n3, kChunk);  // workgroups of the per-drop reductions, per field
  hipLaunchKernelGGL(k_scan_init, dim3(ceil_div(kFrames * D, 256)), dim3(256), 0, stream, rootpos, frames, D);
  hipLaunchKernelGGL(k_drop_scan, dim3(nbc, ntracers), dim3(kBlock), 0, stream, labels, n3, nx, ny, nz, fnx, fny, toff,
                     rootpos, frames);
  hipLaunchKernelGGL(k_drop_box, dim3(ceil_div(D, 256)), dim3(256), 0, stream, (int32_t)D, nx, ny, nz, rootpos, frames,
                     box);
  hipLaunchKernelGGL(k_drop_sums, dim3((unsigned)(D * kSumSplit)), dim3(kBlock), 0, stream, c, labels, nx, ny, nz, toff,
                     rootpos, box, part, flags);
  hipLaunchKernelGGL(k_drop_finish, dim3(ceil_div(D, 256)), dim3(256), 0, stream, (int32_t)D, nx, ny, nz, rootpos, box,
                     part, vol, xyz, flags);
  VOFMT_HIP(ctx, hipGetLastError());
  VOFMT_HIP(ctx, hipMemcpyAsync(fh, flags, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, stream));
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  if (fh[0] & 2) return set_err(ctx, VOFMT_E_ARG, "vofmt_drop_moments: labels do not match ndrops_host");
  if (fh[0]) return set_err(ctx, VOFMT_E_EXTENT, "vofmt_drop_moments: a drop spans half the box or more");
  return VOFMT_OK;
}

// Shapes (and, with vol and xyz, the moments) of the drops: one scan of the
// labels and one pass of sums per tracer.
static int drop_shapes_impl(vofmt_ctx *ctx, const char *fn, bool moments, int32_t nx, int32_t ny, int32_t nz,
                            int32_t ntracers,
                            const double *c, const int32_t *labels, const int32_t *ndrops_host, const double *sx,
                            const double *sy, const double *sz, double *vol, double *xyz, double *inertia,
                            double *chi, double *vel, hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nx < 1 || ny < 1 || nz < 1 || ntracers < 0) return set_err(ctx, VOFMT_E_ARG, "%s: bad sizes", fn);
  if (ntracers == 0) return VOFMT_OK;
  if (!c || !labels || !ndrops_host) return set_err(ctx, VOFMT_E_ARG, "%s: null pointer", fn);
  const bool withu = vel != nullptr;
  if (withu != (sx != nullptr) || withu != (sy != nullptr) || withu != (sz != nullptr))
    return set_err(ctx, VOFMT_E_ARG, "%s: vel, sx, sy and sz must be given together", fn);
  int64_t D = 0;
  for (int t = 0; t < ntracers; ++t) {
    if (ndrops_host[t] < 0) return set_err(ctx, VOFMT_E_ARG, "%s: negative drop count", fn);
    D += ndrops_host[t];
  }
  if (D == 0) return VOFMT_OK;
  if (!inertia || !chi || (moments && (!vol || !xyz))) return set_err(ctx, VOFMT_E_ARG, "%s: null output", fn);
  const int64_t n3 = (int64_t)nx * ny * nz;
  if (n3 >= INT32_MAX) return set_err(ctx, VOFMT_E_ARG, "%s: more than 2^31-1 cells per field", fn);
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  // records of every field's drops, field after field (toff: their offsets)
  int32_t *rootpos = (int32_t *)scratch(ctx, SLOT_LABEL_C, sizeof(int32_t) * (size_t)(D + 1));
  int32_t *box = (int32_t *)scratch(ctx, SLOT_MISC2, sizeof(int32_t) * (6 + kFrames) * (size_t)(D + 1));
  int32_t *frames = box ? box + 6 * (D + 1) : nullptr;
  int32_t *flags = (int32_t *)scratch(ctx, SLOT_MISC, sizeof(int32_t) * (size_t)(2 + ntracers + 1));
  int32_t *toff = flags ? flags + 2 : nullptr;
  double *part = (double *)scratch(ctx, SLOT_LABEL_A, sizeof(double) * kShapeSums * kSumSplit * (size_t)(D + 1));
  int32_t *fh = (int32_t *)host_scratch(ctx, sizeof(int32_t) * (size_t)(2 + ntracers + 1));
  if (!rootpos || !box || !flags || !part || !fh) return VOFMT_E_NOMEM;
  VOFMT_HIP(ctx, upload_offsets(ndrops_host, ntracers, fh + 2, toff, stream));
  VOFMT_HIP(ctx, hipMemsetAsync(flags, 0, sizeof(int32_t) * 2, stream));
  const FastDiv fnx = make_fastdiv((uint32_t)nx), fny = make_fastdiv((uint32_t)ny);
  const unsigned nbc = ceil_div(n3, kChunk);
  hipLaunchKernelGGL(k_scan_init, dim3(ceil_div(kFrames * D, 256)), dim3(256), 0, stream, rootpos, frames, D);
  hipLaunchKernelGGL(k_drop_scan, dim3(nbc, ntracers), dim3(kBlock), 0, stream, labels, n3, nx, ny, nz, fnx, fny, toff,
                     rootpos, frames);
  hipLaunchKernelGGL(k_drop_box, dim3(ceil_div(D, 256)), dim3(256), 0, stream, (int32_t)D, nx, ny, nz, rootpos, frames,
                     box);
  hipLaunchKernelGGL(k_shape_sums, dim3((unsigned)(D * kSumSplit)), dim3(kBlock), 0, stream, c, labels, sx, sy, sz, nx,
                     ny, nz, toff, rootpos, box, part, flags);
  hipLaunchKernelGGL(k_shape_finish, dim3(ceil_div(D, 256)), dim3(256), 0, stream, (int32_t)D, nx, ny, nz, rootpos,
                     box, part, inertia, chi, withu ? vel : nullptr, vol, xyz, flags);
  VOFMT_HIP(ctx, hipGetLastError());
  VOFMT_HIP(ctx, hipMemcpyAsync(fh, flags, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, stream));
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  if (fh[0] & 2) return set_err(ctx, VOFMT_E_ARG, "%s: labels do not match ndrops_host", fn);
  if (fh[0]) return set_err(ctx, VOFMT_E_EXTENT, "%s: a drop spans half the box or more", fn);
  return VOFMT_OK;
}

extern "C" int vofmt_drop_shapes(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers,
                                 const double *c, const int32_t *labels, const int32_t *ndrops_host,
                                 const double *sx, const double *sy, const double *sz, double *inertia, double *chi,
                                 double *vel, hipStream_t stream) {
  return drop_shapes_impl(ctx, "vofmt_drop_shapes", false, nx, ny, nz, ntracers, c, labels, ndrops_host, sx, sy, sz,
                          nullptr, nullptr, inertia, chi, vel, stream);
}

extern "C" int vofmt_drop_moments_shapes(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers,
                                         const double *c, const int32_t *labels, const int32_t *ndrops_host,
                                         const double *sx, const double *sy, const double *sz, double *vol,
                                         double *xyz, double *inertia, double *chi, double *vel, hipStream_t stream) {
  return drop_shapes_impl(ctx, "vofmt_drop_moments_shapes", true, nx, ny, nz, ntracers, c, labels, ndrops_host, sx,
                          sy, sz, vol, xyz, inertia, chi, vel, stream);
}
