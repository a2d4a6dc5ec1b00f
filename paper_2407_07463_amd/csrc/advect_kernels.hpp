// Device bodies of one advection sweep, shared by the plain launches
// (vofmt_advect) and the batched persistent launches (vofmt_advect_batched):
// both paths run exactly this code, so their results agree bit for bit.
//
// Direction-split geometric PLIC advection of N tracer fields (eq. 3 of the
// paper applied to every tracer C_i; its discrete form is the conservative
// split scheme of Weymouth & Yue 2010 with MYC normals).
//
// A sweep is two passes.
//
// plic_body<D>: one wavefront per region of the list of mixed cells
//   (values more than 1e-12 inside (0, 1)) of the sweep's input field. Each entry gathers its 3x3x3
//   block, computes the MYC normal and the plane constant, and writes the flux
//   of every face the cell donates through (its lower face if s < 0 there, its
//   upper face if s > 0) into the face-flux array fmix[t][p] (the lower d-face
//   of cell p). The list is compact, so this FP64 work runs at full SIMD width.
//
// stream_body<D,G>: one thread per (x, row) of the plane transverse to its
//   marching axis, for G tracers at once. For a pure donor the flux is s*c;
//   for a mixed donor it is read from fmix. Sweeps along y or z march along
//   the sweep axis and carry c and the lower-face flux in registers, so every
//   field value is read from memory once; in the x-sweep each lane forms both
//   of its faces from its own and its neighbour lanes' values. A wavefront
//   owns 64 consecutive x-cells of one row, so every load and store of a field
//   row is a coalesced 512-byte transaction and the c > 0.5 indicator of the
//   64 cells is one 64-bit ballot word. The new field is written in the same
//   row layout, and every new mixed cell is appended to the list of the next
//   sweep.
//
// The list is cut into regions of rsize entries, one per wavefront of the
// pass that fills it, each large enough for every cell that wavefront handles
// (64 * chunk * G): entries are written without atomics, in a fixed order,
// and the region's length is stored beside it. No barrier, no LDS.
#pragma once

#include "common.hpp"
#include "plic.hpp"

namespace advect {

constexpr int kMaxGroup = 4;  // tracers per streaming pass (register budget)

// Workgroup grid of a streaming pass (4 wavefronts per workgroup, or wpb
// for the x-sweep).
//   d = 0, wpb = 0 (whole rows): a wavefront takes one y-row and P =
//          max(1, chunk / segments per row) positions along z; gx = 1,
//          gy = groups of 4 rows, gz = groups of P positions;
//   d = 0, wpb > 0: a workgroup takes rpb y-rows of spw consecutive 64-cell
//          x-segments each (spw = min(segments per row, wpb), rpb = wpb/spw);
//          gx = chunks of spw segments, gy = groups of rpb rows, gz = chunks
//          of z.
//   d = 1: rows of a multiple of 4 segments: gx = groups of 4 consecutive
//          64-cell segments (one per wavefront, so a workgroup's loads at
//          each position are one contiguous run), gy = z-rows; other rows:
//          gx = segments, gy = groups of 4 z-rows (no idle wavefronts on
//          short rows); gz = chunks of y.
//   d = 2: the same with y-rows and chunks of z.
struct Tiles {
  int gx, gy, gz;
};
__host__ __device__ inline int x_segments_per_row(int words, int wpb) { return words < wpb ? words : wpb; }
// Planes per whole-row x-sweep wavefront: half a chunk's cells (two 512-cell
// rows at chunk 32; four measured 2% slower on that sweep).
__host__ __device__ inline int x_row_positions(int words, int chunk) {
  return (chunk / 2) / words > 0 ? (chunk / 2) / words : 1;
}
__host__ __device__ inline Tiles stream_tiles(int d, int nx, int ny, int nz, int chunk, int wpb = 4) {
  const int words = (nx + 63) / 64;
  if (d == 0 && wpb == 0) {
    const int P = x_row_positions(words, chunk);
    return Tiles{1, (ny + 3) / 4, (nz + P - 1) / P};
  }
  if (d == 0) {
    const int spw = x_segments_per_row(words, wpb), rpb = wpb / spw;
    return Tiles{(words + spw - 1) / spw, (ny + rpb - 1) / rpb, (nz + chunk - 1) / chunk};
  }
  const bool seg4 = words % 4 == 0;
  if (d == 1) return seg4 ? Tiles{words / 4, nz, (ny + chunk - 1) / chunk}
                          : Tiles{words, (nz + 3) / 4, (ny + chunk - 1) / chunk};
  return seg4 ? Tiles{words / 4, ny, (nz + chunk - 1) / chunk} : Tiles{words, (ny + 3) / 4, (nz + chunk - 1) / chunk};
}

struct Divisors {
  FastDiv n3, nx, ny;  // entry -> (tracer, cell), cell -> (i, j, k)
};

// Mixed cells of the initial field: wavefront w scans tracer-cells
// [w*rsize, (w+1)*rsize) of the whole array.
__device__ __forceinline__ void scan_body(const double *__restrict__ c, int64_t total, uint32_t *__restrict__ list,
                                          int *__restrict__ counts, int64_t nregions, int rsize, int64_t w) {
  const int lane = threadIdx.x & 63;
  if (w >= nregions) return;
  uint32_t *out = list + w * rsize;
  int n = 0;
  const uint64_t below = (1ull << lane) - 1;
  for (int64_t base = w * rsize; base < (w + 1) * rsize && base < total; base += 64) {
    const int64_t q = base + lane;
    const bool mixed = (q < total) && plic::is_mixed(c[q]);
    const uint64_t mask = __ballot(mixed);
    if (mixed) out[n + __popcll(mask & below)] = (uint32_t)q;
    n += __popcll(mask);
  }
  if (lane == 0) counts[w] = n;
}

// Fluxes through the faces along D that a mixed cell donates through, from
// its 3x3x3 block b (centre value b[13]): MYC normal, plane constant, then the
// volume of the sub-box that crosses each face within the sweep: [0, |s|]
// along D for the lower face (when s_lo < 0), [1 - s, 1] for the upper face
// (when s_hi > 0). The flux is s times that volume; faces not donated through
// get 0.
template <int D>
__device__ __forceinline__ void plic_fluxes(const double *b, double s_lo, double s_hi, double &f_lo, double &f_hi) {
  double mx, my, mz;
  plic::myc_normal(b, mx, my, mz);
  const double alpha = plic::alpha_of(mx, my, mz, b[13]);
  const double md = (D == 0) ? mx : ((D == 1) ? my : mz);
  f_lo = 0.0;
  f_hi = 0.0;
#pragma unroll 1
  for (int face = 0; face < 2; ++face) {
    const double sv = (face == 0) ? s_lo : s_hi;
    if (face == 0 ? !(sv < 0.0) : !(sv > 0.0)) continue;
    const double x0 = (face == 0) ? 0.0 : 1.0 - sv;
    const double as = alpha - md * x0;
    const double ms = md * fabs(sv);
    double v;
    if (D == 0) v = plic::volume(ms, my, mz, as);
    else if (D == 1) v = plic::volume(mx, ms, mz, as);
    else v = plic::volume(mx, my, ms, as);
    if (face == 0) f_lo = sv * v;
    else f_hi = sv * v;
  }
}

template <int D>
__device__ __forceinline__ void plic_body(const double *__restrict__ cin, const double *__restrict__ s,
                                          const uint32_t *__restrict__ list, const int *__restrict__ counts,
                                          int64_t nregions, int rsize, double *__restrict__ fmix, int nx, int ny,
                                          int nz, const Divisors &dv, int64_t w) {
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int lane = threadIdx.x & 63;
  if (w >= nregions) return;
  const int nq = counts[w];
  const uint32_t *reg = list + w * rsize;
  for (int q = lane; q < nq; q += 64) {
    const uint32_t e = reg[q];
    const uint32_t t = fast_div(e, dv.n3);
    const uint32_t p32 = e - t * dv.n3.d;
    const uint32_t row = fast_div(p32, dv.nx);
    const int i = (int)(p32 - row * (uint32_t)nx);
    const uint32_t k32 = fast_div(row, dv.ny);
    const int j = (int)(row - k32 * (uint32_t)ny), k = (int)k32;
    const int64_t p = p32;
    const int64_t pu = (D == 0) ? p - i + wrap_inc(i, nx)
                                : ((D == 1) ? ((int64_t)k * ny + wrap_inc(j, ny)) * nx + i
                                            : ((int64_t)wrap_inc(k, nz) * ny + j) * nx + i);
    const double s_lo = s[p], s_hi = s[pu];
    if (!(s_lo < 0.0) && !(s_hi > 0.0)) continue;  // donates through neither face
    const double *ct = cin + t * n3;
    double b[27];
    {
      const int im = wrap_dec(i, nx), ip = wrap_inc(i, nx);
      const int jm = wrap_dec(j, ny), jp = wrap_inc(j, ny);
      const int km = wrap_dec(k, nz), kp = wrap_inc(k, nz);
      const int xs[3] = {im, i, ip};
      const int ys[3] = {jm, j, jp};
      const int zs[3] = {km, k, kp};
#pragma unroll
      for (int az = 0; az < 3; ++az)
#pragma unroll
        for (int ay = 0; ay < 3; ++ay) {
          const double *rowp = ct + ((int64_t)zs[az] * ny + ys[ay]) * nx;
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) b[ax + 3 * ay + 9 * az] = rowp[xs[ax]];
        }
    }
    double f_lo, f_hi;
    plic_fluxes<D>(b, s_lo, s_hi, f_lo, f_hi);
    double *ft = fmix + t * n3;
    if (s_lo < 0.0) ft[p] = f_lo;
    if (s_hi > 0.0) ft[pu] = f_hi;
  }
}

// Lane i receives lane i-1's value (lane 0 keeps its own): a DPP wave shift
// right by one lane on each 32-bit half (all lanes active).
__device__ __forceinline__ double from_lane_below(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = (int)b, hi = (int)(b >> 32);
  const int rlo = __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);
  const int rhi = __builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
  return __longlong_as_double(((long long)rhi << 32) | (long long)(unsigned)rlo);
}
// Lane i receives lane i+1's value (lane 63 keeps its own): wave shift left.
__device__ __forceinline__ double from_lane_above(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = (int)b, hi = (int)(b >> 32);
  const int rlo = __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);
  const int rhi = __builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
  return __longlong_as_double(((long long)rhi << 32) | (long long)(unsigned)rlo);
}

// (tile, tracer group) of work item L of a streaming pass that covers ngrp
// groups of tracers over a gx x gy x gz tile grid (L < gx*gy*gz*ngrp).
// Workgroups are dealt to the 8 XCDs in turn by linear id, so each block of
// 8*ngrp consecutive items holds 8 tiles (fewer in the last block) and gives
// the groups of one tile items that are a multiple of 8 apart: they run on
// the same XCD at about the same time, and the face velocity the groups
// share is read from HBM once and from that XCD's L2 by the others.
// Tiles are numbered row-first (bx, then by, then the chunk bz), or with
// cfast chunk-first (bx, bz, by). The y-sweep takes the latter: neighbouring
// workgroups then march one z-plane at different y (128 KiB apart at 512^2
// planes) instead of neighbouring z-planes at the same y (2 MiB apart); it
// measured 7% faster there and slower on the other two sweeps.
struct GroupTile {
  int bx, by, bz, grp;
};
__host__ __device__ inline GroupTile group_tile(int64_t L, int gx, int gy, int gz, int ngrp, bool cfast) {
  const int64_t ntile = (int64_t)gx * gy * gz;
  const int64_t blk = L / (8 * ngrp), r = L - blk * 8 * ngrp;
  const int64_t q = (ntile - blk * 8 < 8) ? ntile - blk * 8 : 8;  // tiles in this block
  const int64_t tile = blk * 8 + r % q;
  GroupTile o;
  o.grp = (int)(r / q);
  o.bx = (int)(tile % gx);
  if (cfast) {
    o.bz = (int)((tile / gx) % gz);
    o.by = (int)(tile / ((int64_t)gx * gz));
  } else {
    o.by = (int)((tile / gx) % gy);
    o.bz = (int)(tile / ((int64_t)gx * gy));
  }
  return o;
}

// Tile (bx, by, bz) of a streaming pass laid out as a gx x gy x gz grid of
// workgroups (stream_tiles): 4 wavefronts, or WPB for the x-sweep.
template <int D, int G, int WPB = 4>
__device__ __forceinline__ void stream_body(const double *__restrict__ cin, double *__restrict__ cout,
                                            const double *__restrict__ s, const double *__restrict__ fmix,
                                            uint64_t *__restrict__ ccbits, int write_cc, int t0, int nx, int ny,
                                            int nz, int words, int chunk, uint32_t *__restrict__ list_next,
                                            int *__restrict__ counts_next, int64_t region0, int rsize, int bx, int by,
                                            int bz, int gx, int gy) {
  const int lane = threadIdx.x & 63;
  // wavefront-uniform: kept in a scalar register, like everything derived from it
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // x-sweep with WPB = 0: the wavefront marches along whole rows (row 4*by + wv)
  constexpr bool ROWS = (D == 0 && WPB == 0);
  constexpr int W = (D == 0 && !ROWS) ? WPB : 4;  // wavefronts per workgroup
  // x-sweep (WPB > 0): wavefront wv takes segment bx*spw + sw of row by*rpb + rr;
  // whole-row x-sweep: row 4*by + wv; y- and z-sweeps: segment 4*bx + wv of
  // row by when a row has a multiple of 4 segments, else segment bx of row 4*by + wv
  const int spw = (D == 0 && !ROWS) ? x_segments_per_row(words, W) : 1;
  const int rpb = (D == 0 && !ROWS) ? W / spw : 1;
  const int rr = wv / spw, sw = wv % spw;
  const bool tile_ok = (D != 0 || ROWS) || (rr < rpb && by * rpb + rr < ny && bx * spw + sw < words);
  // (the whole-row march moves seg along the row)
  const bool seg4 = D != 0 && words % 4 == 0;
  int seg = (D == 0 && !ROWS) ? bx * spw + sw : (seg4 ? bx * 4 + wv : bx);
  int x = seg * 64 + lane;
  const int row = (D == 0 && !ROWS) ? ((by * rpb + rr < ny) ? by * rpb + rr : ny - 1) : (seg4 ? by : by * 4 + wv);
  const int nrow = (D == 1) ? nz : ny;
  const int nm = (D == 1) ? ny : nz;
  const int64_t wave = region0 + (((int64_t)bz * gy + by) * gx + bx) * W + wv;
  // whole wavefront (the LDS x-sweep keeps every wavefront for its barriers)
  if ((D != 0 || ROWS) && (row >= nrow || (D != 0 && seg >= words))) {
    if (lane == 0) counts_next[wave] = 0;
    return;
  }
  uint32_t *reg = list_next + wave * rsize;
  int nlist = 0;  // wavefront-uniform
  const uint64_t below = (1ull << lane) - 1;
  bool live = tile_ok && x < nx;  // (an idle x-sweep wavefront has no live lane)
  int xs = live ? x : nx - 1;  // dead lanes shadow a valid cell, never store
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int64_t nbits = (int64_t)nz * ny * words;
  const int mchunk = ROWS ? x_row_positions(words, chunk) : chunk;  // positions of this wavefront
  const int m0 = bz * mchunk;
  const int m1 = (m0 + mchunk < nm) ? m0 + mchunk : nm;
  const double *c_g = cin + (int64_t)t0 * n3;
  double *o_g = cout + (int64_t)t0 * n3;
  const double *f_g = fmix + (int64_t)t0 * n3;
  uint64_t *b_g = ccbits + (int64_t)t0 * nbits;

  auto cell = [&](int xx, int mm) -> int64_t {
    if (D == 1) return ((int64_t)row * ny + mm) * nx + xx;
    return ((int64_t)mm * ny + row) * nx + xx;
  };
  auto bitword = [&](int mm) -> int64_t {
    if (D == 1) return ((int64_t)row * ny + mm) * words + seg;
    return ((int64_t)mm * ny + row) * words + seg;
  };
  // flux through the lower face of cell pu: donor = the lower cell (value cl)
  // if s > 0, else the upper cell (value cu); a mixed donor's flux is in fmix
  auto flux = [&](int t, double sv, double cl, double cu, int64_t pu) -> double {
    const double cd = (sv > 0.0) ? cl : cu;
    const bool mixed = (sv != 0.0) && plic::is_mixed(cd);
    double fv = 0.0;
    if (mixed) fv = f_g[t * n3 + pu];
    return mixed ? fv : ((sv == 0.0) ? 0.0 : sv * cd);
  };
  // the c_c bit words of row word wrow that finish() reads (unless this
  // sweep writes them), loaded ahead of their use so their latency overlaps
  // other work
  auto load_words = [&](int64_t wrow, uint64_t *ccw) {
    const bool ok = tile_ok && seg < words;  // idle: no cells
#pragma unroll
    for (int t = 0; t < G; ++t) ccw[t] = (!write_cc && ok) ? b_g[t * nbits + wrow] : 0ull;
  };
  // new value of cell pc, its c_c bit, and its entry in the next list
  auto finish = [&](int t, double cold, double f_lo, double f_hi, double s_lo, double s_hi, int64_t pc, int64_t wrow,
                    uint64_t ccw) {
    double ccv;
    if (write_cc) {
      const uint64_t word = __ballot(live && cold > 0.5);
      if (lane == 0 && tile_ok && seg < words) b_g[t * nbits + wrow] = word;
      ccv = (cold > 0.5) ? 1.0 : 0.0;
    } else {
      ccv = ((ccw >> lane) & 1ull) ? 1.0 : 0.0;
    }
    const double cn = (cold - (f_hi - f_lo)) + ccv * (s_hi - s_lo);
    // streamed out (not read again by this pass): a non-temporal store
    if (live) __builtin_nontemporal_store(cn, &o_g[t * n3 + pc]);
    const bool mixed = live && plic::is_mixed(cn);
    const uint64_t mask = __ballot(mixed);
    if (mixed) reg[nlist + __popcll(mask & below)] = (uint32_t)((int64_t)(t0 + t) * n3 + pc);
    nlist += __popcll(mask);
  };

  if constexpr (D != 0) {
    // ---- march along the sweep axis: faces m0..m1, cells m0..m1-1
    const int ml = (m0 == 0) ? nm - 1 : m0 - 1;
    double cm[G], flo[G];
    const int64_t p0 = cell(xs, m0);
    const double s0 = s[p0];
    double s_lo = s0;
    {
      const int64_t pl = cell(xs, ml);
      double cl[G];
#pragma unroll
      for (int t = 0; t < G; ++t) {
        cl[t] = c_g[t * n3 + pl];
        cm[t] = c_g[t * n3 + p0];
      }
#pragma unroll
      for (int t = 0; t < G; ++t) flo[t] = flux(t, s0, cl[t], cm[t], p0);
    }
    // the upper cell's values, and the bit words of the cell finished next,
    // are loaded one position ahead, so their latency overlaps the previous
    // position's flux work and stores
    double s_nx = 0.0, c_nx[G];
    uint64_t ccw[G];
    if (m0 + 1 <= m1) {
      const int64_t pu = cell(xs, (m0 + 1 == nm) ? 0 : m0 + 1);
      s_nx = s[pu];
#pragma unroll
      for (int t = 0; t < G; ++t) c_nx[t] = c_g[t * n3 + pu];
    }
    load_words(bitword(m0), ccw);
    for (int m = m0 + 1; m <= m1; ++m) {
      const int mm = (m == nm) ? 0 : m;
      const int64_t pu = cell(xs, mm);
      const int64_t pc = cell(xs, m - 1);
      const int64_t wrow = bitword(m - 1);
      const double s_hi = s_nx;
      double cu[G], fhi[G];
      uint64_t ccc[G];
#pragma unroll
      for (int t = 0; t < G; ++t) {
        cu[t] = c_nx[t];
        ccc[t] = ccw[t];
      }
      if (m + 1 <= m1) {
        const int64_t pn = cell(xs, (m + 1 == nm) ? 0 : m + 1);
        s_nx = s[pn];
#pragma unroll
        for (int t = 0; t < G; ++t) c_nx[t] = c_g[t * n3 + pn];
        load_words(bitword(m), ccw);
      }
#pragma unroll
      for (int t = 0; t < G; ++t) fhi[t] = flux(t, s_hi, cm[t], cu[t], pu);
#pragma unroll
      for (int t = 0; t < G; ++t) {
        finish(t, cm[t], flo[t], fhi[t], s_lo, s_hi, pc, wrow, ccc[t]);
        flo[t] = fhi[t];
        cm[t] = cu[t];
      }
      s_lo = s_hi;
    }
  } else if constexpr (ROWS) {
    // ---- x-sweep along whole rows: the wavefront takes its row's 64-cell
    // segments in order, position after position (z-planes m0..m1-1). Lanes
    // take their neighbours inside a segment by wave shifts; lane 0 takes the
    // previous segment's last cell, the last cell the next segment's first,
    // and the row closes periodically through its first and last cells. The
    // next step's values, the last cell of its row and its bit words are
    // loaded one step ahead. No barrier, no LDS.
    auto readlane_d = [](double v, int l) {
      const long long b = __double_as_longlong(v);
      const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
      return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
    };
    // values of (position mm, segment sk): lanes past the row's end shadow its last cell
    const int nk = (m1 - m0) * words;  // steps: (position - m0) * words + segment
    auto load_step = [&](int mm, int sk, double *cv, double &sv) {
      const int xk = sk * 64 + lane;
      const int64_t p = ((int64_t)mm * ny + row) * nx + ((xk < nx) ? xk : nx - 1);
      sv = s[p];
#pragma unroll
      for (int t = 0; t < G; ++t) cv[t] = c_g[t * n3 + p];
    };
    auto load_last = [&](int mm, double *cv) {
      const int64_t p = ((int64_t)mm * ny + row) * nx + (nx - 1);
#pragma unroll
      for (int t = 0; t < G; ++t) cv[t] = c_g[t * n3 + p];
    };
    auto words_of = [&](int mm, int sk, uint64_t *ccw) {
      const int64_t w = ((int64_t)mm * ny + row) * words + sk;
#pragma unroll
      for (int t = 0; t < G; ++t) ccw[t] = write_cc ? 0ull : b_g[t * nbits + w];
    };
    double c_cur[G], c_nxt[G], c_lst[G], c_lst_nxt[G], c_fst[G], c_prv[G];
    double s_cur = 0.0, s_nxt = 0.0, s_fst = 0.0;
    uint64_t ccw[G], ccw_nxt[G];
#pragma unroll
    for (int t = 0; t < G; ++t) c_prv[t] = c_fst[t] = 0.0;
    if (m0 < m1) {
      load_step(m0, 0, c_cur, s_cur);
      load_last(m0, c_lst);
      words_of(m0, 0, ccw);
    }
    int mk = m0, sk = 0;
    for (int k = 0; k < nk; ++k) {
      int mn = mk, sn = sk + 1;
      if (sn == words) {
        sn = 0;
        mn = mk + 1;
      }
      if (mn < m1) {
        load_step(mn, sn, c_nxt, s_nxt);
        if (sn == 0) load_last(mn, c_lst_nxt);
        words_of(mn, sn, ccw_nxt);
      }
      seg = sk;
      x = sk * 64 + lane;
      live = x < nx;
      xs = live ? x : nx - 1;
      const int last = (sk == words - 1) ? (nx - 1) - 64 * sk : 63;  // the segment's last live lane
      const bool at_end = (lane == last);
      const bool row_end = (sk == words - 1);
      if (sk == 0) {  // the row's first cell closes it at its end
#pragma unroll
        for (int t = 0; t < G; ++t) c_fst[t] = readlane_d(c_cur[t], 0);
        s_fst = readlane_d(s_cur, 0);
      }
      const int64_t rb = ((int64_t)mk * ny + row) * nx;
      const int64_t pc = rb + xs;
      const int64_t pr = (xs == nx - 1) ? rb : pc + 1;
      const int64_t wrow = ((int64_t)mk * ny + row) * words + sk;
      const double s_lo = s_cur;
      const double s_dn = from_lane_above(s_cur);
      const double s_end = row_end ? s_fst : readlane_d(s_nxt, 0);
      const double s_hi = at_end ? s_end : s_dn;
      double cl[G], cr[G], flo[G], fhi[G];
#pragma unroll
      for (int t = 0; t < G; ++t) {
        const double up = from_lane_below(c_cur[t]);
        const double dn = from_lane_above(c_cur[t]);
        const double beg = (sk == 0) ? c_lst[t] : c_prv[t];
        const double end = row_end ? c_fst[t] : readlane_d(c_nxt[t], 0);
        cl[t] = (lane == 0) ? beg : up;
        cr[t] = at_end ? end : dn;
      }
#pragma unroll
      for (int t = 0; t < G; ++t) {
        flo[t] = flux(t, s_lo, cl[t], c_cur[t], pc);
        fhi[t] = flux(t, s_hi, c_cur[t], cr[t], pr);
      }
#pragma unroll
      for (int t = 0; t < G; ++t) finish(t, c_cur[t], flo[t], fhi[t], s_lo, s_hi, pc, wrow, ccw[t]);
      // carry to the next step
#pragma unroll
      for (int t = 0; t < G; ++t) {
        c_prv[t] = readlane_d(c_cur[t], 63);
        c_cur[t] = c_nxt[t];
        ccw[t] = ccw_nxt[t];
        if (sn == 0) c_lst[t] = c_lst_nxt[t];
      }
      s_cur = s_nxt;
      mk = mn;
      sk = sn;
    }
  } else {
    // ---- x-sweep: positions are z-planes; faces along x inside the row.
    // Each lane forms both of its faces from its own and its neighbour lanes'
    // values. The values beyond a segment's two ends come from the adjacent
    // wavefronts of the workgroup through LDS (one barrier per position,
    // double-buffered); only the workgroup's own two ends read memory, or
    // wrap inside the workgroup when it holds the whole row.
    __shared__ double edge[2][W][2][G + 1];  // [parity][wavefront][first, last][tracers..., s]
    const int ngs = (words - bx * spw < spw) ? words - bx * spw : spw;  // segments of this row chunk
    const bool whole_row = (bx == 0) && (words <= spw);
    const int x_last = (seg * 64 + 63 < nx) ? seg * 64 + 63 : nx - 1;
    const bool first = (lane == 0);
    const bool last = tile_ok && (x == x_last);
    const int xl = (xs == 0) ? nx - 1 : xs - 1;
    const int xr = (xs == nx - 1) ? 0 : xs + 1;
    // the neighbours come from LDS unless they lie outside the workgroup's row chunk
    const bool l_lds = tile_ok && ((sw > 0) || whole_row);
    const bool r_lds = tile_ok && ((sw + 1 < ngs) || whole_row);
    const int wl = !tile_ok ? wv : ((sw > 0) ? wv - 1 : wv + ngs - 1);
    const int wr = !tile_ok ? wv : ((sw + 1 < ngs) ? wv + 1 : wv - sw);
    for (int m = m0; m < m1; ++m) {
      const int64_t pc = cell(xs, m);
      const int64_t pl = cell(xl, m);
      const int64_t pr = cell(xr, m);
      const int64_t wrow = bitword(m);
      const int par = m & 1;
      const double s_lo = s[pc];
      double c0[G], cl[G], cr[G];
#pragma unroll
      for (int t = 0; t < G; ++t) c0[t] = c_g[t * n3 + pc];
      if (tile_ok && (first || last)) {
        const int side = first ? 0 : 1;
#pragma unroll
        for (int t = 0; t < G; ++t) edge[par][wv][side][t] = c0[t];
        edge[par][wv][side][G] = s_lo;
      }
      if (first && last) {  // a one-cell segment is both ends
#pragma unroll
        for (int t = 0; t < G; ++t) edge[par][wv][1][t] = c0[t];
        edge[par][wv][1][G] = s_lo;
      }
      __syncthreads();
      double s_end = 0.0, c_beg[G], c_end[G];
#pragma unroll
      for (int t = 0; t < G; ++t) {
        c_beg[t] = 0.0;
        c_end[t] = 0.0;
      }
      if (first) {
        if (l_lds) {
#pragma unroll
          for (int t = 0; t < G; ++t) c_beg[t] = edge[par][wl][1][t];
        } else {
#pragma unroll
          for (int t = 0; t < G; ++t) c_beg[t] = c_g[t * n3 + pl];
        }
      }
      if (last) {
        if (r_lds) {
          s_end = edge[par][wr][0][G];
#pragma unroll
          for (int t = 0; t < G; ++t) c_end[t] = edge[par][wr][0][t];
        } else {
          s_end = s[pr];
#pragma unroll
          for (int t = 0; t < G; ++t) c_end[t] = c_g[t * n3 + pr];
        }
      }
      const double s_dn = __shfl_down(s_lo, 1, 64);
      const double s_hi = last ? s_end : s_dn;
#pragma unroll
      for (int t = 0; t < G; ++t) {
        const double up = __shfl_up(c0[t], 1, 64);
        const double dn = __shfl_down(c0[t], 1, 64);
        cl[t] = first ? c_beg[t] : up;
        cr[t] = last ? c_end[t] : dn;
      }
      double flo[G], fhi[G];
#pragma unroll
      for (int t = 0; t < G; ++t) {
        flo[t] = flux(t, s_lo, cl[t], c0[t], pc);
        fhi[t] = flux(t, s_hi, c0[t], cr[t], pr);
      }
#pragma unroll
      for (int t = 0; t < G; ++t) {
        const uint64_t ccw = (!write_cc && tile_ok && seg < words) ? b_g[t * nbits + wrow] : 0ull;
        finish(t, c0[t], flo[t], fhi[t], s_lo, s_hi, pc, wrow, ccw);
      }
    }
  }
  if (lane == 0) counts_next[wave] = nlist;
}

// ---------------------------------------------------------------- host side

// Wavefronts of one streaming pass along axis d (each owns one list region).
static inline int64_t stream_waves(int d, int nx, int ny, int nz, int chunk, int wpb = 4) {
  const Tiles g = stream_tiles(d, nx, ny, nz, chunk, wpb);
  return ((d == 0 && wpb > 0) ? wpb : 4) * (int64_t)g.gx * g.gy * g.gz;
}

// Tracer groups of one sweep: kMaxGroup tracers at a time, then groups of
// 2 and 1 for the rest. Launches and the sizing of the list regions both use
// these functions.
static inline int group_size(int left) {
  if (left >= kMaxGroup) return kMaxGroup;
  if (left >= 2) return 2;
  return 1;
}
static inline int num_groups(int ntr) {
  int n = 0;
  for (int t = 0; t < ntr; t += group_size(ntr - t)) ++n;
  return n;
}
// List entries per region: every cell a wavefront of a streaming pass writes.
static inline int region_size(int chunk) { return 64 * chunk * kMaxGroup; }
// Regions of one list: the largest streaming sweep, or the initial scan.
static inline int64_t max_regions(int nx, int ny, int nz, int ntr, int chunk, int wpb = 4) {
  int64_t r = 0;
  for (int d = 0; d < 3; ++d) {
    const int64_t w = stream_waves(d, nx, ny, nz, chunk, wpb) * num_groups(ntr);
    r = w > r ? w : r;
  }
  const int64_t total = (int64_t)ntr * nx * ny * nz;
  const int64_t scan = (total + region_size(chunk) - 1) / region_size(chunk);
  return scan > r ? scan : r;
}

}  // namespace advect
