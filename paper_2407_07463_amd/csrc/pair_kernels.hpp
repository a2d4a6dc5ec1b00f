// Two consecutive sweeps of the split advection scheme (eq. 3 of the paper
// applied to every tracer; the discrete scheme of Weymouth & Yue 2010) with
// one read and one write of the fields.
//
// Sweeps i (axis A) and i+1 (axis B) of a call take F0 (the fields before
// sweep i) through F1 to F2. Four launches per pair:
//
//   K1 plic_body<A>: the mixed cells of F0 -> face fluxes fmA (as in a
//      single sweep).
//   K2 cand_body<A,B>: over the candidate list of F1, the value F1 of each
//      candidate, formed exactly as the streaming pass of sweep A forms it;
//      keeps the mixed ones that donate through a B-face.
//   K3 plic_b_body<A,B>: over those, the 3x3x3 block of F1 around the cell
//      (each value formed from F0, s_A, c_c and fmA the same way), MYC normal,
//      plane constant and the B-face fluxes -> fmB.
//   K4 k_pair<A,B,N>: F2 from F0 on every cell. A workgroup owns a 64 x 8
//      tile of an x-y plane and marches along z through 64 planes, keeping
//      planes of F0, F1 and F2 (each with the halo the next stage reads) in
//      LDS rings. It writes F2, the mixed cells of F2 (the next K1's list)
//      and the candidates of the following sweep along N (the next K2's list).
//
// A cell is a candidate for a sweep when one of its two faces along the
// sweep axis has a mixed donor (that flux needs the PLIC pass) or when the
// value the sweep gives it with pure-donor fluxes lies strictly between 0
// and 1. Every cell that is mixed after the sweep is therefore a candidate,
// including the round-off excursions of bulk cells (1 - 2^-53 after a
// converging face pair), which the scheme counts as mixed.
//
// Every value is formed by the same expressions, in the same order, as in
// stream_body and plic_body, so a paired pass and two single sweeps give
// bit-identical fields.
//
// c_c bits: phase = i mod 3. Phase 0 (sweep i starts a step): c_c = F0 > 0.5,
// written for the step. Phase 1: both sweeps read the bits of their step.
// Phase 2 (sweep i+1 starts the next step): sweep i reads the bits of its
// step, sweep i+1 uses F1 > 0.5 and writes them for the next step, into the
// other of two bit arrays (one per step parity), so no launch reads bits that
// it also writes.
#pragma once

#include "advect_kernels.hpp"

namespace advect {

constexpr int kPairTY = 8;     // tile rows (y) of a paired pass
constexpr int kPairTZ = 64;    // planes (z) per workgroup of a paired pass
constexpr int kPairThreads = 256;
constexpr int kNoAxis = 3;     // no following sweep: no candidate list
static_assert(2 * 64 * kPairTZ <= 64 * 32 * kMaxGroup, "a paired wavefront's list entries fit one region");

// Flux through the lower face of cell u (Courant number sv), lower cell value
// cl, upper cell value cu; a mixed donor's flux is fm[f]. Same expression as
// the streaming pass.
__device__ __forceinline__ double face_flux(double sv, double cl, double cu, const double *__restrict__ fm,
                                            int64_t f) {
  const double cd = (sv > 0.0) ? cl : cu;
  const bool mixed = (sv != 0.0) && cd > 0.0 && cd < 1.0;
  double fv = 0.0;
  if (mixed) fv = fm[f];
  return mixed ? fv : ((sv == 0.0) ? 0.0 : sv * cd);
}
__device__ __forceinline__ bool mixed_donor(double sv, double cl, double cu) {
  const double cd = (sv > 0.0) ? cl : cu;
  return (sv != 0.0) && cd > 0.0 && cd < 1.0;
}
__device__ __forceinline__ double pure_flux(double sv, double cl, double cu) {
  const double cd = (sv > 0.0) ? cl : cu;
  return (sv == 0.0) ? 0.0 : sv * cd;
}
// New value of a cell: eq. 3 in conservative split form with the c_c term.
__device__ __forceinline__ double swept(double c0, double flo, double fhi, double slo, double shi, double cc) {
  return (c0 - (fhi - flo)) + cc * (shi - slo);
}
__device__ __forceinline__ bool is_mixed(double c) { return c > 0.0 && c < 1.0; }

// g mapped into [0, n) periodically (g within a few periods of the box).
__device__ __forceinline__ int wrap_off(int g, int n) {
  if (g < 0) {
    g += n;
    if (g < 0) {
      g %= n;
      if (g < 0) g += n;
    }
  } else if (g >= n) {
    g -= n;
    if (g >= n) g %= n;
  }
  return g;
}
__device__ __forceinline__ int64_t cidx(int x, int y, int z, int nx, int ny) {
  return ((int64_t)z * ny + y) * nx + x;
}
// c_c of cell (x, y, z) from the bit array of one tracer, as 0.0 or 1.0.
__device__ __forceinline__ double cc_bit(const uint64_t *__restrict__ b, int x, int y, int z, int ny, int words) {
  const uint64_t w = b[((int64_t)z * ny + y) * words + (x >> 6)];
  return ((w >> (x & 63)) & 1ull) ? 1.0 : 0.0;
}
// Flat index of the upper neighbour along D of cell (x, y, z).
template <int D>
__device__ __forceinline__ int64_t upper(int x, int y, int z, int nx, int ny, int nz) {
  if (D == 0) return cidx(wrap_inc(x, nx), y, z, nx, ny);
  if (D == 1) return cidx(x, wrap_inc(y, ny), z, nx, ny);
  return cidx(x, y, wrap_inc(z, nz), nx, ny);
}

// Tracer and coordinates of a list entry (tracer * n3 + cell).
struct Entry {
  int t, i, j, k;
};
__device__ __forceinline__ Entry decode(uint32_t e, int nx, int ny, const Divisors &dv) {
  Entry r;
  const uint32_t t = fast_div(e, dv.n3);
  const uint32_t p32 = e - t * dv.n3.d;
  const uint32_t row = fast_div(p32, dv.nx);
  r.i = (int)(p32 - row * (uint32_t)nx);
  const uint32_t k32 = fast_div(row, dv.ny);
  r.j = (int)(row - k32 * (uint32_t)ny);
  r.k = (int)k32;
  r.t = (int)t;
  return r;
}

// Mixed cells of the fields and candidates of the first sweep (axis A, the
// first of a step: c_c = c > 0.5). Wavefront w scans tracer-cells
// [w*rsize, (w+1)*rsize).
template <int A>
__device__ __forceinline__ void scan_pair_body(const double *__restrict__ c, const double *__restrict__ sA,
                                               int64_t total, int nx, int ny, int nz, const Divisors &dv,
                                               uint32_t *__restrict__ listL, int *__restrict__ cntL,
                                               uint32_t *__restrict__ listC, int *__restrict__ cntC,
                                               int64_t nregions, int rsize, int64_t w) {
  const int lane = threadIdx.x & 63;
  if (w >= nregions) return;
  const int64_t n3 = (int64_t)nx * ny * nz;
  uint32_t *outL = listL + w * rsize;
  uint32_t *outC = listC + w * rsize;
  int nL = 0, nC = 0;
  const uint64_t below = (1ull << lane) - 1;
  const int64_t end = ((w + 1) * rsize < total) ? (w + 1) * rsize : total;
#pragma unroll 4
  for (int64_t base = w * rsize; base < end; base += 64) {
    const int64_t q = base + lane;
    bool mixed = false, cand = false;
    if (q < end) {
      const Entry e = decode((uint32_t)q, nx, ny, dv);
      const double *ct = c + (int64_t)e.t * n3;
      const int64_t p = cidx(e.i, e.j, e.k, nx, ny);
      const int64_t pu = upper<A>(e.i, e.j, e.k, nx, ny, nz);
      const int64_t pl = (A == 0) ? cidx(wrap_dec(e.i, nx), e.j, e.k, nx, ny)
                                  : ((A == 1) ? cidx(e.i, wrap_dec(e.j, ny), e.k, nx, ny)
                                              : cidx(e.i, e.j, wrap_dec(e.k, nz), nx, ny));
      const double c0 = ct[p], cl = ct[pl], cu = ct[pu];
      const double slo = sA[p], shi = sA[pu];
      mixed = is_mixed(c0);
      if (mixed_donor(slo, cl, c0) || mixed_donor(shi, c0, cu)) {
        cand = true;
      } else {
        const double cc = (c0 > 0.5) ? 1.0 : 0.0;
        cand = is_mixed(swept(c0, pure_flux(slo, cl, c0), pure_flux(shi, c0, cu), slo, shi, cc));
      }
    }
    const uint64_t mL = __ballot(mixed);
    if (mixed) outL[nL + __popcll(mL & below)] = (uint32_t)q;
    nL += __popcll(mL);
    const uint64_t mC = __ballot(cand);
    if (cand) outC[nC + __popcll(mC & below)] = (uint32_t)q;
    nC += __popcll(mC);
  }
  if (lane == 0) {
    cntL[w] = nL;
    cntC[w] = nC;
  }
}

// K2: candidates of F1 -> cells mixed in F1 that donate through a B-face.
// Region w of the candidate list is filtered into region w of `out`.
template <int A, int B>
__device__ __forceinline__ void cand_body(const double *__restrict__ cin, const double *__restrict__ sA,
                                          const double *__restrict__ sB, const double *__restrict__ fmA,
                                          const uint64_t *__restrict__ bits, int cc_from_field,
                                          const uint32_t *__restrict__ list, const int *__restrict__ counts,
                                          int64_t nregions, int rsize, uint32_t *__restrict__ out,
                                          int *__restrict__ out_counts, int nx, int ny, int nz, int words,
                                          const Divisors &dv, int64_t w) {
  const int lane = threadIdx.x & 63;
  if (w >= nregions) return;
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int64_t nbits = (int64_t)nz * ny * words;
  const int nq = counts[w];
  const uint32_t *reg = list + w * rsize;
  uint32_t *oreg = out + w * rsize;
  const uint64_t below = (1ull << lane) - 1;
  int n = 0;
  for (int q0 = 0; q0 < nq; q0 += 64) {
    const int q = q0 + lane;
    bool keep = false;
    uint32_t ent = 0;
    if (q < nq) {
      ent = reg[q];
      const Entry e = decode(ent, nx, ny, dv);
      const double *ct = cin + (int64_t)e.t * n3;
      const int64_t p = cidx(e.i, e.j, e.k, nx, ny);
      const int64_t pu = upper<A>(e.i, e.j, e.k, nx, ny, nz);
      const int64_t pl = (A == 0) ? cidx(wrap_dec(e.i, nx), e.j, e.k, nx, ny)
                                  : ((A == 1) ? cidx(e.i, wrap_dec(e.j, ny), e.k, nx, ny)
                                              : cidx(e.i, e.j, wrap_dec(e.k, nz), nx, ny));
      const double c0 = ct[p], cl = ct[pl], cu = ct[pu];
      const double slo = sA[p], shi = sA[pu];
      const double cc = cc_from_field ? ((c0 > 0.5) ? 1.0 : 0.0)
                                      : cc_bit(bits + (int64_t)e.t * nbits, e.i, e.j, e.k, ny, words);
      const double *fa = fmA + (int64_t)e.t * n3;
      const double f1 = swept(c0, face_flux(slo, cl, c0, fa, p), face_flux(shi, c0, cu, fa, pu), slo, shi, cc);
      if (is_mixed(f1)) {
        const int64_t pb = upper<B>(e.i, e.j, e.k, nx, ny, nz);
        keep = (sB[p] < 0.0) || (sB[pb] > 0.0);
      }
    }
    const uint64_t mask = __ballot(keep);
    if (keep) oreg[n + __popcll(mask & below)] = ent;
    n += __popcll(mask);
  }
  if (lane == 0) out_counts[w] = n;
}

// Index in a 3x3x3 block (x fastest) of the cell at offset o along A and
// transverse offsets (u, v) along the lower and the upper of the other axes.
template <int A>
__host__ __device__ constexpr int block_index(int o, int u, int v) {
  return (A == 0) ? (o + 1) + 3 * (u + 1) + 9 * (v + 1)
                  : ((A == 1) ? (u + 1) + 3 * (o + 1) + 9 * (v + 1) : (u + 1) + 3 * (v + 1) + 9 * (o + 1));
}
__device__ __forceinline__ int step_wrap(int c, int d, int n) {
  return (d < 0) ? wrap_dec(c, n) : ((d > 0) ? wrap_inc(c, n) : c);
}

// K3: PLIC of sweep B on F1 for the cells K2 kept. F1 on the 3x3x3 block
// comes from F0 on the block extended by 2 cells along A: on each of the 9
// lines along A, F0 at offsets -2..2, s_A on the faces -1..2 and c_c at
// -1..1 give F1 at -1, 0, 1. A wavefront takes its entries 64 at a time:
// first the (entry, line) items are spread over all lanes (independent
// gathers) and the values go to the wavefront's LDS slice `bl`
// (27 x 64 doubles, entry-minor), then each lane runs the PLIC of one entry
// on its block read back from LDS.
constexpr int kPlicPairSlice = 27 * 64;  // doubles of LDS per wavefront
template <int A, int B>
__device__ __forceinline__ void plic_b_body(const double *__restrict__ cin, const double *__restrict__ sA,
                                            const double *__restrict__ sB, const double *__restrict__ fmA,
                                            const uint64_t *__restrict__ bits, int cc_from_field,
                                            const uint32_t *__restrict__ list, const int *__restrict__ counts,
                                            int64_t nregions, int rsize, double *__restrict__ fmB, int nx, int ny,
                                            int nz, int words, const Divisors &dv, double *__restrict__ bl,
                                            int64_t w) {
  const int lane = threadIdx.x & 63;
  if (w >= nregions) return;
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int64_t nbits = (int64_t)nz * ny * words;
  const int nq = counts[w];
  const uint32_t *reg = list + w * rsize;
  constexpr int T1 = (A == 0) ? 1 : 0;  // lower transverse axis of A
  constexpr int T2 = (A == 2) ? 1 : 2;  // upper transverse axis of A
  const int n_[3] = {nx, ny, nz};
  for (int base = 0; base < nq; base += 64) {
    const int nb = (nq - base < 64) ? nq - base : 64;
    // ---- phase 1: F1 on the lines of the batch's blocks
#pragma unroll 3
    for (int x = lane; x < 9 * nb; x += 64) {
      const int eb = x / 9, l = x - 9 * eb;
      const Entry e = decode(reg[base + eb], nx, ny, dv);
      const int c_[3] = {e.i, e.j, e.k};
      const double *ct = cin + (int64_t)e.t * n3;
      const double *fa = fmA + (int64_t)e.t * n3;
      const uint64_t *bt = bits + (int64_t)e.t * nbits;
      const int u = l % 3 - 1, v = l / 3 - 1;
      int xyz[3];
      xyz[T1] = step_wrap(c_[T1], u, n_[T1]);
      xyz[T2] = step_wrap(c_[T2], v, n_[T2]);
      int P[5];
      P[2] = c_[A];
      P[1] = wrap_dec(P[2], n_[A]);
      P[0] = wrap_dec(P[1], n_[A]);
      P[3] = wrap_inc(P[2], n_[A]);
      P[4] = wrap_inc(P[3], n_[A]);
      double c5[5], s4[4];
      uint32_t idx[5];
#pragma unroll
      for (int o = 0; o < 5; ++o) {
        xyz[A] = P[o];
        idx[o] = ((uint32_t)xyz[2] * (uint32_t)ny + (uint32_t)xyz[1]) * (uint32_t)nx + (uint32_t)xyz[0];
        c5[o] = ct[idx[o]];
      }
#pragma unroll
      for (int o = 0; o < 4; ++o) s4[o] = sA[idx[o + 1]];
      // face f (f = 0..3) is the lower face of the cell at offset f - 1: its
      // mixed-donor flag, then all flux loads at once, then the three values
      bool dm[4];
      double fv[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) dm[f] = mixed_donor(s4[f], c5[f], c5[f + 1]);
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        fv[f] = 0.0;
        if (dm[f]) fv[f] = fa[idx[f + 1]];
      }
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        xyz[A] = P[o + 1];
        const double c0 = c5[o + 1];
        const double cc = cc_from_field ? ((c0 > 0.5) ? 1.0 : 0.0) : cc_bit(bt, xyz[0], xyz[1], xyz[2], ny, words);
        const double slo = s4[o], shi = s4[o + 1];
        const double flo = dm[o] ? fv[o] : pure_flux(slo, c5[o], c0);
        const double fhi = dm[o + 1] ? fv[o + 1] : pure_flux(shi, c0, c5[o + 2]);
        bl[block_index<A>(o - 1, u, v) * 64 + eb] = swept(c0, flo, fhi, slo, shi, cc);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // ---- phase 2: one entry per lane
    if (lane < nb) {
      double b[27];
#pragma unroll
      for (int k = 0; k < 27; ++k) b[k] = bl[k * 64 + lane];
      const Entry e = decode(reg[base + lane], nx, ny, dv);
      const int64_t p = cidx(e.i, e.j, e.k, nx, ny);
      const int64_t pb = upper<B>(e.i, e.j, e.k, nx, ny, nz);
      const double s_lo = sB[p], s_hi = sB[pb];
      double f_lo, f_hi;
      plic_fluxes<B>(b, s_lo, s_hi, f_lo, f_hi);
      double *ft = fmB + (int64_t)e.t * n3;
      if (s_lo < 0.0) ft[p] = f_lo;
      if (s_hi > 0.0) ft[pb] = f_hi;
    }
    // the next batch overwrites the slice
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// K4: F2 from F0 for one tracer on a 64 x kPairTY x kPairTZ brick (see the
// top of this file). Stages per plane j of the march (one barrier after
// each of the first three):
//   0  F0 at plane j on R0 (the tile grown by the halos of stages 1-3),
//   1  F1 at plane j - [A = z] on R1 (the tile grown for stages 2-3),
//   2  F2 at plane j1 - [B = z] on R2 (the tile grown by one cell along N),
//   3  at plane j2 - [N = z]: F2 stored, mixed cells and candidates listed,
//      c_c bits written.
// Ring slot of plane j: (j - jb) mod depth, jb the first plane loaded.
struct PairArgs {
  const double *cin;
  double *cout;
  const double *sA, *sB, *sN;
  const double *fmA, *fmB;
  const uint64_t *bits_rd;
  uint64_t *bits_wr;
  int phase;
  int ntr, nx, ny, nz, words, ntx, nty, nzc;
  uint32_t *listL;
  int *cntL;
  uint32_t *listC;
  int *cntC;
  int rsize;
};

template <int A, int B, int N>
__device__ __forceinline__ void pair_body(const PairArgs &a, int logical) {
  constexpr int TY = kPairTY;
  constexpr int h2x = (N == 0), h2y = (N == 1), hz2 = (N == 2);
  constexpr int h1x = h2x + (B == 0), h1y = h2y + (B == 1), hz1 = hz2 + (B == 2);
  constexpr int h0x = h1x + (A == 0), h0y = h1y + (A == 1), hz0 = hz1 + (A == 2);
  constexpr int W2 = 64 + 2 * h2x, H2 = TY + 2 * h2y, P2 = W2 * H2;
  constexpr int W1 = 64 + 2 * h1x, H1 = TY + 2 * h1y, P1 = W1 * H1;
  constexpr int W0 = 64 + 2 * h0x, H0 = TY + 2 * h0y, P0 = W0 * H0;
  constexpr int D0 = 1 + 2 * (A == 2), D1 = 1 + 2 * (B == 2), D2 = 1 + 2 * (N == 2);
  // in-plane offsets of the neighbours along A (in R0), B (in R1), N (in R2);
  // neighbours along z are in the adjacent ring slots instead
  constexpr int oA = (A == 0) ? 1 : ((A == 1) ? W0 : 0);
  constexpr int oB = (B == 0) ? 1 : ((B == 1) ? W1 : 0);
  constexpr int oN = (N == 0) ? 1 : ((N == 1) ? W2 : 0);
  __shared__ double f0[D0 * P0];
  __shared__ double f1[D1 * P1];
  __shared__ double f2[D2 * P2];
  __shared__ uint8_t ca[D1 * P1];  // c_c of sweep A on R1
  __shared__ uint8_t cb[D2 * P2];  // c_c of sweep B on R2

  // cells of each region per thread (q = tid + k * kPairThreads)
  constexpr int NQ0 = (P0 + kPairThreads - 1) / kPairThreads;
  constexpr int NQ1 = (P1 + kPairThreads - 1) / kPairThreads;
  constexpr int NQ2 = (P2 + kPairThreads - 1) / kPairThreads;
  constexpr int NQ3 = TY / 4;

  const int nx = a.nx, ny = a.ny, nz = a.nz, words = a.words;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int t = logical % a.ntr;
  int rest = logical / a.ntr;
  const int bx = rest % a.ntx;
  rest /= a.ntx;
  const int by = rest % a.nty;
  const int bz = rest / a.nty;
  const int x0 = bx * 64, y0 = by * TY, z0 = bz * kPairTZ;
  const int z1 = (z0 + kPairTZ < nz) ? z0 + kPairTZ : nz;
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int64_t nbits = (int64_t)nz * ny * words;
  const double *c_t = a.cin + t * n3;
  double *o_t = a.cout + t * n3;
  const double *fa = a.fmA + t * n3;
  const double *fb = a.fmB + t * n3;
  const uint64_t *br = a.bits_rd + t * nbits;
  uint64_t *bw = a.bits_wr + t * nbits;
  const int phase = a.phase;
  const int64_t wave = (int64_t)logical * 4 + wv;
  uint32_t *regL = a.listL + wave * a.rsize;
  uint32_t *regC = (N == kNoAxis) ? nullptr : a.listC + wave * a.rsize;
  int nL = 0, nC = 0;  // wavefront-uniform
  const uint64_t below = (1ull << lane) - 1;

  // In-plane offsets (y * nx + x, 32 bits: a tracer has fewer than 2^32
  // cells) of this thread's cells in R0, R1, R2 and the tile, and of their
  // upper neighbours along the stage's axis when that axis is in the plane;
  // they are the same on every plane of the march.
  const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
  uint32_t o0[NQ0], o1[NQ1], o1u[NQ1], o2[NQ2], o2u[NQ2], o3[NQ3], o3u[NQ3], w1[NQ1];
  int sh1[NQ1];
#pragma unroll
  for (int k = 0; k < NQ0; ++k) {
    const int q = tid + k * kPairThreads;
    const int ry = q / W0, rx = q - ry * W0;
    const int gx = wrap_off(x0 - h0x + rx, nx), gy = wrap_off(y0 - h0y + ry, ny);
    o0[k] = (uint32_t)gy * nx + gx;
  }
#pragma unroll
  for (int k = 0; k < NQ1; ++k) {
    const int q = tid + k * kPairThreads;
    const int ry = q / W1, rx = q - ry * W1;
    const int gx = wrap_off(x0 - h1x + rx, nx), gy = wrap_off(y0 - h1y + ry, ny);
    o1[k] = (uint32_t)gy * nx + gx;
    o1u[k] = (A == 0) ? (uint32_t)gy * nx + wrap_inc(gx, nx) : ((A == 1) ? (uint32_t)wrap_inc(gy, ny) * nx + gx : o1[k]);
    w1[k] = (uint32_t)gy * words + (gx >> 6);
    sh1[k] = gx & 63;
  }
#pragma unroll
  for (int k = 0; k < NQ2; ++k) {
    const int q = tid + k * kPairThreads;
    const int ry = q / W2, rx = q - ry * W2;
    const int gx = wrap_off(x0 - h2x + rx, nx), gy = wrap_off(y0 - h2y + ry, ny);
    o2[k] = (uint32_t)gy * nx + gx;
    o2u[k] = (B == 0) ? (uint32_t)gy * nx + wrap_inc(gx, nx) : ((B == 1) ? (uint32_t)wrap_inc(gy, ny) * nx + gx : o2[k]);
  }
#pragma unroll
  for (int it = 0; it < NQ3; ++it) {
    const int gx = (x0 + lane < nx) ? x0 + lane : nx - 1;
    const int gy0 = y0 + wv + 4 * it, gy = (gy0 < ny) ? gy0 : ny - 1;
    o3[it] = (uint32_t)gy * nx + gx;
    o3u[it] = (N == 0) ? (uint32_t)gy * nx + wrap_inc(gx, nx) : ((N == 1) ? (uint32_t)wrap_inc(gy, ny) * nx + gx : o3[it]);
  }
  // offset of plane j (periodic) and of the plane above it
  auto plane = [&](int j) -> uint32_t { return (uint32_t)wrap_off(j, nz) * nxy; };
  auto plane_up = [&](int j) -> uint32_t { return (uint32_t)wrap_inc(wrap_off(j, nz), nz) * nxy; };
  const uint32_t nwy = (uint32_t)ny * (uint32_t)words;

  // Every load that does not depend on computed values is issued one plane
  // ahead, into registers that the stage using it consumes: F0 (stage 0),
  // s_A and the c_c word (stage 1), s_B (stage 2), s_N (stage 3). Planes
  // outside the box wrap; loads for planes that no stage uses are harmless.
  double r0[NQ0], rA[NQ1][2], rB[NQ2][2], rN[NQ3][2];
  uint64_t rW[NQ1];
  auto load0 = [&](int j) {
    const uint32_t pz = plane(j);
#pragma unroll
    for (int k = 0; k < NQ0; ++k)
      if (tid + k * kPairThreads < P0) r0[k] = c_t[pz + o0[k]];
  };
  auto load1 = [&](int j1) {
    const uint32_t pz = plane(j1), pzu = (A == 2) ? plane_up(j1) : pz;
    const uint32_t bz_ = (uint32_t)wrap_off(j1, nz) * nwy;
#pragma unroll
    for (int k = 0; k < NQ1; ++k)
      if (tid + k * kPairThreads < P1) {
        rA[k][0] = a.sA[pz + o1[k]];
        rA[k][1] = a.sA[pzu + o1u[k]];
        if (phase != 0) rW[k] = br[bz_ + w1[k]];
      }
  };
  auto load2 = [&](int j2) {
    const uint32_t pz = plane(j2), pzu = (B == 2) ? plane_up(j2) : pz;
#pragma unroll
    for (int k = 0; k < NQ2; ++k)
      if (tid + k * kPairThreads < P2) {
        rB[k][0] = a.sB[pz + o2[k]];
        rB[k][1] = a.sB[pzu + o2u[k]];
      }
  };
  auto load3 = [&](int j3) {
    if (N == kNoAxis) return;
    const uint32_t pz = plane(j3), pzu = (N == 2) ? plane_up(j3) : pz;
#pragma unroll
    for (int it = 0; it < NQ3; ++it) {
      rN[it][0] = a.sN[pz + o3[it]];
      rN[it][1] = a.sN[pzu + o3u[it]];
    }
  };

  const int jb = z0 - hz0;
  load0(jb);
  load1(jb - (A == 2));
  load2(jb - (A == 2) - (B == 2));
  load3(jb - hz0);
  for (int j = jb; j < z1 + hz0; ++j) {
    // ---- stage 0: F0 on R0 at plane j
    {
      double *dst = f0 + ((j - jb) % D0) * P0;
#pragma unroll
      for (int k = 0; k < NQ0; ++k) {
        const int q = tid + k * kPairThreads;
        if (q < P0) dst[q] = r0[k];
      }
      load0(j + 1);
    }
    __syncthreads();
    // ---- stage 1: F1 on R1 at plane j1
    const int j1 = j - (A == 2);
    if (j1 >= z0 - hz1 && j1 < z1 + hz1) {
      const uint32_t pz = plane(j1), pzu = (A == 2) ? plane_up(j1) : pz;
      const int s1 = (j1 - jb) % D1;
      const double *src = f0 + ((j1 - jb) % D0) * P0;
      const double *srcl = (A == 2) ? f0 + ((j1 - 1 - jb) % D0) * P0 : src;
      const double *srcu = (A == 2) ? f0 + ((j1 + 1 - jb) % D0) * P0 : src;
      // mixed donors first, then all their flux loads at once, then the values
      bool dl[NQ1], dh[NQ1];
      double fl[NQ1], fh[NQ1];
#pragma unroll
      for (int k = 0; k < NQ1; ++k) {
        const int q = tid + k * kPairThreads;
        dl[k] = dh[k] = false;
        if (q < P1) {
          const int ry = q / W1, rx = q - ry * W1;
          const int i0 = (ry + (A == 1)) * W0 + rx + (A == 0);
          const double c0 = src[i0], cl = srcl[i0 - oA], cu = srcu[i0 + oA];
          dl[k] = mixed_donor(rA[k][0], cl, c0);
          dh[k] = mixed_donor(rA[k][1], c0, cu);
        }
      }
#pragma unroll
      for (int k = 0; k < NQ1; ++k) {
        fl[k] = 0.0;
        fh[k] = 0.0;
        if (dl[k]) fl[k] = fa[pz + o1[k]];
        if (dh[k]) fh[k] = fa[pzu + o1u[k]];
      }
#pragma unroll
      for (int k = 0; k < NQ1; ++k) {
        const int q = tid + k * kPairThreads;
        if (q < P1) {
          const int ry = q / W1, rx = q - ry * W1;
          const int i0 = (ry + (A == 1)) * W0 + rx + (A == 0);
          const double c0 = src[i0], cl = srcl[i0 - oA], cu = srcu[i0 + oA];
          const double slo = rA[k][0], shi = rA[k][1];
          const double cc = (phase == 0) ? ((c0 > 0.5) ? 1.0 : 0.0) : (((rW[k] >> sh1[k]) & 1ull) ? 1.0 : 0.0);
          const double flo = dl[k] ? fl[k] : pure_flux(slo, cl, c0);
          const double fhi = dh[k] ? fh[k] : pure_flux(shi, c0, cu);
          f1[s1 * P1 + q] = swept(c0, flo, fhi, slo, shi, cc);
          ca[s1 * P1 + q] = (cc != 0.0);
        }
      }
    }
    load1(j1 + 1);
    __syncthreads();
    // ---- stage 2: F2 on R2 at plane j2
    const int j2 = j1 - (B == 2);
    if (j2 >= z0 - hz2 && j2 < z1 + hz2) {
      const uint32_t pz = plane(j2), pzu = (B == 2) ? plane_up(j2) : pz;
      const int s2 = (j2 - jb) % D2;
      const int s1 = (j2 - jb) % D1;
      const double *src = f1 + s1 * P1;
      const double *srcl = (B == 2) ? f1 + ((j2 - 1 - jb) % D1) * P1 : src;
      const double *srcu = (B == 2) ? f1 + ((j2 + 1 - jb) % D1) * P1 : src;
      bool dl[NQ2], dh[NQ2];
      double fl[NQ2], fh[NQ2];
#pragma unroll
      for (int k = 0; k < NQ2; ++k) {
        const int q = tid + k * kPairThreads;
        dl[k] = dh[k] = false;
        if (q < P2) {
          const int ry = q / W2, rx = q - ry * W2;
          const int i1 = (ry + (B == 1)) * W1 + rx + (B == 0);
          const double c0 = src[i1], cl = srcl[i1 - oB], cu = srcu[i1 + oB];
          dl[k] = mixed_donor(rB[k][0], cl, c0);
          dh[k] = mixed_donor(rB[k][1], c0, cu);
        }
      }
#pragma unroll
      for (int k = 0; k < NQ2; ++k) {
        fl[k] = 0.0;
        fh[k] = 0.0;
        if (dl[k]) fl[k] = fb[pz + o2[k]];
        if (dh[k]) fh[k] = fb[pzu + o2u[k]];
      }
#pragma unroll
      for (int k = 0; k < NQ2; ++k) {
        const int q = tid + k * kPairThreads;
        if (q < P2) {
          const int ry = q / W2, rx = q - ry * W2;
          const int i1 = (ry + (B == 1)) * W1 + rx + (B == 0);
          const double c0 = src[i1], cl = srcl[i1 - oB], cu = srcu[i1 + oB];
          const double slo = rB[k][0], shi = rB[k][1];
          const bool ccb = (phase == 2) ? (c0 > 0.5) : (ca[s1 * P1 + i1] != 0);
          const double cc = ccb ? 1.0 : 0.0;
          const double flo = dl[k] ? fl[k] : pure_flux(slo, cl, c0);
          const double fhi = dh[k] ? fh[k] : pure_flux(shi, c0, cu);
          f2[s2 * P2 + q] = swept(c0, flo, fhi, slo, shi, cc);
          cb[s2 * P2 + q] = ccb;
        }
      }
    }
    load2(j2 + 1);
    __syncthreads();
    // ---- stage 3: outputs at plane j3 (inside the box: no wrap)
    const int j3 = j2 - (N == 2);
    if (j3 >= z0 && j3 < z1) {
      const uint32_t pz = (uint32_t)j3 * nxy;
      const int s2 = (j3 - jb) % D2;
      const double *src = f2 + s2 * P2;
      const double *srcl = (N == 2) ? f2 + ((j3 - 1 - jb) % D2) * P2 : src;
      const double *srcu = (N == 2) ? f2 + ((j3 + 1 - jb) % D2) * P2 : src;
#pragma unroll
      for (int it = 0; it < NQ3; ++it) {
        const int iy = wv + 4 * it;
        const int gy = y0 + iy;
        const bool live = (x0 + lane < nx) && gy < ny;
        const int i2 = (iy + h2y) * W2 + lane + h2x;
        const double c2 = src[i2];
        const bool ccb = cb[s2 * P2 + i2] != 0;
        const uint32_t p = pz + o3[it];
        if (live) o_t[p] = c2;
        const bool mixed = live && is_mixed(c2);
        const uint64_t mL = __ballot(mixed);
        if (mixed) regL[nL + __popcll(mL & below)] = (uint32_t)(t * n3) + p;
        nL += __popcll(mL);
        if (phase != 1) {
          const uint64_t word = __ballot(live && ccb);
          if (lane == 0 && gy < ny) bw[(uint32_t)j3 * nwy + (uint32_t)gy * words + bx] = word;
        }
        if (N != kNoAxis) {
          bool cand = false;
          if (live) {
            const double cl = srcl[i2 - oN], cu = srcu[i2 + oN];
            const double slo = rN[it][0], shi = rN[it][1];
            if (mixed_donor(slo, cl, c2) || mixed_donor(shi, c2, cu)) {
              cand = true;
            } else {
              const double cc = (phase == 1) ? ((c2 > 0.5) ? 1.0 : 0.0) : (ccb ? 1.0 : 0.0);
              cand = is_mixed(swept(c2, pure_flux(slo, cl, c2), pure_flux(shi, c2, cu), slo, shi, cc));
            }
          }
          const uint64_t mC = __ballot(cand);
          if (cand) regC[nC + __popcll(mC & below)] = (uint32_t)(t * n3) + p;
          nC += __popcll(mC);
        }
      }
    }
    load3(j3 + 1);
  }
  if (lane == 0) {
    a.cntL[wave] = nL;
    if (N != kNoAxis) a.cntC[wave] = nC;
  }
}

// Block index -> logical brick. Workgroups are dealt to the 8 XCDs in turn;
// this numbering gives each XCD a contiguous run of logical bricks, so the
// tracers of one tile (consecutive numbers) and neighbouring tiles share an
// L2 for the face velocities and the halos.
__device__ __forceinline__ int xcd_logical(int b, int nb) {
  const int xcd = b & 7, k = b >> 3, q = nb >> 3, r = nb & 7;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

// ---------------------------------------------------------------- host side

// Bricks (workgroups) of a paired pass.
static inline int64_t pair_blocks(int nx, int ny, int nz, int ntr) {
  return (int64_t)ntr * ((nx + 63) / 64) * ((ny + kPairTY - 1) / kPairTY) * ((nz + kPairTZ - 1) / kPairTZ);
}

}  // namespace advect
