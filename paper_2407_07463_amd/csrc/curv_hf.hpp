// Height-function curvature of one mixed cell (device function shared by the
// full-grid and the list launches).
//
// The paper computes the curvature kappa_i of each tracer "as for a single
// tracer" (section "The no-coalescence.h algorithm", citing Popinet's review
// of surface-tension methods). Reading: fixed 7-cell height columns
// (Cummins, Francois & Kothe 2005). For every mixed cell (0 < c < 1): the MYC
// normal m orders the candidate column axes by decreasing |m_d| (ties to the
// lower axis); an axis is usable when each of the 3x3 columns has its end on
// the phase side (-sign(m_d), sign(0) = +1) full (c >= 1 - 1e-6) and its
// other end empty (c <= 1e-6); the column sums H(u, v), offsets -3..3, with
// (u, v) along the transverse axes in increasing order give
//   kappa*Delta = -[Hxx(1+Hy^2) + Hyy(1+Hx^2) - 2 Hxy Hx Hy] / (1+Hx^2+Hy^2)^{3/2},
// +2/R on a sphere of radius R cells. Every expression is evaluated in the
// written order.
#pragma once

#include "common.hpp"
#include "plic.hpp"

namespace curv {

// i + k for |k| <= 3, taken periodically into [0, n): one conditional add
// for n >= 3, the general rule below that.
__device__ __forceinline__ int wrap3(int i, int n) {
  if (n < 3) return wrap_any(i, n);
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

// kappa*Delta and the status (1..3 valid on the 1st..3rd axis tried, 4 no
// valid axis) of the mixed cell p (below 2^31) of c.
// Coordinates and axis choices are kept in scalars (no arrays indexed at run
// time), so the function stays in registers. The three middle cells of every
// column come from the 3x3x3 block; the other 36 cells of an axis are loaded
// at once, then the columns are checked.
__device__ __forceinline__ void hf_cell(const double *__restrict__ c, int64_t p, int nx, int ny, int nz,
                                        double &kappa_out, uint8_t &status_out) {
  const uint32_t row = (uint32_t)p / (uint32_t)nx;
  const int x0 = (int)((uint32_t)p - row * (uint32_t)nx);
  const int x2 = (int)(row / (uint32_t)ny);
  const int x1 = (int)(row - (uint32_t)x2 * (uint32_t)ny);
  double b[27];
  {
    const int xs[3] = {wrap_dec(x0, nx), x0, wrap_inc(x0, nx)};
    const int ys[3] = {wrap_dec(x1, ny), x1, wrap_inc(x1, ny)};
    const int zs[3] = {wrap_dec(x2, nz), x2, wrap_inc(x2, nz)};
#pragma unroll
    for (int az = 0; az < 3; ++az)
#pragma unroll
      for (int ay = 0; ay < 3; ++ay)
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) b[ax + 3 * ay + 9 * az] = c[(int64_t)(zs[az] * ny + ys[ay]) * nx + xs[ax]];
  }
  double m0, m1, m2;
  plic::myc_normal(b, m0, m1, m2);
  auto mv = [&](int a) { return a == 0 ? m0 : (a == 1 ? m1 : m2); };
  // axes by decreasing |m_d|, ties to the lower axis
  int o0 = 0, o1 = 1, o2 = 2;
  auto order2 = [&](int &a, int &bb) {
    if (fabs(mv(bb)) > fabs(mv(a)) || (fabs(mv(bb)) == fabs(mv(a)) && bb < a)) {
      const int t = a;
      a = bb;
      bb = t;
    }
  };
  order2(o0, o1);
  order2(o0, o2);
  order2(o1, o2);
  double result = __builtin_nan("");
  uint8_t st = 4;
#pragma unroll 1
  for (int at = 0; at < 3; ++at) {
    const int d = (at == 0) ? o0 : ((at == 1) ? o1 : o2);
    const int t1 = (d == 0) ? 1 : 0;
    const int t2 = (d == 2) ? 1 : 2;
    const bool up = mv(d) >= 0.0;
    // the cell's coordinates along d, t1, t2 and the strides of those axes
    auto coord = [&](int a) { return a == 0 ? x0 : (a == 1 ? x1 : x2); };
    auto extent = [&](int a) { return a == 0 ? nx : (a == 1 ? ny : nz); };
    auto stride = [&](int a) { return a == 0 ? (int64_t)1 : (a == 1 ? (int64_t)nx : (int64_t)nx * ny); };
    const int cd = coord(d), ed = extent(d);
    const int64_t sd = stride(d), s1 = stride(t1), s2 = stride(t2);
    const int c1 = coord(t1), e1 = extent(t1), c2 = coord(t2), e2 = extent(t2);
    // rows of the columns along d at offsets -3, -2, 2, 3 (the middle three are in b)
    const int64_t r_m3 = (int64_t)wrap3(cd - 3, ed) * sd, r_m2 = (int64_t)wrap3(cd - 2, ed) * sd;
    const int64_t r_p2 = (int64_t)wrap3(cd + 2, ed) * sd, r_p3 = (int64_t)wrap3(cd + 3, ed) * sd;
    double H[3][3];
    bool ok = true;
#pragma unroll
    for (int v = -1; v <= 1; ++v)
#pragma unroll
      for (int u = -1; u <= 1; ++u) {
        const int64_t base = (int64_t)wrap3(c1 + u, e1) * s1 + (int64_t)wrap3(c2 + v, e2) * s2;
        const double vm3 = c[base + r_m3], vm2 = c[base + r_m2], vp2 = c[base + r_p2], vp3 = c[base + r_p3];
        // block entry at offset e along d, u along t1, v along t2
        auto mid = [&](int e) {
          const double a0 = b[(e + 1) + 3 * (u + 1) + 9 * (v + 1)];  // d = 0: t1 = y, t2 = z
          const double a1 = b[(u + 1) + 3 * (e + 1) + 9 * (v + 1)];  // d = 1: t1 = x, t2 = z
          const double a2 = b[(u + 1) + 3 * (v + 1) + 9 * (e + 1)];  // d = 2: t1 = x, t2 = y
          return d == 0 ? a0 : (d == 1 ? a1 : a2);
        };
        double h = 0.0;
        h += vm3;
        h += vm2;
        h += mid(-1);
        h += mid(0);
        h += mid(1);
        h += vp2;
        h += vp3;
        const double full_end = up ? vm3 : vp3;
        const double empty_end = up ? vp3 : vm3;
        ok = ok && (full_end >= 1.0 - 1e-6 && empty_end <= 1e-6);
        H[u + 1][v + 1] = h;
      }
    if (ok) {
      const double Hx = (H[2][1] - H[0][1]) / 2.0;
      const double Hy = (H[1][2] - H[1][0]) / 2.0;
      const double Hxx = (H[2][1] - 2.0 * H[1][1]) + H[0][1];
      const double Hyy = (H[1][2] - 2.0 * H[1][1]) + H[1][0];
      const double Hxy = (((H[2][2] - H[2][0]) - H[0][2]) + H[0][0]) / 4.0;
      const double num = (Hxx * (1.0 + Hy * Hy) + Hyy * (1.0 + Hx * Hx)) - ((2.0 * Hxy) * Hx) * Hy;
      const double den = (1.0 + Hx * Hx) + Hy * Hy;
      result = -num / (den * sqrt(den));
      st = (uint8_t)(1 + at);
      break;
    }
  }
  kappa_out = result;
  status_out = st;
}

}  // namespace curv
