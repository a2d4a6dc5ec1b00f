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

// kappa*Delta and the status (1..3 valid on the 1st..3rd axis tried, 4 no
// valid axis) of the mixed cell p of c.
// Coordinates and axis choices are kept in scalars (no arrays indexed at run
// time), so the function stays in registers.
__device__ __forceinline__ void hf_cell(const double *__restrict__ c, int64_t p, int nx, int ny, int nz,
                                        double &kappa_out, uint8_t &status_out) {
  const int x0 = (int)(p % nx), x1 = (int)((p / nx) % ny), x2 = (int)(p / ((int64_t)nx * ny));
  double b[27];
#pragma unroll
  for (int az = -1; az <= 1; ++az)
#pragma unroll
    for (int ay = -1; ay <= 1; ++ay)
#pragma unroll
      for (int ax = -1; ax <= 1; ++ax)
        b[(ax + 1) + 3 * (ay + 1) + 9 * (az + 1)] =
            c[((int64_t)wrap_any(x2 + az, nz) * ny + wrap_any(x1 + ay, ny)) * nx + wrap_any(x0 + ax, nx)];
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
  bool done = false;
#pragma unroll 1
  for (int at = 0; at < 3 && !done; ++at) {
    const int d = (at == 0) ? o0 : ((at == 1) ? o1 : o2);
    const int t1 = (d == 0) ? 1 : 0;
    const int t2 = (d == 2) ? 1 : 2;
    const bool up = mv(d) >= 0.0;
    double H[3][3];
    bool ok = true;
#pragma unroll
    for (int v = -1; v <= 1; ++v)
#pragma unroll
      for (int u = -1; u <= 1; ++u) {
        double h = 0.0, first = 0.0, last = 0.0;
        if (ok) {
          // column through the cell offset by u along t1 and v along t2
          const int y0 = wrap_any(x0 + (t1 == 0 ? u : 0) + (t2 == 0 ? v : 0), nx);
          const int y1 = wrap_any(x1 + (t1 == 1 ? u : 0) + (t2 == 1 ? v : 0), ny);
          const int y2 = wrap_any(x2 + (t1 == 2 ? u : 0) + (t2 == 2 ? v : 0), nz);
          for (int e = -3; e <= 3; ++e) {
            const int z0 = (d == 0) ? wrap_any(y0 + e, nx) : y0;
            const int z1 = (d == 1) ? wrap_any(y1 + e, ny) : y1;
            const int z2 = (d == 2) ? wrap_any(y2 + e, nz) : y2;
            const double v_ = c[((int64_t)z2 * ny + z1) * nx + z0];
            if (e == -3) first = v_;
            if (e == 3) last = v_;
            h += v_;
          }
          const double full_end = up ? first : last;
          const double empty_end = up ? last : first;
          if (!(full_end >= 1.0 - 1e-6 && empty_end <= 1e-6)) ok = false;
        }
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
      done = true;
    }
  }
  kappa_out = result;
  status_out = st;
}

}  // namespace curv
