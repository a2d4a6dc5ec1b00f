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
__device__ __forceinline__ void hf_cell(const double *__restrict__ c, int64_t p, int nx, int ny, int nz,
                                        double &kappa_out, uint8_t &status_out) {
  const int n[3] = {nx, ny, nz};
  const int x[3] = {(int)(p % nx), (int)((p / nx) % ny), (int)(p / ((int64_t)nx * ny))};
  double b[27];
  for (int az = -1; az <= 1; ++az)
    for (int ay = -1; ay <= 1; ++ay)
      for (int ax = -1; ax <= 1; ++ax)
        b[(ax + 1) + 3 * (ay + 1) + 9 * (az + 1)] =
            c[((int64_t)wrap_any(x[2] + az, nz) * ny + wrap_any(x[1] + ay, ny)) * nx + wrap_any(x[0] + ax, nx)];
  double m[3];
  plic::myc_normal(b, m[0], m[1], m[2]);
  int order[3] = {0, 1, 2};
  for (int a = 0; a < 3; ++a)
    for (int bb = a + 1; bb < 3; ++bb)
      if (fabs(m[order[bb]]) > fabs(m[order[a]]) ||
          (fabs(m[order[bb]]) == fabs(m[order[a]]) && order[bb] < order[a])) {
        int t = order[a];
        order[a] = order[bb];
        order[bb] = t;
      }
  double result = __builtin_nan("");
  uint8_t st = 4;
  for (int at = 0; at < 3; ++at) {
    const int d = order[at];
    const int t1 = (d == 0) ? 1 : 0;
    const int t2 = (d == 2) ? 1 : 2;
    const bool up = m[d] >= 0.0;
    double H[3][3];
    bool ok = true;
    for (int v = -1; v <= 1 && ok; ++v)
      for (int u = -1; u <= 1 && ok; ++u) {
        int y[3] = {x[0], x[1], x[2]};
        y[t1] = wrap_any(y[t1] + u, n[t1]);
        y[t2] = wrap_any(y[t2] + v, n[t2]);
        double h = 0.0, first = 0.0, last = 0.0;
        for (int e = -3; e <= 3; ++e) {
          int z[3] = {y[0], y[1], y[2]};
          z[d] = wrap_any(z[d] + e, n[d]);
          const double v_ = c[((int64_t)z[2] * ny + z[1]) * nx + z[0]];
          if (e == -3) first = v_;
          if (e == 3) last = v_;
          h += v_;
        }
        const double full_end = up ? first : last;
        const double empty_end = up ? last : first;
        if (!(full_end >= 1.0 - 1e-6 && empty_end <= 1e-6)) ok = false;
        H[u + 1][v + 1] = h;
      }
    if (!ok) continue;
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
  kappa_out = result;
  status_out = st;
}

}  // namespace curv
