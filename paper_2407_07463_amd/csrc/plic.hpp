// Device-side PLIC geometry: plane/unit-cube volume, its inverse and the
// Mixed-Youngs-Centred normal. The paper names geometric PLIC VoF (section
// "Numerical method") without its discrete form; these follow Scardovelli &
// Zaleski (2000) for the volume and Aulisa et al. (2007) for the normal.
//
// Every expression is evaluated in the written order (the library is built
// with -ffp-contract=off): the volume function and the normal are therefore
// the same floating-point functions of their inputs as any other
// implementation that writes the same formulas in the same order.
#pragma once

#include <hip/hip_runtime.h>

namespace plic {

// Volume of {x in [0,1]^3 : m.x <= alpha}. Negative components are reflected
// (x_i -> 1 - x_i) in x, y, z order; the symmetric half alpha > M/2 maps to
// 1 - V(M - alpha); the sorted components m1 <= m2 <= m3 select one of five
// closed forms (inclusion-exclusion over the cube's vertices, rearranged so
// that no case divides by a component that can vanish).
__device__ __forceinline__ double volume_sorted_half(double m1, double m2, double m3, double alpha) {
  // requires 0 < alpha <= M/2 and 0 <= m1 <= m2 <= m3
  if (alpha < m1) return alpha * alpha * alpha / (6.0 * m1 * m2 * m3);
  double base = 3.0 * alpha * alpha - 3.0 * alpha * m1 + m1 * m1;
  if (alpha < m2) return base / (6.0 * m2 * m3);
  if (alpha < fmin(m3, m1 + m2)) {
    double u = alpha - m2;
    double corr = (u == 0.0) ? 0.0 : u * u * u / m1;
    return (base - corr) / (6.0 * m2 * m3);
  }
  if (m3 <= m1 + m2) {
    double u2 = alpha - m2, u3 = alpha - m3;
    double num = u2 * u2 * u2 + u3 * u3 * u3;
    double corr = (num == 0.0) ? 0.0 : num / m1;
    return (base - corr) / (6.0 * m2 * m3);
  }
  return (alpha - (m1 + m2) / 2.0) / m3;
}

__device__ __forceinline__ void sort3(double &a, double &b, double &c) {
  double t;
  if (a > b) { t = a; a = b; b = t; }
  if (b > c) { t = b; b = c; c = t; }
  if (a > b) { t = a; a = b; b = t; }
}

__device__ __forceinline__ double volume(double mx, double my, double mz, double alpha) {
  if (mx < 0.0) { alpha = alpha - mx; mx = -mx; }
  if (my < 0.0) { alpha = alpha - my; my = -my; }
  if (mz < 0.0) { alpha = alpha - mz; mz = -mz; }
  double M = (mx + my) + mz;
  if (alpha <= 0.0) return 0.0;
  if (alpha >= M) return 1.0;
  bool flip = 2.0 * alpha > M;
  if (flip) {
    alpha = M - alpha;
    // the reflected problem: all components already non-negative
    if (alpha <= 0.0) return 1.0;
    if (alpha >= M) return 0.0;
  }
  double m1 = mx, m2 = my, m3 = mz;
  sort3(m1, m2, m3);
  double v = volume_sorted_half(m1, m2, m3, alpha);
  return flip ? 1.0 - v : v;
}

// Volume and derivative dV/dalpha on the sorted half range, for Newton steps.
__device__ __forceinline__ void volume_deriv_sorted(double m1, double m2, double m3, double a, double &V, double &dV) {
  double den = 6.0 * m2 * m3;
  if (a < m1) {
    double d3 = 6.0 * m1 * m2 * m3;
    V = a * a * a / d3;
    dV = 3.0 * a * a / d3;
    return;
  }
  double base = 3.0 * a * a - 3.0 * a * m1 + m1 * m1;
  double dbase = 6.0 * a - 3.0 * m1;
  if (a < m2) {
    V = base / den;
    dV = dbase / den;
    return;
  }
  if (a < fmin(m3, m1 + m2)) {
    double u = a - m2;
    V = (base - u * u * u / m1) / den;
    dV = (dbase - 3.0 * u * u / m1) / den;
    return;
  }
  if (m3 <= m1 + m2) {
    double u2 = a - m2, u3 = a - m3;
    V = (base - (u2 * u2 * u2 + u3 * u3 * u3) / m1) / den;
    dV = (dbase - 3.0 * (u2 * u2 + u3 * u3) / m1) / den;
    return;
  }
  V = (a - (m1 + m2) / 2.0) / m3;
  dV = 1.0 / m3;
}

// Plane constant alpha with volume(m, alpha) = c for 0 < c < 1.
// The half range c <= 1/2 is solved on the sorted, reflected normal: closed
// forms where V is a monomial or quadratic in alpha (corner, prism and
// parallel cases), safeguarded Newton iteration in the two cubic cases, then
// Newton polishing to the last bits. The result is mapped back through the
// symmetry and the reflections.
__device__ __forceinline__ double alpha_of(double mx, double my, double mz, double c) {
  double neg = 0.0;
  if (mx < 0.0) neg += mx;
  if (my < 0.0) neg += my;
  if (mz < 0.0) neg += mz;
  double m1 = fabs(mx), m2 = fabs(my), m3 = fabs(mz);
  sort3(m1, m2, m3);
  double M = (m1 + m2) + m3;
  bool flip = c > 0.5;
  double v = flip ? 1.0 - c : c;
  double a;
  double v1 = (m1 > 0.0) ? m1 * m1 / (6.0 * m2 * m3) : 0.0;
  double v2 = (m2 > 0.0) ? (3.0 * m2 * m2 - 3.0 * m2 * m1 + m1 * m1) / (6.0 * m2 * m3) : 0.0;
  double m12 = m1 + m2;
  if (v < v1) {
    a = cbrt(6.0 * m1 * m2 * m3 * v);
  } else if (v < v2) {
    a = 0.5 * m1 + sqrt(fmax(2.0 * m2 * m3 * v - m1 * m1 / 12.0, 0.0));
  } else if (m3 >= m12 && v >= m12 / (2.0 * m3)) {
    a = v * m3 + 0.5 * m12;
  } else {
    // cubic cases: alpha in [m2, M/2]; start from the chord between the
    // bracket ends (V(m2) = v2, V(M/2) = 1/2) and take safeguarded Newton
    // steps; V is convex-concave here, so a few steps reach the last bits
    double lo = m2, hi = 0.5 * M;
    a = lo + (hi - lo) * ((v - v2) / (0.5 - v2));
    for (int it = 0; it < 12; ++it) {
      double V, dV;
      volume_deriv_sorted(m1, m2, m3, a, V, dV);
      double f = V - v;
      if (f < 0.0) lo = a;
      else hi = a;
      double an = (dV > 0.0) ? a - f / dV : 0.5 * (lo + hi);
      if (!(an >= lo && an <= hi)) an = 0.5 * (lo + hi);
      const double step = fabs(an - a);
      a = an;
      if (step <= 4e-16 * a) break;
    }
  }
  // one Newton polish step (the closed forms lose a few bits near case ends)
  {
    double V, dV;
    volume_deriv_sorted(m1, m2, m3, a, V, dV);
    if (dV > 0.0) {
      double an = a - (V - v) / dV;
      if (an >= 0.0 && an <= 0.5 * M) a = an;
    }
  }
  if (flip) a = M - a;
  return a + neg;
}

// Mixed-Youngs-Centred normal of the centre of a 3x3x3 block
// b[(ax+1) + 3(ay+1) + 9(az+1)]: outward (pointing away from the phase),
// L1-normalised. Centred-columns candidates: for each column axis d, column
// sums H over the 3 cells along d, orientation from the two end layers, the
// centred slopes g of H along the two transverse axes (in increasing axis
// order), candidate (sigma, -g1, -g2)/(|g1|+|g2|+1) of quality 1/(|g1|+|g2|+1);
// the best quality wins (ties to the lower axis). Youngs: weighted central
// differences (weights 1,2,1) of the block. The centred-columns candidate is
// kept unless Youngs is defined and its largest component is strictly
// smaller than the centred-columns quality. All sums run in increasing
// stencil index.
__device__ __forceinline__ void myc_normal(const double *b, double &nx_, double &ny_, double &nz_) {
#define B(ax, ay, az) b[((ax) + 1) + 3 * ((ay) + 1) + 9 * ((az) + 1)]
  double cs[3][3];
  double q[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double H[3][3];
    double slo = 0.0, shi = 0.0;
#pragma unroll
    for (int v = -1; v <= 1; ++v)
#pragma unroll
      for (int u = -1; u <= 1; ++u) {
        double e0, e1, e2;
        if (d == 0) { e0 = B(-1, u, v); e1 = B(0, u, v); e2 = B(1, u, v); }
        else if (d == 1) { e0 = B(u, -1, v); e1 = B(u, 0, v); e2 = B(u, 1, v); }
        else { e0 = B(u, v, -1); e1 = B(u, v, 0); e2 = B(u, v, 1); }
        H[u + 1][v + 1] = (e0 + e1) + e2;
        slo += e0;
        shi += e2;
      }
    double sigma = (slo >= shi) ? 1.0 : -1.0;
    double g1 = (H[2][1] - H[0][1]) / 2.0;
    double g2 = (H[1][2] - H[1][0]) / 2.0;
    double D = (fabs(g1) + fabs(g2)) + 1.0;
    double nd = sigma / D, n1 = -g1 / D, n2 = -g2 / D;
    if (d == 0) { cs[d][0] = nd; cs[d][1] = n1; cs[d][2] = n2; }
    else if (d == 1) { cs[d][1] = nd; cs[d][0] = n1; cs[d][2] = n2; }
    else { cs[d][2] = nd; cs[d][0] = n1; cs[d][1] = n2; }
    q[d] = 1.0 / D;
  }
  int ds = 0;
  if (q[1] > q[ds]) ds = 1;
  if (q[2] > q[ds]) ds = 2;
  double Gx = 0.0, Gy = 0.0, Gz = 0.0;
  const double w[3] = {1.0, 2.0, 1.0};
#pragma unroll
  for (int az = -1; az <= 1; ++az)
#pragma unroll
    for (int ay = -1; ay <= 1; ++ay) Gx += (w[ay + 1] * w[az + 1]) * (B(1, ay, az) - B(-1, ay, az));
#pragma unroll
  for (int az = -1; az <= 1; ++az)
#pragma unroll
    for (int ax = -1; ax <= 1; ++ax) Gy += (w[ax + 1] * w[az + 1]) * (B(ax, 1, az) - B(ax, -1, az));
#pragma unroll
  for (int ay = -1; ay <= 1; ++ay)
#pragma unroll
    for (int ax = -1; ax <= 1; ++ax) Gz += (w[ax + 1] * w[ay + 1]) * (B(ax, ay, 1) - B(ax, ay, -1));
#undef B
  double L1 = (fabs(Gx) + fabs(Gy)) + fabs(Gz);
  double cx = ds == 0 ? cs[0][0] : (ds == 1 ? cs[1][0] : cs[2][0]);
  double cy = ds == 0 ? cs[0][1] : (ds == 1 ? cs[1][1] : cs[2][1]);
  double cz = ds == 0 ? cs[0][2] : (ds == 1 ? cs[1][2] : cs[2][2]);
  double qd = ds == 0 ? q[0] : (ds == 1 ? q[1] : q[2]);
  if (L1 > 0.0) {
    double yx = -Gx / L1, yy = -Gy / L1, yz = -Gz / L1;
    double qy = fmax(fmax(fabs(yx), fabs(yy)), fabs(yz));
    if (!(qd <= qy)) {
      nx_ = yx;
      ny_ = yy;
      nz_ = yz;
      return;
    }
  }
  nx_ = cx;
  ny_ = cy;
  nz_ = cz;
}

}  // namespace plic
