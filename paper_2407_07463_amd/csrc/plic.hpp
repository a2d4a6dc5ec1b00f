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
// The half range v = min(c, 1-c) is solved on the sorted, reflected normal
// m1 <= m2 <= m3 with den = 6 m2 m3, where 6 m1 m2 m3 V = alpha^3 -
// sum (alpha - m_i)_+^3 + ...: closed forms where V is a monomial or a
// quadratic in alpha (corner, prism and parallel cases), otherwise Newton
// steps on N(alpha) = den V(alpha) (one division per step, reciprocal of m1
// precomputed), then one Newton polish step on V itself. The result is
// mapped back through the symmetry and the reflections.
__device__ __forceinline__ double alpha_of(double mx, double my, double mz, double c) {
  double neg = 0.0;
  if (mx < 0.0) neg += mx;
  if (my < 0.0) neg += my;
  if (mz < 0.0) neg += mz;
  double m1 = fabs(mx), m2 = fabs(my), m3 = fabs(mz);
  sort3(m1, m2, m3);
  const double M = (m1 + m2) + m3;
  const bool flip = c > 0.5;
  const double v = flip ? 1.0 - c : c;
  const double den = 6.0 * m2 * m3;
  const double m12 = m1 + m2;
  const double vden = v * den;
  const double base2 = 3.0 * m2 * m2 - 3.0 * m2 * m1 + m1 * m1;  // den * V(m2)
  double a;
  if (m1 > 0.0 && vden < m1 * m1) {
    a = cbrt(vden * m1);
  } else if (m2 > 0.0 && vden < base2) {
    a = 0.5 * m1 + sqrt(fmax(2.0 * m2 * m3 * v - m1 * m1 / 12.0, 0.0));
  } else if (m3 >= m12 && 2.0 * m3 * v >= m12) {
    a = v * m3 + 0.5 * m12;
  } else {
    // cubic cases, alpha in [m2, M/2]: start on the chord between the ends
    // (den V = base2 at m2, den/2 at M/2) and take Newton steps on den V
    const double inv1 = 1.0 / m1;
    double lo = m2, hi = 0.5 * M;
    a = lo + (hi - lo) * ((vden - base2) / (0.5 * den - base2));
#pragma unroll 1
    for (int it = 0; it < 8; ++it) {
      const double u2 = a - m2;
      const double u3 = fmax(a - m3, 0.0);
      const double N = (3.0 * a * a - 3.0 * a * m1 + m1 * m1) - (u2 * u2 * u2 + u3 * u3 * u3) * inv1;
      const double dN = (6.0 * a - 3.0 * m1) - 3.0 * (u2 * u2 + u3 * u3) * inv1;
      const double f = N - vden;
      if (f < 0.0) lo = a;
      else hi = a;
      double an = (dN > 0.0) ? a - f / dN : 0.5 * (lo + hi);
      if (!(an >= lo && an <= hi)) an = 0.5 * (lo + hi);
      const double step = fabs(an - a);
      a = an;
      if (step <= 1e-15 * a) break;
    }
  }
  // one Newton polish step on V itself (the closed forms lose bits near case ends)
  {
    double V, dV;
    volume_deriv_sorted(m1, m2, m3, a, V, dV);
    if (dV > 0.0) {
      const double an = a - (V - v) / dV;
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
// order), candidate (sigma, -g1, -g2)/D of quality 1/D, D = (|g1|+|g2|)+1;
// the best quality (smallest D) wins, ties to the lower axis, and only that
// candidate is normalised. Youngs: weighted central
// differences (weights 1,2,1) of the block. The centred-columns candidate is
// kept unless Youngs is defined and its largest component is strictly
// smaller than the centred-columns quality. All sums run in increasing
// stencil index. Values within kResidue of 0 or 1 enter as 0 or 1: the
// round-off residue that conservative fluxes leave in cells the interface
// never reached must not decide the normal of a small isolated sliver (the
// plane constant still matches the cell's own value).
constexpr double kResidue = 1e-12;
__device__ __forceinline__ double clean_residue(double v) {
  return (v <= kResidue) ? 0.0 : ((v >= 1.0 - kResidue) ? 1.0 : v);
}
// An interface (mixed) cell of the advection: its value lies more than
// kResidue inside (0, 1). Every other cell, round-off residues included,
// donates like a pure cell (flux s * c).
__device__ __forceinline__ bool is_mixed(double v) { return v > kResidue && v < 1.0 - kResidue; }
// sigma_low: bit d set when the centred-columns orientation of axis d is +1
// (the low end layer's sums at least the high one's).
__device__ __forceinline__ void myc_normal_sigma(const double *b_in, double &nx_, double &ny_, double &nz_,
                                                 int &sigma_low) {
  double b[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) b[q] = clean_residue(b_in[q]);
#define B(ax, ay, az) b[((ax) + 1) + 3 * ((ay) + 1) + 9 * ((az) + 1)]
  // best centred-columns axis: smallest D = (|g1| + |g2|) + 1, ties to the lower axis
  int ds = 0, sig = 0;
  double bD = 0.0, bs = 0.0, bg1 = 0.0, bg2 = 0.0;
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
    const double sigma = (slo >= shi) ? 1.0 : -1.0;
    if (slo >= shi) sig |= 1 << d;
    const double g1 = (H[2][1] - H[0][1]) / 2.0;
    const double g2 = (H[1][2] - H[1][0]) / 2.0;
    const double D = (fabs(g1) + fabs(g2)) + 1.0;
    if (d == 0 || D < bD) {
      ds = d;
      bD = D;
      bs = sigma;
      bg1 = g1;
      bg2 = g2;
    }
  }
  sigma_low = sig;
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
  const double qd = 1.0 / bD;
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
  const double nd = bs / bD, n1 = -bg1 / bD, n2 = -bg2 / bD;
  if (ds == 0) { nx_ = nd; ny_ = n1; nz_ = n2; }
  else if (ds == 1) { nx_ = n1; ny_ = nd; nz_ = n2; }
  else { nx_ = n1; ny_ = n2; nz_ = nd; }
}
__device__ __forceinline__ void myc_normal(const double *b_in, double &nx_, double &ny_, double &nz_) {
  int sigma_low;
  myc_normal_sigma(b_in, nx_, ny_, nz_, sigma_low);
}

}  // namespace plic
