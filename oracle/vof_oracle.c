/*
 * CPU FP64 ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised reference of every computation on
 * the hot path of the non-coalescing multi-tracer Volume-of-Fluid method
 * (Fintzi, Pierson & Popinet, arXiv 2407.07463). Only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does. It shares no code, header or table with the HIP
 * library: both are written independently from the same definitions.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no fused multiply-add, so
 * every expression below is evaluated exactly in the order written).
 *
 * Grid conventions: cell (i,j,k) is [i,i+1]x[j,j+1]x[k,k+1] in cell units,
 * linear index p = i + nx*(j + ny*k), tri-periodic. Fields of several
 * tracers are stored one after another: c[t][k][j][i]. The face Courant
 * number s_d[p] lives on the lower d-face of cell p.
 *
 * The paper specifies the physics (eq. 3: each colour function obeys
 * dC/dt + u.grad C = 0; section "The no-coalescence.h algorithm": one such
 * equation per tracer C_i) and names geometric PLIC VoF (section "Numerical
 * method") without giving its discrete form. The advection below therefore
 * follows these published methods, read as stated in each function:
 *   - Mixed-Youngs-Centred normals (Aulisa, Manservisi, Scardovelli & Zaleski
 *     2007), with the choice rule "centred-columns unless Youngs' dominant
 *     component is strictly smaller", a reading;
 *   - the plane/unit-cube volume and its inverse (Scardovelli & Zaleski 2000);
 *     the inverse is found here by plain bisection;
 *   - conservative direction-split advection with the c_c dilatation term
 *     (Weymouth & Yue 2010).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of threads the OpenMP loops below use (1 without OpenMP). */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets the number of threads of the OpenMP loops (timing of the baseline). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

#define ORC_OK 0
#define ORC_E_ARG -1
#define ORC_E_CAPACITY -3
#define ORC_E_EXTENT -4

static inline int64_t wrapi(int64_t i, int64_t n) {
  i %= n;
  return i < 0 ? i + n : i;
}

/* =========================================================================
 * Plane volume V(m, alpha): volume of {x in [0,1]^3 : m.x <= alpha}.
 * Piecewise cubic of Scardovelli & Zaleski (2000), written for a sorted,
 * reflected normal; each case is the inclusion-exclusion sum
 * [alpha^3 - sum_i (alpha-m_i)_+^3 + ...] / (6 m1 m2 m3) simplified so that
 * no case divides by a component that may vanish.
 * ========================================================================= */
double orc_plane_volume(double mx, double my, double mz, double alpha) {
  double m[3] = {mx, my, mz};
  /* reflect each negative axis: x_i -> 1 - x_i */
  for (int i = 0; i < 3; ++i) {
    if (m[i] < 0.0) {
      alpha = alpha - m[i];
      m[i] = -m[i];
    }
  }
  double M = (m[0] + m[1]) + m[2];
  if (alpha <= 0.0) return 0.0;
  if (alpha >= M) return 1.0;
  /* central symmetry: V(alpha) = 1 - V(M - alpha) */
  if (2.0 * alpha > M) return 1.0 - orc_plane_volume(m[0], m[1], m[2], M - alpha);
  double m1 = m[0], m2 = m[1], m3 = m[2], t;
  if (m1 > m2) { t = m1; m1 = m2; m2 = t; }
  if (m2 > m3) { t = m2; m2 = m3; m3 = t; }
  if (m1 > m2) { t = m1; m1 = m2; m2 = t; }
  /* (i) the plane cuts off one corner tetrahedron */
  if (alpha < m1) return alpha * alpha * alpha / (6.0 * m1 * m2 * m3);
  double base = 3.0 * alpha * alpha - 3.0 * alpha * m1 + m1 * m1;
  /* (ii) a prism over a triangle truncated by the m1 face */
  if (alpha < m2) return base / (6.0 * m2 * m3);
  /* (iii) the m2 face is crossed as well */
  if (alpha < fmin(m3, m1 + m2)) {
    double u = alpha - m2;
    double corr = (u == 0.0) ? 0.0 : u * u * u / m1;
    return (base - corr) / (6.0 * m2 * m3);
  }
  /* (iv) m3 <= m1 + m2: the m3 face is crossed too (alpha <= M/2 <= m1+m2) */
  if (m3 <= m1 + m2) {
    double u2 = alpha - m2, u3 = alpha - m3;
    double num = u2 * u2 * u2 + u3 * u3 * u3;
    double corr = (num == 0.0) ? 0.0 : num / m1;
    return (base - corr) / (6.0 * m2 * m3);
  }
  /* (v) m3 > m1 + m2: the plane crosses all four edges parallel to axis 3 */
  return (alpha - (m1 + m2) / 2.0) / m3;
}

/* alpha such that V(m, alpha) = c, by bisection on the bracket
 * [sum of negative m_i, sum of positive m_i] (where V = 0 and 1) until the
 * bracket stops shrinking; returns the end point whose volume is closer. */
double orc_plane_alpha(double mx, double my, double mz, double c) {
  double m[3] = {mx, my, mz};
  double lo = 0.0, hi = 0.0;
  for (int i = 0; i < 3; ++i) {
    if (m[i] < 0.0) lo += m[i];
    else hi += m[i];
  }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (orc_plane_volume(mx, my, mz, mid) < c) lo = mid;
    else hi = mid;
  }
  double elo = fabs(orc_plane_volume(mx, my, mz, lo) - c);
  double ehi = fabs(orc_plane_volume(mx, my, mz, hi) - c);
  return (elo <= ehi) ? lo : hi;
}

/* =========================================================================
 * Mixed-Youngs-Centred normal of the centre cell of a 3x3x3 block.
 * b[(ax+1) + 3(ay+1) + 9(az+1)], a in {-1,0,1}^3. Result: outward normal
 * (pointing away from the phase) with |m_x|+|m_y|+|m_z| = 1 up to rounding;
 * the phase is {m.x <= alpha} in the unit cell.
 * Sums run in increasing stencil index, left to right.
 * ========================================================================= */
static inline double blk(const double *b, int ax, int ay, int az) {
  return b[(ax + 1) + 3 * (ay + 1) + 9 * (az + 1)];
}

/* value at offset e along axis d and (u,v) along the transverse axes t1<t2 */
static inline double blk_axis(const double *b, int d, int e, int u, int v) {
  int a[3];
  int t1 = (d == 0) ? 1 : 0;
  int t2 = (d == 2) ? 1 : 2;
  a[d] = e;
  a[t1] = u;
  a[t2] = v;
  return blk(b, a[0], a[1], a[2]);
}

/* Returns 1 if the centred-columns candidate was used, 0 for Youngs.
 * Centred columns: for each column axis d the candidate is
 * (sigma, -g1, -g2)/D with D = (|g1| + |g2|) + 1 and quality 1/D; the best
 * quality is the smallest D (ties: lowest axis), and only that candidate is
 * normalised.
 * Reading: the normal is taken from the block with every value within
 * ORC_RESIDUE of 0 or of 1 replaced by 0 or 1. Conservative fluxes leave such
 * residues (+-1e-17 and below) in cells the interface never reached; they
 * carry no interface information, yet the normal of an interface cell whose
 * neighbours are all residues (a small isolated sliver) would be decided by
 * their rounding noise. The plane constant still matches the cell's own c,
 * so volume is conserved as before. */
#define ORC_RESIDUE 1e-12
int orc_myc_normal_sigma(const double *b_in, double *m_out, double *sigma_out);

int orc_myc_normal(const double *b_in, double *m_out) { return orc_myc_normal_sigma(b_in, m_out, NULL); }

/* The MYC normal as above; sigma_out (nullable) receives the centred-columns
 * orientation of every axis d: +1 when the column sums on the low side of the
 * block (offset -1 along d) are at least those on the high side, else -1. */
int orc_myc_normal_sigma(const double *b_in, double *m_out, double *sigma_out) {
  double b[27];
  for (int q = 0; q < 27; ++q) {
    double v = b_in[q];
    b[q] = (v <= ORC_RESIDUE) ? 0.0 : ((v >= 1.0 - ORC_RESIDUE) ? 1.0 : v);
  }
  double Dd[3], sg[3], g1d[3], g2d[3];
  for (int d = 0; d < 3; ++d) {
    double H[3][3]; /* H[u+1][v+1]: column sums along d */
    for (int v = -1; v <= 1; ++v)
      for (int u = -1; u <= 1; ++u)
        H[u + 1][v + 1] = (blk_axis(b, d, -1, u, v) + blk_axis(b, d, 0, u, v)) + blk_axis(b, d, 1, u, v);
    double slo = 0.0, shi = 0.0;
    for (int v = -1; v <= 1; ++v)
      for (int u = -1; u <= 1; ++u) {
        slo += blk_axis(b, d, -1, u, v);
        shi += blk_axis(b, d, 1, u, v);
      }
    sg[d] = (slo >= shi) ? 1.0 : -1.0;
    g1d[d] = (H[2][1] - H[0][1]) / 2.0;
    g2d[d] = (H[1][2] - H[1][0]) / 2.0;
    Dd[d] = (fabs(g1d[d]) + fabs(g2d[d])) + 1.0;
  }
  int ds = 0;
  for (int d = 1; d < 3; ++d)
    if (Dd[d] < Dd[ds]) ds = d;
  double cs[3];
  {
    int t1 = (ds == 0) ? 1 : 0;
    int t2 = (ds == 2) ? 1 : 2;
    cs[ds] = sg[ds] / Dd[ds];
    cs[t1] = -g1d[ds] / Dd[ds];
    cs[t2] = -g2d[ds] / Dd[ds];
  }
  double qcs = 1.0 / Dd[ds];
  /* Youngs: weighted central differences over the 3x3x3 block */
  static const double w[3] = {1.0, 2.0, 1.0};
  double G[3] = {0.0, 0.0, 0.0};
  for (int az = -1; az <= 1; ++az)
    for (int ay = -1; ay <= 1; ++ay)
      G[0] += (w[ay + 1] * w[az + 1]) * (blk(b, 1, ay, az) - blk(b, -1, ay, az));
  for (int az = -1; az <= 1; ++az)
    for (int ax = -1; ax <= 1; ++ax)
      G[1] += (w[ax + 1] * w[az + 1]) * (blk(b, ax, 1, az) - blk(b, ax, -1, az));
  for (int ay = -1; ay <= 1; ++ay)
    for (int ax = -1; ax <= 1; ++ax)
      G[2] += (w[ax + 1] * w[ay + 1]) * (blk(b, ax, ay, 1) - blk(b, ax, ay, -1));
  double L1 = (fabs(G[0]) + fabs(G[1])) + fabs(G[2]);
  int use_cs = 1;
  double my[3] = {0.0, 0.0, 0.0};
  if (L1 > 0.0) {
    for (int i = 0; i < 3; ++i) my[i] = -G[i] / L1;
    double qy = fmax(fmax(fabs(my[0]), fabs(my[1])), fabs(my[2]));
    use_cs = (qcs <= qy);
  }
  for (int i = 0; i < 3; ++i) m_out[i] = use_cs ? cs[i] : my[i];
  if (sigma_out)
    for (int d = 0; d < 3; ++d) sigma_out[d] = sg[d];
  return use_cs;
}

/* =========================================================================
 * Direction-split advection (Weymouth & Yue 2010 reading).
 * ========================================================================= */
static void gather_block(const double *c, int64_t nx, int64_t ny, int64_t nz, int64_t i, int64_t j, int64_t k,
                         double *b) {
  for (int az = -1; az <= 1; ++az)
    for (int ay = -1; ay <= 1; ++ay)
      for (int ax = -1; ax <= 1; ++ax)
        b[(ax + 1) + 3 * (ay + 1) + 9 * (az + 1)] =
            c[wrapi(i + ax, nx) + nx * (wrapi(j + ay, ny) + ny * wrapi(k + az, nz))];
}

/* Flux through the lower d-face of cell (i,j,k) for face Courant number s,
 * read from the pre-sweep field c: s times the phase fraction of the
 * donor's upwind sub-box of width |s|. */
double orc_face_flux(const double *c, int64_t nx, int64_t ny, int64_t nz, int d, int64_t i, int64_t j, int64_t k,
                     double s) {
  if (s == 0.0) return 0.0;
  int64_t di = i, dj = j, dk = k;
  double x0;
  if (s > 0.0) {
    if (d == 0) di = wrapi(i - 1, nx);
    if (d == 1) dj = wrapi(j - 1, ny);
    if (d == 2) dk = wrapi(k - 1, nz);
    x0 = 1.0 - s;
  } else {
    x0 = 0.0;
  }
  double cd = c[di + nx * (dj + ny * dk)];
  double phi;
  if (!(cd > ORC_RESIDUE && cd < 1.0 - ORC_RESIDUE)) {
    phi = cd; /* pure donor, round-off residues and excursions included */
  } else {
    double b[27], m[3];
    gather_block(c, nx, ny, nz, di, dj, dk, b);
    orc_myc_normal(b, m);
    double alpha = orc_plane_alpha(m[0], m[1], m[2], cd);
    double mp[3] = {m[0], m[1], m[2]};
    mp[d] = m[d] * fabs(s);
    double ap = alpha - m[d] * x0;
    phi = orc_plane_volume(mp[0], mp[1], mp[2], ap);
  }
  return s * phi;
}

/* One sweep along axis d: cout[p] = (c[p] - (F[p+e_d] - F[p])) + cc[p](s[p+e_d] - s[p]),
 * every flux computed from the pre-sweep field cin (Jacobi update). */
void orc_sweep(int64_t nx, int64_t ny, int64_t nz, int d, const double *cin, double *cout, const double *s,
               const uint8_t *cc) {
  int64_t n3 = nx * ny * nz;
  double *F = (double *)malloc(sizeof(double) * n3);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        int64_t p = i + nx * (j + ny * k);
        F[p] = orc_face_flux(cin, nx, ny, nz, d, i, j, k, s[p]);
      }
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        int64_t p = i + nx * (j + ny * k);
        int64_t ip = wrapi(i + (d == 0), nx), jp = wrapi(j + (d == 1), ny), kp = wrapi(k + (d == 2), nz);
        int64_t q = ip + nx * (jp + ny * kp);
        double ccv = cc[p] ? 1.0 : 0.0;
        cout[p] = (cin[p] - (F[q] - F[p])) + ccv * (s[q] - s[p]);
      }
  free(F);
}

/* nsteps direction-split steps of every tracer, in place. Step g (counted
 * from step0) sweeps the axes g mod 3, (g+1) mod 3, (g+2) mod 3; c_c is the
 * indicator c > 0.5 of the field at the start of the step. */
int orc_advect(int64_t nx, int64_t ny, int64_t nz, int ntracers, double *c, const double *sx, const double *sy,
               const double *sz, int64_t step0, int nsteps) {
  if (nx < 1 || ny < 1 || nz < 1 || ntracers < 0 || nsteps < 0 || step0 < 0) return ORC_E_ARG;
  int64_t n3 = nx * ny * nz;
  double *tmp = (double *)malloc(sizeof(double) * n3);
  uint8_t *cc = (uint8_t *)malloc(n3);
  const double *s3[3] = {sx, sy, sz};
  for (int st = 0; st < nsteps; ++st) {
    int64_t g = step0 + st;
    for (int t = 0; t < ntracers; ++t) {
      double *ct = c + (int64_t)t * n3;
      for (int64_t p = 0; p < n3; ++p) cc[p] = ct[p] > 0.5;
      for (int r = 0; r < 3; ++r) {
        int d = (int)((g + r) % 3);
        orc_sweep(nx, ny, nz, d, ct, tmp, s3[d], cc);
        memcpy(ct, tmp, sizeof(double) * n3);
      }
    }
  }
  free(tmp);
  free(cc);
  return ORC_OK;
}

/* =========================================================================
 * Drop labelling: the paper's tag.h step ("The no-coalescence.h algorithm"
 * section) assigns one value per region bounded by interfaces. Reading:
 * regions are the 6-connected periodic components of {c > c_eps}, numbered
 * 1..K in increasing order of their smallest linear index; background 0.
 * Plain breadth-first flood fill seeded in linear order.
 * ========================================================================= */
int orc_label(int64_t nx, int64_t ny, int64_t nz, const double *c, double c_eps, int32_t *labels) {
  int64_t n3 = nx * ny * nz;
  int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (n3 > 0 ? n3 : 1));
  for (int64_t p = 0; p < n3; ++p) labels[p] = 0;
  int32_t next = 0;
  for (int64_t p0 = 0; p0 < n3; ++p0) {
    if (!(c[p0] > c_eps) || labels[p0] != 0) continue;
    ++next;
    int64_t head = 0, tail = 0;
    labels[p0] = next;
    queue[tail++] = p0;
    while (head < tail) {
      int64_t p = queue[head++];
      int64_t i = p % nx, j = (p / nx) % ny, k = p / (nx * ny);
      int64_t nb[6] = {wrapi(i - 1, nx) + nx * (j + ny * k), wrapi(i + 1, nx) + nx * (j + ny * k),
                       i + nx * (wrapi(j - 1, ny) + ny * k), i + nx * (wrapi(j + 1, ny) + ny * k),
                       i + nx * (j + ny * wrapi(k - 1, nz)), i + nx * (j + ny * wrapi(k + 1, nz))};
      for (int e = 0; e < 6; ++e) {
        int64_t q = nb[e];
        if (c[q] > c_eps && labels[q] == 0) {
          labels[q] = next;
          queue[tail++] = q;
        }
      }
    }
  }
  free(queue);
  return next;
}

/* =========================================================================
 * Drop moments: the paper integrates the VoF field over the cells of one tag
 * to get drop properties such as the centre of mass. Volume V = sum c; the
 * periodic centroid takes offsets from the drop's first cell p0 wrapped into
 * [-n/2, n/2): x = (p0 + 0.5) + sum(c delta)/V, wrapped into [0, n).
 * Returns ORC_E_EXTENT if a drop spans n/2 or more cells along an axis.
 * ========================================================================= */
int orc_drop_moments(int64_t nx, int64_t ny, int64_t nz, const double *c, const int32_t *labels, int32_t K,
                     double *vol, double *xyz) {
  int64_t n3 = nx * ny * nz;
  int64_t *p0 = (int64_t *)malloc(sizeof(int64_t) * (K > 0 ? K : 1));
  double *S = (double *)calloc((size_t)(K > 0 ? K : 1) * 4, sizeof(double));
  int64_t *lo = (int64_t *)malloc(sizeof(int64_t) * 3 * (K > 0 ? K : 1));
  int64_t *hi = (int64_t *)malloc(sizeof(int64_t) * 3 * (K > 0 ? K : 1));
  for (int32_t l = 0; l < K; ++l) p0[l] = -1;
  int64_t n[3] = {nx, ny, nz};
  int rc = ORC_OK;
  for (int64_t p = 0; p < n3; ++p) {
    int32_t l = labels[p];
    if (l <= 0) continue;
    if (l > K) { rc = ORC_E_ARG; break; }
    int32_t a = l - 1;
    int64_t x[3] = {p % nx, (p / nx) % ny, p / (nx * ny)};
    if (p0[a] < 0) {
      p0[a] = p;
      for (int e = 0; e < 3; ++e) lo[3 * a + e] = hi[3 * a + e] = 0;
    }
    int64_t r[3] = {p0[a] % nx, (p0[a] / nx) % ny, p0[a] / (nx * ny)};
    S[4 * a] += c[p];
    for (int e = 0; e < 3; ++e) {
      int64_t dd = wrapi(x[e] - r[e], n[e]);
      if (2 * dd >= n[e]) dd -= n[e];
      S[4 * a + 1 + e] += c[p] * (double)dd;
      if (dd < lo[3 * a + e]) lo[3 * a + e] = dd;
      if (dd > hi[3 * a + e]) hi[3 * a + e] = dd;
    }
  }
  for (int32_t a = 0; a < K && rc == ORC_OK; ++a) {
    vol[a] = S[4 * a];
    if (p0[a] < 0) { rc = ORC_E_ARG; break; }
    int64_t r[3] = {p0[a] % nx, (p0[a] / nx) % ny, p0[a] / (nx * ny)};
    for (int e = 0; e < 3; ++e) {
      if (2 * (hi[3 * a + e] - lo[3 * a + e]) >= n[e]) rc = ORC_E_EXTENT;
      double x = ((double)r[e] + 0.5) + S[4 * a + 1 + e] / S[4 * a];
      if (x >= (double)n[e]) x -= (double)n[e];
      if (x < 0.0) x += (double)n[e];
      xyz[3 * a + e] = x;
    }
  }
  free(p0);
  free(S);
  free(lo);
  free(hi);
  return rc;
}

/* =========================================================================
 * Drop shape: inertia tensor about the centroid (appendix "Deformation of the
 * drops": I is the volume integral over the drop of (r.r) delta - r r, with r
 * measured from the drop's centre of mass) and, when face Courant numbers are
 * given, the drop's mean velocity.
 * Reading: the fluid of a cell fills it uniformly with density c, so the cell
 * at offset r from the centroid contributes c ((r.r) delta - r r) + (c/6)
 * delta (the second moment of a uniform unit cube about its centre is delta /
 * 12). r is the cell centre minus the centroid xyz (as vofmt drop moments
 * give it), wrapped into [-n/2, n/2) per axis. The cell velocity is the mean
 * of its two faces' Courant numbers, (s_d[p] + s_d[p + e_d]) / 2, and the drop
 * velocity is sum(c u) / sum(c), in cells per step.
 * inertia: [K][6] = (Ixx, Iyy, Izz, Ixy, Ixz, Iyz). vel: [K][3] or NULL.
 * ========================================================================= */
int orc_drop_shapes(int64_t nx, int64_t ny, int64_t nz, const double *c, const int32_t *labels, int32_t K,
                    const double *xyz, const double *sx, const double *sy, const double *sz, double *inertia,
                    double *vel) {
  int64_t n3 = nx * ny * nz;
  int64_t n[3] = {nx, ny, nz};
  const double *s[3] = {sx, sy, sz};
  double *V = (double *)calloc((size_t)(K > 0 ? K : 1), sizeof(double));
  double *U = (double *)calloc((size_t)(K > 0 ? K : 1) * 3, sizeof(double));
  for (int64_t a = 0; a < 6 * (int64_t)K; ++a) inertia[a] = 0.0;
  int rc = ORC_OK;
  for (int64_t p = 0; p < n3; ++p) {
    int32_t l = labels[p];
    if (l <= 0) continue;
    if (l > K) { rc = ORC_E_ARG; break; }
    int32_t a = l - 1;
    int64_t x[3] = {p % nx, (p / nx) % ny, p / (nx * ny)};
    double r[3];
    for (int e = 0; e < 3; ++e) {
      double d = ((double)x[e] + 0.5) - xyz[3 * a + e];
      if (d >= 0.5 * (double)n[e]) d -= (double)n[e];
      if (d < -0.5 * (double)n[e]) d += (double)n[e];
      r[e] = d;
    }
    double w = c[p];
    double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double *I = inertia + 6 * (int64_t)a;
    I[0] += w * (rr - r[0] * r[0]) + w / 6.0;
    I[1] += w * (rr - r[1] * r[1]) + w / 6.0;
    I[2] += w * (rr - r[2] * r[2]) + w / 6.0;
    I[3] -= w * r[0] * r[1];
    I[4] -= w * r[0] * r[2];
    I[5] -= w * r[1] * r[2];
    V[a] += w;
    if (vel) {
      for (int e = 0; e < 3; ++e) {
        int64_t q[3] = {x[0], x[1], x[2]};
        q[e] = wrapi(q[e] + 1, n[e]);
        double u = 0.5 * (s[e][p] + s[e][q[0] + nx * (q[1] + ny * q[2])]);
        U[3 * a + e] += w * u;
      }
    }
  }
  for (int32_t a = 0; a < K && rc == ORC_OK; ++a) {
    if (!(V[a] > 0.0)) { rc = ORC_E_ARG; break; }
    if (vel)
      for (int e = 0; e < 3; ++e) vel[3 * a + e] = U[3 * a + e] / V[a];
  }
  free(V);
  free(U);
  return rc;
}

/* =========================================================================
 * Multi-tracer surface-tension force (section "The no-coalescence.h
 * algorithm": the force is the sum over the tracers of gamma kappa_i grad C_i,
 * each kappa_i computed as for a single tracer), in the balanced-force
 * face-centred form the paper refers to (Popinet 2018, section "Numerical
 * method"): on the lower d-face of cell p, between m = p - e_d and p,
 *   F_d[p] = gamma * sum_i phi_i (C_i[p] - C_i[m]),
 * with phi_i the mean of kappa_i[p] and kappa_i[m] where both are defined,
 * the defined one where only one is, and no contribution where neither is
 * or where C_i[p] == C_i[m]. Undefined curvature is NaN (as the height
 * functions leave it off the interface). Cell units: kappa in 1/cells, the
 * difference per cell width. Tracers are summed in increasing order.
 * c, kappa: [ntr][nz][ny][nx]; fx, fy, fz: [nz][ny][nx] outputs.
 * ========================================================================= */
static double csf_face(double cp, double cm, double kp, double km) {
  double d = cp - cm;
  if (d == 0.0) return 0.0;
  int hp = !isnan(kp), hm = !isnan(km);
  if (hp && hm) return ((kp + km) / 2.0) * d;
  if (hp) return kp * d;
  if (hm) return km * d;
  return 0.0;
}

void orc_csf_force(int64_t nx, int64_t ny, int64_t nz, int32_t ntr, const double *c, const double *kappa,
                   double gamma, double *fx, double *fy, double *fz) {
  int64_t n3 = nx * ny * nz;
  double *f[3] = {fx, fy, fz};
  for (int64_t p = 0; p < n3; ++p) {
    int64_t i = p % nx, j = (p / nx) % ny, k = p / (nx * ny);
    int64_t m[3] = {wrapi(i - 1, nx) + nx * (j + ny * k), i + nx * (wrapi(j - 1, ny) + ny * k),
                    i + nx * (j + ny * wrapi(k - 1, nz))};
    for (int d = 0; d < 3; ++d) {
      double sum = 0.0;
      for (int32_t t = 0; t < ntr; ++t) {
        const double *ct = c + (int64_t)t * n3, *kt = kappa + (int64_t)t * n3;
        sum += csf_face(ct[p], ct[m[d]], kt[p], kt[m[d]]);
      }
      f[d][p] = gamma * sum;
    }
  }
}

/* =========================================================================
 * Tracer recolouring: Steps 1-4 of the no-coalescence algorithm.
 * Reading: drops are (tracer t, label l); two distinct drops are neighbours
 * when occupied cells p, q of each satisfy |o|^2 < (1+tau)^2 for the periodic
 * offset o = q - p (o = 0 included across tracers), i.e. fewer than tau empty
 * cell widths separate them. Neighbours in the same tracer conflict (the
 * distinct-tag requirement of Step 3 holds by construction). Drops are taken
 * in ascending (t, l); a drop moves when an earlier neighbour has its current
 * tracer, to the smallest tracer n != T(D) used by none of its neighbours, or
 * to a new tracer N when every existing one is taken (Step 4).
 * Moves: every moved cell is first cleared in its old field, then added to
 * its new field; fields of newly created tracers start from zero.
 * ========================================================================= */
typedef struct {
  int32_t a, b;
} orc_edge;

static int edge_cmp(const void *x, const void *y) {
  const orc_edge *e = (const orc_edge *)x, *f = (const orc_edge *)y;
  if (e->a != f->a) return e->a < f->a ? -1 : 1;
  if (e->b != f->b) return e->b < f->b ? -1 : 1;
  return 0;
}

/* Symmetric neighbour list (both directions), sorted and unique.
 * Returns the number of directed edges; *out is malloc'ed. */
int64_t orc_neighbours(int64_t nx, int64_t ny, int64_t nz, int ntr, const int32_t *labels, const int32_t *ndrops,
                       double tau, orc_edge **out) {
  int64_t n3 = nx * ny * nz;
  int32_t *off = (int32_t *)malloc(sizeof(int32_t) * (ntr + 1));
  off[0] = 0;
  for (int t = 0; t < ntr; ++t) off[t + 1] = off[t] + ndrops[t];
  double lim = (1.0 + tau) * (1.0 + tau);
  int R = (int)floor(1.0 + tau);
  int64_t cap = 1024, ne = 0;
  orc_edge *E = (orc_edge *)malloc(sizeof(orc_edge) * cap);
  for (int t = 0; t < ntr; ++t)
    for (int64_t p = 0; p < n3; ++p) {
      int32_t l = labels[(int64_t)t * n3 + p];
      if (l <= 0) continue;
      int32_t ga = off[t] + l - 1;
      int64_t i = p % nx, j = (p / nx) % ny, k = p / (nx * ny);
      for (int oz = -R; oz <= R; ++oz)
        for (int oy = -R; oy <= R; ++oy)
          for (int ox = -R; ox <= R; ++ox) {
            double o2 = (double)(ox * ox + oy * oy + oz * oz);
            if (!(o2 < lim)) continue;
            int64_t q = wrapi(i + ox, nx) + nx * (wrapi(j + oy, ny) + ny * wrapi(k + oz, nz));
            for (int u = 0; u < ntr; ++u) {
              int32_t l2 = labels[(int64_t)u * n3 + q];
              if (l2 <= 0) continue;
              int32_t gb = off[u] + l2 - 1;
              if (gb == ga) continue;
              if (ne == cap) {
                cap *= 2;
                E = (orc_edge *)realloc(E, sizeof(orc_edge) * cap);
              }
              E[ne].a = ga;
              E[ne].b = gb;
              ++ne;
            }
          }
    }
  qsort(E, ne, sizeof(orc_edge), edge_cmp);
  int64_t m = 0;
  for (int64_t e = 0; e < ne; ++e)
    if (m == 0 || edge_cmp(&E[m - 1], &E[e]) != 0) E[m++] = E[e];
  free(off);
  *out = E;
  return m;
}

/* Export of the neighbour list for tests: fills pairs[2*e], pairs[2*e+1]
 * (directed, sorted) up to cap entries; returns the count. */
int64_t orc_neighbour_pairs(int64_t nx, int64_t ny, int64_t nz, int ntr, const int32_t *labels,
                            const int32_t *ndrops, double tau, int32_t *pairs, int64_t cap) {
  orc_edge *E = NULL;
  int64_t m = orc_neighbours(nx, ny, nz, ntr, labels, ndrops, tau, &E);
  for (int64_t e = 0; e < m && e < cap; ++e) {
    pairs[2 * e] = E[e].a;
    pairs[2 * e + 1] = E[e].b;
  }
  free(E);
  return m;
}

/* =========================================================================
 * The near-contact criterion of Steps 1-3 read literally, on the 5x5(x5)
 * stencil: a cell p of tracer t with no drop (label 0: "C_i = 0 at the
 * centre") and two opposite cells p + o, p - o, o in {-2..2}^3 \ {0}, both
 * occupied ("C_i > 1" read as C_i > 0, per the figure caption) -- Step 1 --
 * whose labels differ -- Step 3. Per cell of one tracer's labels:
 * flags[p] = 0 (no), 1 (Step 1 only), 2 (Steps 1 and 3).
 * ========================================================================= */
void orc_stencil_flags(int64_t nx, int64_t ny, int64_t nz, const int32_t *lab, uint8_t *flags) {
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) {
        int64_t p = i + nx * (j + ny * k);
        uint8_t f = 0;
        if (lab[p] == 0) {
          for (int oz = -2; oz <= 2; ++oz)
            for (int oy = -2; oy <= 2; ++oy)
              for (int ox = -2; ox <= 2; ++ox) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                int32_t a = lab[wrapi(i + ox, nx) + nx * (wrapi(j + oy, ny) + ny * wrapi(k + oz, nz))];
                int32_t b = lab[wrapi(i - ox, nx) + nx * (wrapi(j - oy, ny) + ny * wrapi(k - oz, nz))];
                if (a > 0 && b > 0) {
                  if (f < 1) f = 1;
                  if (a != b) f = 2;
                }
              }
        }
        flags[p] = f;
      }
}

/* Neighbour list of the literal mode (symmetric, sorted, unique):
 * - drops of one tracer are neighbours when the criterion of Steps 1-3
 *   holds for some centre with one opposite cell in each (the conflicts);
 * - drops of different tracers are in contact (Step 4's "tracers already
 *   in contact with the region") when a cell of one lies within the
 *   stencil's reach of a cell of the other: 4 cells along every axis (the
 *   two opposite cells of a 5-cell stencil are 4 apart), overlap included.
 *   Reading: the paper does not define this contact. */
int64_t orc_neighbours_stencil(int64_t nx, int64_t ny, int64_t nz, int ntr, const int32_t *labels,
                               const int32_t *ndrops, orc_edge **out) {
  int64_t n3 = nx * ny * nz;
  int32_t *off = (int32_t *)malloc(sizeof(int32_t) * (ntr + 1));
  off[0] = 0;
  for (int t = 0; t < ntr; ++t) off[t + 1] = off[t] + ndrops[t];
  int64_t cap = 1024, ne = 0;
  orc_edge *E = (orc_edge *)malloc(sizeof(orc_edge) * cap);
#define ORC_ADD_EDGE(ga, gb)                                    \
  do {                                                          \
    if (ne == cap) {                                            \
      cap *= 2;                                                 \
      E = (orc_edge *)realloc(E, sizeof(orc_edge) * cap);       \
    }                                                           \
    E[ne].a = (ga);                                             \
    E[ne].b = (gb);                                             \
    ++ne;                                                       \
  } while (0)
  for (int t = 0; t < ntr; ++t) {
    const int32_t *lab = labels + (int64_t)t * n3;
    for (int64_t p = 0; p < n3; ++p) {
      int64_t i = p % nx, j = (p / nx) % ny, k = p / (nx * ny);
      int32_t l = lab[p];
      if (l == 0) {
        /* Steps 1 and 3 about centre p */
        for (int oz = -2; oz <= 2; ++oz)
          for (int oy = -2; oy <= 2; ++oy)
            for (int ox = -2; ox <= 2; ++ox) {
              if (ox == 0 && oy == 0 && oz == 0) continue;
              int32_t a = lab[wrapi(i + ox, nx) + nx * (wrapi(j + oy, ny) + ny * wrapi(k + oz, nz))];
              int32_t b = lab[wrapi(i - ox, nx) + nx * (wrapi(j - oy, ny) + ny * wrapi(k - oz, nz))];
              if (a > 0 && b > 0 && a != b) ORC_ADD_EDGE(off[t] + a - 1, off[t] + b - 1);
            }
      } else if (l > 0) {
        /* drops of other tracers within reach of this cell */
        for (int oz = -4; oz <= 4; ++oz)
          for (int oy = -4; oy <= 4; ++oy)
            for (int ox = -4; ox <= 4; ++ox) {
              int64_t q = wrapi(i + ox, nx) + nx * (wrapi(j + oy, ny) + ny * wrapi(k + oz, nz));
              for (int u = 0; u < ntr; ++u) {
                if (u == t) continue;
                int32_t l2 = labels[(int64_t)u * n3 + q];
                if (l2 > 0) ORC_ADD_EDGE(off[t] + l - 1, off[u] + l2 - 1);
              }
            }
      }
    }
  }
#undef ORC_ADD_EDGE
  qsort(E, ne, sizeof(orc_edge), edge_cmp);
  int64_t m = 0;
  for (int64_t e = 0; e < ne; ++e)
    if (m == 0 || edge_cmp(&E[m - 1], &E[e]) != 0) E[m++] = E[e];
  free(off);
  *out = E;
  return m;
}

/* Export of the literal mode's neighbour list for tests (as orc_neighbour_pairs). */
int64_t orc_neighbour_pairs_stencil(int64_t nx, int64_t ny, int64_t nz, int ntr, const int32_t *labels,
                                    const int32_t *ndrops, int32_t *pairs, int64_t cap) {
  orc_edge *E = NULL;
  int64_t m = orc_neighbours_stencil(nx, ny, nz, ntr, labels, ndrops, &E);
  for (int64_t e = 0; e < m && e < cap; ++e) {
    pairs[2 * e] = E[e].a;
    pairs[2 * e + 1] = E[e].b;
  }
  free(E);
  return m;
}

/* Steps 4 and the cell moves, given the symmetric sorted neighbour list E
 * (freed here). */
static int recolor_given_edges(int64_t nx, int64_t ny, int64_t nz, int32_t *ntracers, int32_t max_tracers, double *c,
                               const int32_t *labels, const int32_t *ndrops, orc_edge *E, int64_t ne,
                               int32_t *new_tracer, int32_t *nmoved) {
  int ntr = *ntracers;
  int64_t n3 = nx * ny * nz;
  int32_t D = 0;
  for (int t = 0; t < ntr; ++t) D += ndrops[t];
  int32_t *T = (int32_t *)malloc(sizeof(int32_t) * (D > 0 ? D : 1));
  {
    int32_t g = 0;
    for (int t = 0; t < ntr; ++t)
      for (int32_t l = 1; l <= ndrops[t]; ++l, ++g) T[g] = t;
  }
  int64_t *first = (int64_t *)malloc(sizeof(int64_t) * (D + 1));
  {
    int64_t e = 0;
    for (int32_t g = 0; g <= D; ++g) {
      while (e < ne && E[e].a < g) ++e;
      first[g] = e;
    }
  }
  int N = ntr;
  int32_t moved = 0;
  uint8_t *used = (uint8_t *)malloc((size_t)max_tracers + 1);
  int rc = ORC_OK;
  for (int32_t g = 0; g < D; ++g) {
    int conflict = 0;
    for (int64_t e = first[g]; e < first[g + 1]; ++e)
      if (E[e].b < g && T[E[e].b] == T[g]) conflict = 1;
    if (!conflict) continue;
    memset(used, 0, (size_t)max_tracers + 1);
    for (int64_t e = first[g]; e < first[g + 1]; ++e) used[T[E[e].b]] = 1;
    int n = -1;
    for (int cand = 0; cand < N; ++cand)
      if (cand != T[g] && !used[cand]) { n = cand; break; }
    if (n < 0) {
      if (N + 1 > max_tracers) { rc = ORC_E_CAPACITY; break; }
      n = N++;
    }
    T[g] = n;
    ++moved;
  }
  if (rc == ORC_OK) {
    for (int t = ntr; t < N; ++t) memset(c + (int64_t)t * n3, 0, sizeof(double) * n3);
    /* the drop of each (tracer, label) in the old state */
    int32_t *off = (int32_t *)malloc(sizeof(int32_t) * (ntr + 1));
    off[0] = 0;
    for (int t = 0; t < ntr; ++t) off[t + 1] = off[t] + ndrops[t];
    double *save = (double *)malloc(sizeof(double) * (size_t)ntr * n3);
    memcpy(save, c, sizeof(double) * (size_t)ntr * n3);
    for (int t = 0; t < ntr; ++t)
      for (int64_t p = 0; p < n3; ++p) {
        int32_t l = labels[(int64_t)t * n3 + p];
        if (l > 0 && T[off[t] + l - 1] != t) c[(int64_t)t * n3 + p] = 0.0;
      }
    for (int t = 0; t < ntr; ++t)
      for (int64_t p = 0; p < n3; ++p) {
        int32_t l = labels[(int64_t)t * n3 + p];
        if (l > 0) {
          int32_t n = T[off[t] + l - 1];
          if (n != t) c[(int64_t)n * n3 + p] += save[(int64_t)t * n3 + p];
        }
      }
    free(save);
    free(off);
    for (int32_t g = 0; g < D; ++g) new_tracer[g] = T[g];
    *ntracers = N;
    *nmoved = moved;
  }
  free(T);
  free(E);
  free(first);
  free(used);
  return rc;
}

int orc_recolor(int64_t nx, int64_t ny, int64_t nz, int32_t *ntracers, int32_t max_tracers, double *c,
                const int32_t *labels, const int32_t *ndrops, double tau, int32_t *new_tracer, int32_t *nmoved) {
  int ntr = *ntracers;
  if (ntr < 0 || ntr > max_tracers || tau < 0.0) return ORC_E_ARG;
  orc_edge *E = NULL;
  int64_t ne = orc_neighbours(nx, ny, nz, ntr, labels, ndrops, tau, &E);
  return recolor_given_edges(nx, ny, nz, ntracers, max_tracers, c, labels, ndrops, E, ne, new_tracer, nmoved);
}

/* Steps 1-4 with the literal stencil criterion (orc_neighbours_stencil). */
int orc_recolor_stencil(int64_t nx, int64_t ny, int64_t nz, int32_t *ntracers, int32_t max_tracers, double *c,
                        const int32_t *labels, const int32_t *ndrops, int32_t *new_tracer, int32_t *nmoved) {
  int ntr = *ntracers;
  if (ntr < 0 || ntr > max_tracers) return ORC_E_ARG;
  orc_edge *E = NULL;
  int64_t ne = orc_neighbours_stencil(nx, ny, nz, ntr, labels, ndrops, &E);
  return recolor_given_edges(nx, ny, nz, ntracers, max_tracers, c, labels, ndrops, E, ne, new_tracer, nmoved);
}

/* =========================================================================
 * Tracer compaction. The paper reports the number of tracers in use, N(t)
 * (section "The no-coalescence.h algorithm"), and notes that its algorithm
 * could be optimised. Reading: a tracer holding no drop is retired; the
 * other fields keep their order and move down over the gaps; the freed
 * fields are zeroed. The retired fields' values (none above the labelling
 * threshold) are summed, tracer by tracer and cell by cell, into
 * *discarded. new_index[t] is the new position of tracer t or -1. Returns
 * the new tracer count.
 * ========================================================================= */
int orc_compact_tracers(int64_t n3, int32_t ntr, double *c, const int32_t *ndrops, int32_t *new_index,
                        double *discarded) {
  double sum = 0.0;
  int32_t k = 0;
  for (int32_t t = 0; t < ntr; ++t) {
    if (ndrops[t] > 0) {
      new_index[t] = k;
      if (k != t) memcpy(c + (int64_t)k * n3, c + (int64_t)t * n3, sizeof(double) * n3);
      ++k;
    } else {
      new_index[t] = -1;
      for (int64_t p = 0; p < n3; ++p) sum += c[(int64_t)t * n3 + p];
    }
  }
  for (int32_t t = k; t < ntr; ++t) memset(c + (int64_t)t * n3, 0, sizeof(double) * n3);
  *discarded = sum;
  return k;
}

/* =========================================================================
 * Nearest-particle statistics ("Nearest particle statistics" section,
 * eq. 4 with the tie weight h_ij = 1/N_i, the estimators eqs. 6, 8 and 10,
 * and the moments of eqs. 11 and 14 read as averages over the events:
 * M = (1/E) sum h r, R = (1/E) sum h r r^T).
 *
 * Minimum image per axis: r = x_j - x_i; r -= L if r > L/2; r += L if
 * r <= -L/2. d2 = (rx^2 + ry^2) + rz^2. The nearest set of i is every j != i
 * with d2 equal to the minimum (exact equality); nn_index is the smallest.
 * Histogram: radial bin k with r2_edges[k] <= d2 < r2_edges[k+1]; polar bin
 * m = number of interior polar edges e (1..ntheta-1) with cos(theta) <=
 * cos_edges[e], tested without sqrt as rv|rv| <= (ce|ce|) d2, theta measured
 * from the vertical axis. Weights are integers in units of 1/720720
 * (720720 = lcm(1..16)); an event outside the radial range goes to the
 * last slot hist[nr*ntheta].
 * ========================================================================= */
int orc_nearest_pair_stats(int32_t n, const double *xyz, const double *box, int32_t vaxis, int32_t nr,
                           int32_t nth, const double *r2_edges, const double *cos_edges, int32_t *nn_index,
                           int32_t *nn_ties, uint64_t *hist, double *M, double *R, double *A) {
  if (n < 2 || vaxis < 0 || vaxis > 2 || nr < 1 || nth < 1) return ORC_E_ARG;
  memset(hist, 0, sizeof(uint64_t) * ((size_t)nr * nth + 1));
  double SM[3] = {0, 0, 0}, SR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int32_t i = 0; i < n; ++i) {
    double best = INFINITY;
    int32_t bj = -1, ties = 0;
    for (int32_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double r[3];
      for (int a = 0; a < 3; ++a) {
        double d = xyz[3 * j + a] - xyz[3 * i + a];
        if (d > 0.5 * box[a]) d -= box[a];
        else if (d <= -0.5 * box[a]) d += box[a];
        r[a] = d;
      }
      double d2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
      if (d2 < best) { best = d2; bj = j; ties = 1; }
      else if (d2 == best) ties += 1;
    }
    nn_index[i] = bj;
    nn_ties[i] = ties;
    double h = 1.0 / (double)ties;
    uint64_t wfix = 720720u / (uint64_t)ties;
    for (int32_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double r[3];
      for (int a = 0; a < 3; ++a) {
        double d = xyz[3 * j + a] - xyz[3 * i + a];
        if (d > 0.5 * box[a]) d -= box[a];
        else if (d <= -0.5 * box[a]) d += box[a];
        r[a] = d;
      }
      double d2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
      if (d2 != best) continue;
      int32_t k = -1;
      for (int32_t e = 0; e <= nr; ++e)
        if (r2_edges[e] <= d2) k = e;
      int32_t m = 0;
      double rv = r[vaxis];
      for (int32_t e = 1; e < nth; ++e) {
        double ce = cos_edges[e];
        if (rv * fabs(rv) <= (ce * fabs(ce)) * d2) m = e;
      }
      if (k < 0 || k >= nr) hist[(size_t)nr * nth] += wfix;
      else hist[(size_t)k * nth + m] += wfix;
      for (int a = 0; a < 3; ++a) {
        SM[a] += h * r[a];
        for (int b = 0; b < 3; ++b) SR[3 * a + b] += h * (r[a] * r[b]);
      }
    }
  }
  for (int a = 0; a < 3; ++a) M[a] = SM[a] / (double)n;
  for (int a = 0; a < 9; ++a) R[a] = SR[a] / (double)n;
  /* deviatoric part A = R - (tr R / 3) delta (second-moment section; its
   * "3 tr(R)" in the text on the figure is read as tr(R) = R : delta) */
  double tr = (R[0] + R[4]) + R[8];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) A[3 * a + b] = (a == b) ? R[3 * a + b] - tr / 3.0 : R[3 * a + b];
  return ORC_OK;
}

/* =========================================================================
 * Probability densities of the nearest-particle vector from an accumulated
 * histogram ("Nearest particle statistics", eqs. 8 and 10): with E events
 * and E_k the (fixed-point) weight of bin k,
 *   P_nst(r, theta) = E_km / (E 2 pi r^2 sin(theta) dr dtheta),
 *   P_r-nst(r)      = (sum over theta of E_km) / (E 4 pi r^2 dr),
 * evaluated at the bin centres r_c = (r_k + r_k+1)/2, theta_c = (theta_m +
 * theta_m+1)/2 (reading: the paper writes the left edges, which makes the
 * first radial bin and the first polar bin singular). r_edges[nr+1] ascending
 * and th_edges[nth+1] ascending in [0, pi] are the edges whose squares and
 * cosines binned the histogram. Weights are in units of 1/720720.
 * P[nr][nth], Pr[nr]. Returns ORC_E_ARG for bad sizes or events < 1.
 * ========================================================================= */
int orc_pair_pdfs(int32_t nr, int32_t nth, const double *r_edges, const double *th_edges, const uint64_t *hist,
                  int64_t events, double *P, double *Pr) {
  if (nr < 1 || nth < 1 || events < 1) return ORC_E_ARG;
  const double pi = 3.14159265358979323846;
  const double E = (double)events * 720720.0;
  for (int32_t k = 0; k < nr; ++k) {
    double rc = 0.5 * (r_edges[k] + r_edges[k + 1]);
    double dr = r_edges[k + 1] - r_edges[k];
    uint64_t row = 0;
    for (int32_t m = 0; m < nth; ++m) {
      double tc = 0.5 * (th_edges[m] + th_edges[m + 1]);
      double dth = th_edges[m + 1] - th_edges[m];
      uint64_t ek = hist[(size_t)k * nth + m];
      row += ek;
      P[(size_t)k * nth + m] = (double)ek / (E * (2.0 * pi * (rc * rc) * sin(tc) * dr * dth));
    }
    Pr[k] = (double)row / (E * (4.0 * pi * (rc * rc) * dr));
  }
  return ORC_OK;
}

/* =========================================================================
 * Height-function curvature of one tracer (the paper computes kappa_i of
 * each tracer "as for a single tracer", citing Popinet 2018). Reading:
 * fixed 7-cell columns (Cummins, Francois & Kothe 2005). For an interface
 * cell (c more than ORC_RESIDUE inside (0, 1): round-off residues of pure
 * cells are not interface cells) take the MYC normal m; try the column axes in order of
 * decreasing |m_d| (ties: lower axis first); an axis is valid when every one
 * of the 3x3 columns has its end on the phase side (-sign(m_d), sign(0)=+1)
 * full (c >= 1-1e-6) and its other end empty (c <= 1e-6). Heights are the
 * column sums H(u,v) over offsets -3..3; with (u,v) along the transverse
 * axes in increasing order,
 *   kappa*Delta = -[Hxx(1+Hy^2) + Hyy(1+Hx^2) - 2 Hxy Hx Hy] / (1+Hx^2+Hy^2)^{3/2}
 * which is +2/R on a sphere of radius R cells. status: 0 not an interface
 * cell (kappa NaN), 1..3 = valid on the 1st..3rd axis tried, 4 = no valid
 * axis (kappa NaN).
 * ========================================================================= */
int orc_curvature_hf(int64_t nx, int64_t ny, int64_t nz, const double *c, double *kappa, uint8_t *status) {
  int64_t n3 = nx * ny * nz;
  int64_t n[3] = {nx, ny, nz};
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t p = 0; p < n3; ++p) {
    double cp = c[p];
    kappa[p] = NAN;
    status[p] = 0;
    if (!(cp > ORC_RESIDUE && cp < 1.0 - ORC_RESIDUE)) continue; /* interface cells only */
    int64_t x[3] = {p % nx, (p / nx) % ny, p / (nx * ny)};
    double b[27], m[3];
    gather_block(c, nx, ny, nz, x[0], x[1], x[2], b);
    orc_myc_normal(b, m);
    int order[3] = {0, 1, 2};
    for (int a = 0; a < 3; ++a)
      for (int bb = a + 1; bb < 3; ++bb)
        if (fabs(m[order[bb]]) > fabs(m[order[a]]) ||
            (fabs(m[order[bb]]) == fabs(m[order[a]]) && order[bb] < order[a])) {
          int t = order[a];
          order[a] = order[bb];
          order[bb] = t;
        }
    status[p] = 4;
    for (int at = 0; at < 3; ++at) {
      int d = order[at];
      int t1 = (d == 0) ? 1 : 0;
      int t2 = (d == 2) ? 1 : 2;
      int sigma = (m[d] >= 0.0) ? 1 : -1;
      double H[3][3];
      int ok = 1;
      for (int v = -1; v <= 1 && ok; ++v)
        for (int u = -1; u <= 1 && ok; ++u) {
          double col[7];
          for (int e = -3; e <= 3; ++e) {
            int64_t y[3] = {x[0], x[1], x[2]};
            y[d] = wrapi(y[d] + e, n[d]);
            y[t1] = wrapi(y[t1] + u, n[t1]);
            y[t2] = wrapi(y[t2] + v, n[t2]);
            col[e + 3] = c[y[0] + nx * (y[1] + ny * y[2])];
          }
          double full_end = (sigma > 0) ? col[0] : col[6];
          double empty_end = (sigma > 0) ? col[6] : col[0];
          if (!(full_end >= 1.0 - 1e-6 && empty_end <= 1e-6)) ok = 0;
          double h = 0.0;
          for (int e = 0; e < 7; ++e) h += col[e];
          H[u + 1][v + 1] = h;
        }
      if (!ok) continue;
      double Hx = (H[2][1] - H[0][1]) / 2.0;
      double Hy = (H[1][2] - H[1][0]) / 2.0;
      double Hxx = (H[2][1] - 2.0 * H[1][1]) + H[0][1];
      double Hyy = (H[1][2] - 2.0 * H[1][1]) + H[1][0];
      double Hxy = (((H[2][2] - H[2][0]) - H[0][2]) + H[0][0]) / 4.0;
      double num = (Hxx * (1.0 + Hy * Hy) + Hyy * (1.0 + Hx * Hx)) - ((2.0 * Hxy) * Hx) * Hy;
      double den = (1.0 + Hx * Hx) + Hy * Hy;
      kappa[p] = -num / (den * sqrt(den));
      status[p] = (uint8_t)(1 + at);
      break;
    }
  }
  return ORC_OK;
}
