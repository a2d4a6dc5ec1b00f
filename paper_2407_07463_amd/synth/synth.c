/*
 * Seeded synthetic inputs shared by the HIP path and the CPU oracle.
 *
 * This file holds no arithmetic of the Volume-of-Fluid method itself: no
 * interface reconstruction, no plane/cube volume, no flux. It provides
 *   - the splitmix64 generator (Steele, Lea & Flood 2014), uniform doubles
 *     from the top 53 bits;
 *   - random sequential addition (RSA) of non-overlapping spheres in a
 *     periodic box, accelerated with a bucket grid;
 *   - accurate volume fractions of ellipsoids (spheres included) on a
 *     tri-periodic grid, computed as the z-integral of the exact area of the
 *     elliptic slice inside each cell's xy-square (circle/polygon clipping in
 *     the affine frame where the slice is a disc), by Gauss-Legendre
 *     quadrature between the points where that area is not smooth.
 *
 * The drops of the paper's simulations are spheres in a periodic box
 * (Numerical method section); the ellipsoids serve the curvature training
 * data. Everything is in cell units: cell (i,j,k) is [i,i+1]x[j,j+1]x[k,k+1].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------- splitmix64 ---------------- */

static inline uint64_t sm64_next(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline double sm64_unif(uint64_t *s) {
  return (double)(sm64_next(s) >> 11) * 0x1.0p-53;
}

/* Fill out[0..n) with uniform doubles in [0,1) from the stream seeded by
 * *state; the state is advanced in place so streams can be continued. */
void synth_uniform(uint64_t *state, int64_t n, double *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = sm64_unif(state);
}

/* ---------------- random sequential addition ---------------- */

static double wrap_delta(double d, double L) {
  if (d > 0.5 * L) return d - L;
  if (d <= -0.5 * L) return d + L;
  return d;
}

/*
 * Place spheres of the given radii one after another at uniform random
 * centres in the periodic box [0,L)^3, rejecting a candidate whose surface
 * comes closer than `gap` to an already placed sphere (periodic distance).
 * Each sphere gets at most max_attempts tries. Returns the number placed;
 * centres[3*i..3*i+2] holds sphere i. The RNG stream is advanced in place.
 */
int synth_rsa(uint64_t *state, int n, const double *radii, double Lx, double Ly,
              double Lz, double gap, int64_t max_attempts, double *centres) {
  double rmax = 0.0;
  for (int i = 0; i < n; ++i) rmax = radii[i] > rmax ? radii[i] : rmax;
  double reach = 2.0 * rmax + gap; /* largest centre distance that can conflict */
  int bx = (int)floor(Lx / reach), by = (int)floor(Ly / reach), bz = (int)floor(Lz / reach);
  if (bx < 1) bx = 1;
  if (by < 1) by = 1;
  if (bz < 1) bz = 1;
  int nb = bx * by * bz;
  int *head = (int *)malloc(sizeof(int) * nb);
  int *next = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
  for (int b = 0; b < nb; ++b) head[b] = -1;
  int placed = 0;
  for (int i = 0; i < n; ++i) {
    int ok = 0;
    for (int64_t a = 0; a < max_attempts && !ok; ++a) {
      double x = sm64_unif(state) * Lx, y = sm64_unif(state) * Ly, z = sm64_unif(state) * Lz;
      int cx = (int)(x / Lx * bx), cy = (int)(y / Ly * by), cz = (int)(z / Lz * bz);
      if (cx >= bx) cx = bx - 1;
      if (cy >= by) cy = by - 1;
      if (cz >= bz) cz = bz - 1;
      ok = 1;
      int rx = bx < 3 ? 0 : 1, ry = by < 3 ? 0 : 1, rz = bz < 3 ? 0 : 1;
      int full = (bx < 3 || by < 3 || bz < 3);
      if (full) {
        for (int j = 0; j < placed && ok; ++j) {
          double dx = wrap_delta(centres[3 * j] - x, Lx);
          double dy = wrap_delta(centres[3 * j + 1] - y, Ly);
          double dz = wrap_delta(centres[3 * j + 2] - z, Lz);
          double lim = radii[i] + radii[j] + gap;
          if (dx * dx + dy * dy + dz * dz < lim * lim) ok = 0;
        }
      } else {
        for (int oz = -rz; oz <= rz && ok; ++oz)
          for (int oy = -ry; oy <= ry && ok; ++oy)
            for (int ox = -rx; ox <= rx && ok; ++ox) {
              int b = ((cx + ox + bx) % bx) + bx * (((cy + oy + by) % by) + by * ((cz + oz + bz) % bz));
              for (int j = head[b]; j >= 0 && ok; j = next[j]) {
                double dx = wrap_delta(centres[3 * j] - x, Lx);
                double dy = wrap_delta(centres[3 * j + 1] - y, Ly);
                double dz = wrap_delta(centres[3 * j + 2] - z, Lz);
                double lim = radii[i] + radii[j] + gap;
                if (dx * dx + dy * dy + dz * dz < lim * lim) ok = 0;
              }
            }
      }
      if (ok) {
        centres[3 * i] = x;
        centres[3 * i + 1] = y;
        centres[3 * i + 2] = z;
        int b = cx + bx * (cy + by * cz);
        next[i] = head[b];
        head[b] = i;
        placed = i + 1;
      }
    }
    if (!ok) break;
  }
  free(head);
  free(next);
  return placed;
}

/* ---------------- Gauss-Legendre nodes ---------------- */

#define GL_MAX 32
static double gl_x[GL_MAX], gl_w[GL_MAX];
static int gl_n = 0;

/* Nodes and weights on [0,1] by Newton iteration on the Legendre polynomial. */
static void gl_init(int n) {
  if (gl_n == n) return;
  for (int i = 0; i < n; ++i) {
    double x = cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
    }
    gl_x[i] = 0.5 * (1.0 - x);
    gl_w[i] = 1.0 / ((1.0 - x * x) * dp * dp);
  }
  gl_n = n;
}

/* ---------------- disc / polygon clipping ---------------- */

/* Signed area of disc(0,r) intersected with triangle (0, A, B). */
static double tri_disc(double r, double ax, double ay, double bx, double by) {
  double dx = bx - ax, dy = by - ay;
  double a = dx * dx + dy * dy;
  double r2 = r * r;
  if (a == 0.0) return 0.0;
  double b = ax * dx + ay * dy;
  double c = ax * ax + ay * ay - r2;
  double disc = b * b - a * c;
  double t1 = 1.0, t2 = 1.0; /* inside interval [t1,t2] clipped to [0,1] */
  if (disc > 0.0) {
    double sq = sqrt(disc);
    t1 = (-b - sq) / a;
    t2 = (-b + sq) / a;
    if (t1 < 0.0) t1 = 0.0;
    if (t2 > 1.0) t2 = 1.0;
    if (t1 >= t2) { t1 = 1.0; t2 = 1.0; }
  }
  double px = ax + t1 * dx, py = ay + t1 * dy;
  double qx = ax + t2 * dx, qy = ay + t2 * dy;
  double area = 0.0;
  /* outside piece A -> P: circular sector */
  if (t1 > 0.0) area += 0.5 * r2 * atan2(ax * py - ay * px, ax * px + ay * py);
  /* inside piece P -> Q: triangle */
  if (t2 > t1) area += 0.5 * (px * qy - py * qx);
  /* outside piece Q -> B: sector */
  if (t2 < 1.0) area += 0.5 * r2 * atan2(qx * by - qy * bx, qx * bx + qy * by);
  return area;
}

typedef struct {
  double c[3];
  double Q[9];   /* (p-c)^T Q (p-c) <= 1 */
  double W[9];   /* Q^{-1} */
  double Q2inv[4];
  double Lt[4];  /* L^T where Q2 = L L^T (upper triangular) */
  double detL;
  double s;      /* Qzz - q^T Q2^{-1} q */
  double lam_min;
} body_t;

static void inv3(const double *A, double *B) {
  double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
               A[2] * (A[3] * A[7] - A[4] * A[6]);
  B[0] = (A[4] * A[8] - A[5] * A[7]) / det;
  B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
  B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
  B[3] = (A[5] * A[6] - A[3] * A[8]) / det;
  B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
  B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
  B[6] = (A[3] * A[7] - A[4] * A[6]) / det;
  B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
  B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
}

static void body_setup(body_t *b, const double *c, const double *Q) {
  memcpy(b->c, c, sizeof(double) * 3);
  memcpy(b->Q, Q, sizeof(double) * 9);
  inv3(Q, b->W);
  double a = Q[0], bb = Q[1], d = Q[4];
  double det2 = a * d - bb * bb;
  b->Q2inv[0] = d / det2;
  b->Q2inv[1] = -bb / det2;
  b->Q2inv[2] = -bb / det2;
  b->Q2inv[3] = a / det2;
  double qx = Q[2], qy = Q[5];
  b->s = Q[8] - (qx * (b->Q2inv[0] * qx + b->Q2inv[1] * qy) + qy * (b->Q2inv[2] * qx + b->Q2inv[3] * qy));
  /* Cholesky of Q2 = L L^T, L lower: L00 = sqrt(a), L10 = bb/L00, L11 = sqrt(d - L10^2) */
  double L00 = sqrt(a), L10 = bb / L00, L11 = sqrt(d - L10 * L10);
  b->Lt[0] = L00;
  b->Lt[1] = L10;
  b->Lt[2] = 0.0;
  b->Lt[3] = L11;
  b->detL = L00 * L11;
  /* smallest eigenvalue lower bound via Gershgorin, clamped positive */
  double lm = 1e300;
  for (int r = 0; r < 3; ++r) {
    double g = Q[4 * r];
    for (int k = 0; k < 3; ++k)
      if (k != r) g -= fabs(Q[3 * r + k]);
    if (g < lm) lm = g;
  }
  /* 1/trace(Q^{-1}) is another lower bound; keep the larger */
  double lt = 1.0 / (b->W[0] + b->W[4] + b->W[8]);
  b->lam_min = lm > lt ? lm : lt;
}

/* Exact area of the slice z of body b inside [x0,x1]x[y0,y1]. */
static double slice_area(const body_t *b, double z, double x0, double x1, double y0, double y1) {
  double dz = z - b->c[2];
  double rho2 = 1.0 - dz * dz * b->s;
  if (rho2 <= 0.0) return 0.0;
  double qx = b->Q[2], qy = b->Q[5];
  double mx = b->c[0] - dz * (b->Q2inv[0] * qx + b->Q2inv[1] * qy);
  double my = b->c[1] - dz * (b->Q2inv[2] * qx + b->Q2inv[3] * qy);
  double px[4] = {x0 - mx, x1 - mx, x1 - mx, x0 - mx};
  double py[4] = {y0 - my, y0 - my, y1 - my, y1 - my};
  double wx[4], wy[4];
  for (int k = 0; k < 4; ++k) {
    wx[k] = b->Lt[0] * px[k] + b->Lt[1] * py[k];
    wy[k] = b->Lt[2] * px[k] + b->Lt[3] * py[k];
  }
  double r = sqrt(rho2);
  double area = 0.0;
  for (int k = 0; k < 4; ++k) {
    int k1 = (k + 1) & 3;
    area += tri_disc(r, wx[k], wy[k], wx[k1], wy[k1]);
  }
  return area / b->detL;
}

static int add_roots(double qa, double qb, double qc, double zc, double lo, double hi, double *out, int n) {
  /* roots of qa t^2 + qb t + qc = 0, z = zc + t, kept if inside (lo,hi) */
  if (qa == 0.0) return n;
  double disc = qb * qb - 4.0 * qa * qc;
  if (disc < 0.0) return n;
  double sq = sqrt(disc);
  double t1 = (-qb - sq) / (2.0 * qa), t2 = (-qb + sq) / (2.0 * qa);
  double z1 = zc + t1, z2 = zc + t2;
  if (z1 > lo && z1 < hi) out[n++] = z1;
  if (z2 > lo && z2 < hi) out[n++] = z2;
  return n;
}

static int cmp_dbl_q(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/* Volume of body b inside the cell [x0,x0+1]x[y0,y0+1]x[z0,z0+1]. */
static double cell_fraction(const body_t *b, double x0, double y0, double z0) {
  double x1 = x0 + 1.0, y1 = y0 + 1.0, z1 = z0 + 1.0;
  /* corner test: all corners inside => fully inside (convexity) */
  int inside = 0;
  for (int k = 0; k < 8; ++k) {
    double p[3] = {((k & 1) ? x1 : x0) - b->c[0], ((k & 2) ? y1 : y0) - b->c[1], ((k & 4) ? z1 : z0) - b->c[2]};
    double f = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) f += p[r] * b->Q[3 * r + s] * p[s];
    if (f <= 1.0) inside++;
  }
  if (inside == 8) return 1.0;
  /* distance lower bound => fully outside */
  double ddx = fmax(fmax(x0 - b->c[0], b->c[0] - x1), 0.0);
  double ddy = fmax(fmax(y0 - b->c[1], b->c[1] - y1), 0.0);
  double ddz = fmax(fmax(z0 - b->c[2], b->c[2] - z1), 0.0);
  if (b->lam_min * (ddx * ddx + ddy * ddy + ddz * ddz) > 1.0) return 0.0;
  /* z extent of the body */
  double hz = sqrt(b->W[8]);
  double lo = fmax(z0, b->c[2] - hz), hi = fmin(z1, b->c[2] + hz);
  if (lo >= hi) return 0.0;
  double bp[40];
  int nbp = 0;
  bp[nbp++] = lo;
  /* tangency with the lines x = x0, x1: projection on (x,z) */
  {
    double a = b->W[0], c = b->W[8], bb = b->W[2];
    double det = a * c - bb * bb; /* projected ellipse matrix = inv([[a,bb],[bb,c]]) */
    double P00 = c / det, P01 = -bb / det, P11 = a / det;
    double xs[2] = {x0, x1};
    for (int k = 0; k < 2; ++k) {
      double dx = xs[k] - b->c[0];
      nbp = add_roots(P11, 2.0 * P01 * dx, P00 * dx * dx - 1.0, b->c[2], lo, hi, bp, nbp);
    }
  }
  {
    double a = b->W[4], c = b->W[8], bb = b->W[5];
    double det = a * c - bb * bb;
    double P00 = c / det, P01 = -bb / det, P11 = a / det;
    double ys[2] = {y0, y1};
    for (int k = 0; k < 2; ++k) {
      double dy = ys[k] - b->c[1];
      nbp = add_roots(P11, 2.0 * P01 * dy, P00 * dy * dy - 1.0, b->c[2], lo, hi, bp, nbp);
    }
  }
  /* corner lines parallel to z */
  for (int k = 0; k < 4; ++k) {
    double dx = ((k & 1) ? x1 : x0) - b->c[0];
    double dy = ((k & 2) ? y1 : y0) - b->c[1];
    const double *Q = b->Q;
    double qa = Q[8];
    double qb = 2.0 * (Q[2] * dx + Q[5] * dy);
    double qc = Q[0] * dx * dx + 2.0 * Q[1] * dx * dy + Q[4] * dy * dy - 1.0;
    nbp = add_roots(qa, qb, qc, b->c[2], lo, hi, bp, nbp);
  }
  bp[nbp++] = hi;
  qsort(bp, nbp, sizeof(double), cmp_dbl_q);
  double vol = 0.0;
  for (int s = 0; s + 1 < nbp; ++s) {
    double a = bp[s], h = bp[s + 1] - bp[s];
    if (h <= 0.0) continue;
    double acc = 0.0;
    for (int q = 0; q < gl_n; ++q) {
      double t = gl_x[q];
      double S = t * t * (3.0 - 2.0 * t), dS = 6.0 * t * (1.0 - t);
      acc += gl_w[q] * dS * slice_area(b, a + h * S, x0, x1, y0, y1);
    }
    vol += h * acc;
  }
  if (vol < 0.0) vol = 0.0;
  if (vol > 1.0) vol = 1.0;
  return vol;
}

/*
 * Accumulate the volume fractions of `nb` ellipsoids into field[t][nz][ny][nx]
 * (x fastest), where body i goes to tracer tracer_of[i]. Body i is
 * {p : (p - centre_i)^T Q_i (p - centre_i) <= 1} with Q_i = Qs[9*i..9*i+8]
 * (row-major, symmetric positive definite); the grid is tri-periodic, so
 * bodies straddling a face wrap round. Planes are distributed over threads;
 * within one cell the contributions are added in body order, so the result is
 * deterministic. `order` is the Gauss-Legendre order per smooth z-segment.
 */
int synth_fill_ellipsoids(int nx, int ny, int nz, double *field, int nb, const double *centres,
                          const double *Qs, const int *tracer_of, int order) {
  if (order < 2 || order > GL_MAX) return -1;
  gl_init(order);
  body_t *bodies = (body_t *)malloc(sizeof(body_t) * (nb > 0 ? nb : 1));
  int *zlo = (int *)malloc(sizeof(int) * (nb > 0 ? nb : 1));
  int *zhi = (int *)malloc(sizeof(int) * (nb > 0 ? nb : 1));
  for (int i = 0; i < nb; ++i) {
    body_setup(&bodies[i], centres + 3 * i, Qs + 9 * i);
    double hz = sqrt(bodies[i].W[8]);
    zlo[i] = (int)floor(bodies[i].c[2] - hz);
    zhi[i] = (int)floor(bodies[i].c[2] + hz);
    /* a body wider than the box would overlap its own periodic images */
    if (2.0 * sqrt(bodies[i].W[0]) >= nx - 1 || 2.0 * sqrt(bodies[i].W[4]) >= ny - 1 || 2.0 * hz >= nz - 1) {
      free(bodies);
      free(zlo);
      free(zhi);
      return -2;
    }
  }
  const int64_t plane = (int64_t)nx * ny;
  const int64_t vol = plane * nz;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < nz; ++k) {
    for (int i = 0; i < nb; ++i) {
      const body_t *b = &bodies[i];
      /* unwrapped planes kk with kk mod nz == k inside [zlo, zhi] */
      int kk0 = zlo[i] + (((k - zlo[i]) % nz) + nz) % nz;
      for (int kk = kk0; kk <= zhi[i]; kk += nz) {
        double hx = sqrt(b->W[0]), hy = sqrt(b->W[4]);
        int ilo = (int)floor(b->c[0] - hx), ihi = (int)floor(b->c[0] + hx);
        int jlo = (int)floor(b->c[1] - hy), jhi = (int)floor(b->c[1] + hy);
        double *f = field + (int64_t)tracer_of[i] * vol + (int64_t)k * plane;
        for (int jj = jlo; jj <= jhi; ++jj) {
          int j = ((jj % ny) + ny) % ny;
          for (int ii = ilo; ii <= ihi; ++ii) {
            int x = ((ii % nx) + nx) % nx;
            double v = cell_fraction(b, (double)ii, (double)jj, (double)kk);
            if (v != 0.0) f[(int64_t)j * nx + x] += v;
          }
        }
      }
    }
  }
  free(bodies);
  free(zlo);
  free(zhi);
  return 0;
}

/* Volume fraction of one body in one cell (for tests of the generator). */
double synth_cell_fraction(const double *centre, const double *Q, double x0, double y0, double z0, int order) {
  body_t b;
  gl_init(order);
  body_setup(&b, centre, Q);
  return cell_fraction(&b, x0, y0, z0);
}

/*
 * Accumulate the volume fractions of infinite circular cylinders parallel to
 * z (axis through (cx, cy), radius r) into field[t][nz][ny][nx]: the fraction
 * of every cell is the exact area of the disc inside the cell's xy-square.
 */
int synth_fill_cylinders_z(int nx, int ny, int nz, double *field, int nb, const double *centres_xy,
                           const double *radii, const int *tracer_of) {
  const int64_t plane = (int64_t)nx * ny;
  const int64_t vol = plane * nz;
  for (int b = 0; b < nb; ++b) {
    double cx = centres_xy[2 * b], cy = centres_xy[2 * b + 1], r = radii[b];
    if (2.0 * r >= nx - 1 || 2.0 * r >= ny - 1) return -2;
    int ilo = (int)floor(cx - r), ihi = (int)floor(cx + r);
    int jlo = (int)floor(cy - r), jhi = (int)floor(cy + r);
    for (int jj = jlo; jj <= jhi; ++jj)
      for (int ii = ilo; ii <= ihi; ++ii) {
        double x0 = ii - cx, x1 = ii + 1 - cx, y0 = jj - cy, y1 = jj + 1 - cy;
        double px[4] = {x0, x1, x1, x0}, py[4] = {y0, y0, y1, y1};
        double a = 0.0;
        for (int k = 0; k < 4; ++k) a += tri_disc(r, px[k], py[k], px[(k + 1) & 3], py[(k + 1) & 3]);
        if (a == 0.0) continue;
        int x = ((ii % nx) + nx) % nx, y = ((jj % ny) + ny) % ny;
        double *f = field + (int64_t)tracer_of[b] * vol + (int64_t)y * nx + x;
        for (int k = 0; k < nz; ++k) f[(int64_t)k * plane] += a;
      }
  }
  return 0;
}
