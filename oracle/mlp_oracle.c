/*
 * CPU FP64 ORACLE FOR THE LEARNED CURVATURE -- TEST INFRASTRUCTURE ONLY.
 *
 * Not in the paper: the paper computes curvature with the method of a single
 * tracer (height functions). The learned estimator is a small multilayer
 * perceptron on 3x3x3 volume-fraction stencils,
 *   input 27 values (zero-padded to 32) -> 128 -> 128 -> 1, ReLU,
 * predicting kappa*Delta. This file is the reference implementation of its
 * arithmetic, written from that definition:
 *   - the two matrix products (layers 1 and 2) and the three of the backward
 *     pass take BF16 operands: weights are FP32 masters rounded to BF16 (round
 *     to nearest even) for each use; the first-layer activations and the
 *     upstream gradients are rounded to BF16; each input value x is carried
 *     as the sum of two BF16 numbers, hi = bf16(x) and lo = bf16(x - hi), both
 *     multiplied by the same weights (about 16 significant bits);
 *   - the last layer (128 -> 1) is a plain FP32 dot product: the second-layer
 *     activations and W3 are not rounded to BF16;
 *   - products and sums are accumulated here in FP64 (the GPU accumulates in
 *     FP32: the tests allow the FP32 bound);
 *   - an activation is rounded to FP32 before its BF16 rounding, as on the GPU;
 *   - ReLU'(z) is taken as (activation > 0), the activation as used;
 *   - loss: mean over the batch of (y - t)^2 / max(|t|, 0.05)^2;
 *   - Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 masters.
 * With exact = 1 no rounding is applied at all (pure FP64), which is what the
 * finite-difference pin of the backward pass uses.
 *
 * Stencil canonicalisation (the 48 symmetries of the cube and the exchange of
 * the phases): if the centre value exceeds 1/2 replace every c by 1 - c, which
 * flips the sign of the curvature; then reflect the axes along which the MYC
 * normal of that block is negative and order the axes by increasing |m|
 * (ties: lower axis first). Reflections and axis permutations leave the
 * curvature unchanged.
 *
 * Parameter layout (FP32): W1[32][128] (input k, unit j), b1[128],
 * W2[128][128], b2[128], W3[128], b3, then 3 floats of padding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int orc_myc_normal(const double *b, double *m_out);
int orc_myc_normal_sigma(const double *b, double *m_out, double *sigma_out);

#define NIN 32
#define NH 128
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NIN * NH)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NH)
#define NPARAMS (OFF_B3 + 4)

int orc_mlp_nparams(void) { return NPARAMS; }

/* FP32 -> BF16 -> FP32, round to nearest even (finite inputs). */
float orc_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return f; /* inf / nan unchanged */
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  u &= 0xffff0000u;
  float r;
  memcpy(&r, &u, 4);
  return r;
}

static double rnd(double v, int exact) { return exact ? v : (double)orc_bf16((float)v); }

/* An input value as the matrix cores see it: hi + lo, two BF16 numbers. */
static double rnd_in(double v, int exact) {
  if (exact) return v;
  float f = (float)v;
  float hi = orc_bf16(f);
  float lo = orc_bf16(f - hi); /* f - hi is exact in FP32 */
  return (double)hi + (double)lo;
}

/* Canonical stencil of a 3x3x3 block b[(ax+1)+3(ay+1)+9(az+1)] (FP64), written
 * as 27 FP32 values; returns +1 or -1, the sign that maps the network output
 * back to the original orientation. Order of the steps: complement (when the
 * centre exceeds 1/2), then the MYC normal of the complemented block decides
 * the reflections and the axis order, so that every canonical stencil has its
 * centre at most 1/2 and a normal with non-negative components in ascending
 * order. */
int orc_canonical_stencil(const double *b, float *x27) {
  int sign = (b[13] > 0.5) ? -1 : 1;
  double bc[27];
  for (int q = 0; q < 27; ++q) bc[q] = (sign < 0) ? 1.0 - b[q] : b[q];
  double m[3];
  orc_myc_normal(bc, m);
  int ord[3] = {0, 1, 2};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (fabs(m[ord[j]]) < fabs(m[ord[i]]) || (fabs(m[ord[j]]) == fabs(m[ord[i]]) && ord[j] < ord[i])) {
        int t = ord[i];
        ord[i] = ord[j];
        ord[j] = t;
      }
  /* canonical offset q along canonical axis k reads original axis ord[k],
   * reflected where the normal is negative */
  for (int q2 = -1; q2 <= 1; ++q2)
    for (int q1 = -1; q1 <= 1; ++q1)
      for (int q0 = -1; q0 <= 1; ++q0) {
        int q[3] = {q0, q1, q2};
        int a[3];
        for (int k = 0; k < 3; ++k) a[ord[k]] = (m[ord[k]] < 0.0) ? -q[k] : q[k];
        x27[(q0 + 1) + 3 * (q1 + 1) + 9 * (q2 + 1)] = (float)bc[(a[0] + 1) + 3 * (a[1] + 1) + 9 * (a[2] + 1)];
      }
  return sign;
}

/* Whether the 3x3x3 block b holds two interfaces, the second trigger of the
 * height-function fallback: on the block as canonicalised (complemented when
 * its centre exceeds 1/2), the centred-columns orientation sigma of MYC along
 * the first axis the height functions try -- the axis of the largest |m_d|,
 * ties to the lower axis -- disagrees with the orientation the height
 * functions take there (full end on the low side when m_d >= 0). One planar
 * interface gives the same side both ways; a second interface in the block
 * can make the column sums and the normal point to opposite sides. */
int orc_two_interfaces(const double *b) {
  const int flip = b[13] > 0.5;
  double bc[27];
  for (int q = 0; q < 27; ++q) bc[q] = flip ? 1.0 - b[q] : b[q];
  double m[3], sg[3];
  orc_myc_normal_sigma(bc, m, sg);
  int d = 0;
  for (int k = 1; k < 3; ++k)
    if (fabs(m[k]) > fabs(m[d])) d = k;
  return (sg[d] > 0.0) != (m[d] >= 0.0);
}

/* Forward pass for one sample. x: 27 FP32. Outputs y and, if wanted, the
 * activations h1[128], h2[128] (as used by the next layer) and the
 * pre-activations z1, z2. */
static double forward1(const float *P, const float *x, int exact, double *h1, double *h2, double *z1, double *z2) {
  double xb[NIN];
  for (int k = 0; k < NIN; ++k) xb[k] = (k < 27) ? rnd_in((double)x[k], exact) : 0.0;
  for (int j = 0; j < NH; ++j) {
    double acc = 0.0;
    for (int k = 0; k < NIN; ++k) acc += xb[k] * rnd((double)P[OFF_W1 + k * NH + j], exact);
    acc += (double)P[OFF_B1 + j];
    z1[j] = acc;
    h1[j] = rnd(acc > 0.0 ? acc : 0.0, exact);
  }
  for (int j = 0; j < NH; ++j) {
    double acc = 0.0;
    for (int k = 0; k < NH; ++k) acc += h1[k] * rnd((double)P[OFF_W2 + k * NH + j], exact);
    acc += (double)P[OFF_B2 + j];
    z2[j] = acc;
    h2[j] = acc > 0.0 ? acc : 0.0;
  }
  double y = 0.0;
  for (int k = 0; k < NH; ++k) y += h2[k] * (double)P[OFF_W3 + k];
  y += (double)P[OFF_B3];
  return y;
}

void orc_mlp_forward(const float *P, int n, const float *x, int exact, double *y, double *acts) {
  double h1[NH], h2[NH], z1[NH], z2[NH];
  for (int i = 0; i < n; ++i) {
    y[i] = forward1(P, x + 27 * (int64_t)i, exact, h1, h2, z1, z2);
    if (acts) {
      for (int j = 0; j < NH; ++j) {
        acts[512 * (int64_t)i + j] = h1[j];
        acts[512 * (int64_t)i + NH + j] = h2[j];
        acts[512 * (int64_t)i + 2 * NH + j] = z1[j];
        acts[512 * (int64_t)i + 3 * NH + j] = z2[j];
      }
    }
  }
}

static double loss_weight(double t) {
  double a = fabs(t) > 0.05 ? fabs(t) : 0.05;
  return 1.0 / (a * a);
}

/* Loss and gradient of the batch loss with respect to every parameter.
 * The upstream gradients dz2, dz1 are rounded like activations (unless
 * exact). grad: NPARAMS FP64. Returns the loss. */
double orc_mlp_grad(const float *P, int n, const float *x, const float *t, int exact, double *grad) {
  memset(grad, 0, sizeof(double) * NPARAMS);
  double h1[NH], h2[NH], z1[NH], z2[NH], dz2[NH], dz1[NH];
  double loss = 0.0;
  for (int i = 0; i < n; ++i) {
    const float *xi = x + 27 * (int64_t)i;
    double y = forward1(P, xi, exact, h1, h2, z1, z2);
    double ti = (double)t[i];
    double w = loss_weight(ti);
    loss += (y - ti) * (y - ti) * w;
    double g = 2.0 * (y - ti) * w / (double)n;
    /* layer 3 */
    for (int k = 0; k < NH; ++k) grad[OFF_W3 + k] += g * h2[k];
    grad[OFF_B3] += g;
    for (int k = 0; k < NH; ++k) {
      double d = (h2[k] > 0.0) ? g * (double)P[OFF_W3 + k] : 0.0;
      dz2[k] = rnd(d, exact);
    }
    /* layer 2 */
    for (int k = 0; k < NH; ++k)
      for (int j = 0; j < NH; ++j) grad[OFF_W2 + k * NH + j] += h1[k] * dz2[j];
    for (int j = 0; j < NH; ++j) grad[OFF_B2 + j] += dz2[j];
    for (int k = 0; k < NH; ++k) {
      double acc = 0.0;
      for (int j = 0; j < NH; ++j) acc += dz2[j] * rnd((double)P[OFF_W2 + k * NH + j], exact);
      dz1[k] = rnd((h1[k] > 0.0) ? acc : 0.0, exact);
    }
    /* layer 1 */
    double xb[NIN];
    for (int k = 0; k < NIN; ++k) xb[k] = (k < 27) ? rnd_in((double)xi[k], exact) : 0.0;
    for (int k = 0; k < NIN; ++k)
      for (int j = 0; j < NH; ++j) grad[OFF_W1 + k * NH + j] += xb[k] * dz1[j];
    for (int j = 0; j < NH; ++j) grad[OFF_B1 + j] += dz1[j];
  }
  return loss / (double)n;
}

/* One Adam step in FP64 on FP32 masters (step is 1-based). */
void orc_adam(float *P, float *M, float *V, const double *grad, int step, double lr) {
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (int i = 0; i < NPARAMS; ++i) {
    double m = b1 * (double)M[i] + (1.0 - b1) * grad[i];
    double v = b2 * (double)V[i] + (1.0 - b2) * grad[i] * grad[i];
    M[i] = (float)m;
    V[i] = (float)v;
    double mh = m / c1, vh = v / c2;
    P[i] = (float)((double)P[i] - lr * mh / (sqrt(vh) + eps));
  }
}

/* One layer on supplied inputs (for layer-by-layer comparison):
 *   layer 1: in [n][27] (split into hi + lo here), out [n][128], act rounded;
 *   layer 2: in [n][128] (rounded to BF16 here), out [n][128], act not rounded;
 *   layer 3: in [n][128], out [n] (no activation, no rounding, FP32 W3).
 * pre: the pre-activation z = sum(in * W) + b; act: ReLU(z), rounded after
 * layer 1 (layer 3: act = pre); absacc: sum |in * W| + |b|, the scale of the
 * accumulation-error bound. Any output may be NULL. */
void orc_mlp_layer(const float *P, int layer, int n, const double *in, int exact, double *pre, double *act,
                   double *absacc) {
  int nin = layer == 1 ? 27 : NH, nout = layer == 3 ? 1 : NH;
  int woff = layer == 1 ? OFF_W1 : layer == 2 ? OFF_W2 : OFF_W3;
  int boff = layer == 1 ? OFF_B1 : layer == 2 ? OFF_B2 : OFF_B3;
  int wstride = layer == 3 ? 1 : NH;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < nout; ++j) {
      double acc = 0.0, aabs = 0.0;
      for (int k = 0; k < nin; ++k) {
        double a = layer == 1 ? rnd_in(in[(int64_t)i * nin + k], exact)
                   : layer == 2 ? rnd(in[(int64_t)i * nin + k], exact) : in[(int64_t)i * nin + k];
        double w = layer == 3 ? (double)P[woff + k * wstride + j] : rnd((double)P[woff + k * wstride + j], exact);
        acc += a * w;
        aabs += fabs(a * w);
      }
      acc += (double)P[boff + j];
      aabs += fabs((double)P[boff + j]);
      int64_t o = (int64_t)i * nout + j;
      if (pre) pre[o] = acc;
      if (act) act[o] = layer == 3 ? acc : layer == 2 ? (acc > 0.0 ? acc : 0.0) : rnd(acc > 0.0 ? acc : 0.0, exact);
      if (absacc) absacc[o] = aabs;
    }
  }
}

/* Backward pass on supplied intermediates (for comparison against a run that
 * produced them): g [n] = dL/dy per sample; h1, h2, dz2_in, dz1_in [n][128].
 *   dz2_out = round(h2 > 0 ? g * W3 : 0)   (W3 FP32)
 *   dz1_out = round(h1 > 0 ? sum_j dz2_in_j * W2[k][j] : 0), dz1_abs its |.| scale
 *   grad    = dW1 = sum x dz1_in, db1 = sum dz1_in, dW2 = sum h1 dz2_in,
 *             db2 = sum dz2_in, dW3 = sum g h2, db3 = sum g (over the batch);
 *   grad_abs: the same sums of absolute values.
 * Any output may be NULL. */
void orc_mlp_backward_given(const float *P, int n, const float *x, const double *g, const double *h1,
                            const double *h2, const double *dz2_in, const double *dz1_in, int exact, double *dz2_out,
                            double *dz1_out, double *dz1_abs, double *grad, double *grad_abs) {
  if (grad) memset(grad, 0, sizeof(double) * NPARAMS);
  if (grad_abs) memset(grad_abs, 0, sizeof(double) * NPARAMS);
  for (int i = 0; i < n; ++i) {
    const double *a1 = h1 + (int64_t)i * NH, *a2 = h2 + (int64_t)i * NH;
    const double *d2 = dz2_in + (int64_t)i * NH, *d1 = dz1_in + (int64_t)i * NH;
    double xb[NIN];
    for (int k = 0; k < NIN; ++k) xb[k] = (k < 27) ? rnd_in((double)x[27 * (int64_t)i + k], exact) : 0.0;
    for (int k = 0; k < NH; ++k) {
      if (dz2_out)
        dz2_out[(int64_t)i * NH + k] = rnd(a2[k] > 0.0 ? g[i] * (double)P[OFF_W3 + k] : 0.0, exact);
      double acc = 0.0, aabs = 0.0;
      for (int j = 0; j < NH; ++j) {
        double t = d2[j] * rnd((double)P[OFF_W2 + k * NH + j], exact);
        acc += t;
        aabs += fabs(t);
      }
      if (dz1_out) dz1_out[(int64_t)i * NH + k] = rnd(a1[k] > 0.0 ? acc : 0.0, exact);
      if (dz1_abs) dz1_abs[(int64_t)i * NH + k] = aabs;
    }
    for (int pass = 0; pass < 2; ++pass) {
      double *G = pass == 0 ? grad : grad_abs;
      if (!G) continue;
#define T(v) (pass == 0 ? (v) : fabs(v))
      for (int k = 0; k < NH; ++k) G[OFF_W3 + k] += T(g[i] * a2[k]);
      G[OFF_B3] += T(g[i]);
      for (int k = 0; k < NH; ++k)
        for (int j = 0; j < NH; ++j) G[OFF_W2 + k * NH + j] += T(a1[k] * d2[j]);
      for (int j = 0; j < NH; ++j) G[OFF_B2 + j] += T(d2[j]);
      for (int k = 0; k < NIN; ++k)
        for (int j = 0; j < NH; ++j) G[OFF_W1 + k * NH + j] += T(xb[k] * d1[j]);
      for (int j = 0; j < NH; ++j) G[OFF_B1 + j] += T(d1[j]);
#undef T
    }
  }
}
