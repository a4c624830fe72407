/*
 * Oracle (test infrastructure only): the learned con2prim starting guess.
 *
 * The paper recovers primitives by two bracketed root solves (App. D).  The
 * learned variant predicts starting guesses for both roots with a small MLP
 * 8 -> 64 -> 64 -> 2 (ReLU) and polishes them by Newton's method; the plain
 * solver decides the answer.  This file is the plain FP64 version
 * of the network part:
 *
 *   features   8 metric-invariant scalars of one state (con2prim depends on
 *              the metric only through q, r^2, calB^2, (r.calB), App. D step 1)
 *   targets    log(mu_+ h0) and log(mu / mu_+) of the plain solver's roots, less
 *              closed-form approximations of both (orc_mlp_baseline)
 *   forward    y = W3 relu(W2 relu(W1 z + b1) + b2) + b3, z the standardized
 *              features
 *   gradient   of L = 1/(2n) sum_samples sum_o (y_o - t_o)^2 by backpropagation
 *              (rows whose first feature is NaN, points without a state, are
 *              skipped but still counted in n; the forward pass gives NaN there)
 *   Adam       one step (Kingma & Ba, 2015, Algorithm 1)
 *
 * With emulate = 1 the forward and backward passes round to bfloat16 and to
 * binary32 at the places where the device kernels do (inputs of every matrix
 * product in bf16, products accumulated exactly, then rounded to binary32,
 * biases added in binary32); with emulate = 0 everything is FP64.
 *
 * Parameter block layout (the same offsets as the library's): W1 [64][8] at
 * 0, b1 [64] at 512, W2 [64][64] at 576, b2 [64] at 4672, W3 [2][64] at 4736,
 * b3 [2] at 4864, feature mean [8] at 4866, inverse std [8] at 4874; 4882 in
 * all, the first 4866 trainable.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include "orc.h"

#define NI 8
#define NH 64
#define NO 2
#define OW1 0
#define OB1 512
#define OW2 576
#define OB2 4672
#define OW3 4736
#define OB3 4864
#define OMEAN 4866
#define OISTD 4874
#define NTRAIN 4866

/* binary32 -> bfloat16 by round-to-nearest-even on the upper 16 bits
 * (NaN kept quiet), returned widened back to binary32 */
float orc_bf16(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
    u |= 0x00400000u;
  } else {
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
  }
  u &= 0xffff0000u;
  memcpy(&x, &u, 4);
  return x;
}

static double q_bf(double v, int emulate) { return emulate ? (double)orc_bf16((float)v) : v; }
static double q_f32(double v, int emulate) { return emulate ? (double)(float)v : v; }

void orc_mlp_features(const double cons[6], const double B[3], const double gdn[6],
                      const double gup[6], double x[8]) {
  double D = cons[0], q = cons[2] / cons[0], r[3], ru[3], cB[3], cBd[3], r2, B2, rB, onep;
  int i;
  for (i = 0; i < 3; ++i) {
    r[i] = cons[3 + i] / D;
    cB[i] = B[i] / sqrt(D);
  }
  ru[0] = gup[0] * r[0] + gup[1] * r[1] + gup[2] * r[2];
  ru[1] = gup[1] * r[0] + gup[3] * r[1] + gup[4] * r[2];
  ru[2] = gup[2] * r[0] + gup[4] * r[1] + gup[5] * r[2];
  cBd[0] = gdn[0] * cB[0] + gdn[1] * cB[1] + gdn[2] * cB[2];
  cBd[1] = gdn[1] * cB[0] + gdn[3] * cB[1] + gdn[4] * cB[2];
  cBd[2] = gdn[2] * cB[0] + gdn[4] * cB[1] + gdn[5] * cB[2];
  r2 = ru[0] * r[0] + ru[1] * r[1] + ru[2] * r[2];
  B2 = cB[0] * cBd[0] + cB[1] * cBd[1] + cB[2] * cBd[2];
  rB = r[0] * cB[0] + r[1] * cB[1] + r[2] * cB[2];
  onep = 1.0 + q;
  x[0] = log10(D);
  x[1] = log10(fmax(q, 1e-30));
  x[2] = log10(r2 + 1e-30);
  x[3] = log10(B2 + 1e-30);
  x[4] = rB * rB / (r2 * B2 + 1e-300);
  x[5] = log10(onep);
  x[6] = log10(r2 / (onep * onep) + 1e-30);
  x[7] = log10(B2 / onep + 1e-30);
}

/* Closed-form approximations of the two log fractions, which the network
 * corrects.  Without a magnetic field (calB = 0, so rbar^2 = r^2 for every mu,
 * App. D) the auxiliary root solves mu sqrt(h0^2 + r^2) = 1 exactly:
 *   b0 = log(h0) - log(h0^2 + r^2) / 2.
 * The second root mu = 1/(h W) is taken as 1/(1 + q), since D (1 + q) = tau + D
 * is the energy density, about rho h W^2 for a cold, weakly magnetised fluid:
 *   b1 = -log(1 + q) + log(h0^2 + r^2) / 2.
 * cons = (D, Y_e D, tau, S_i) undensitized, gup the inverse physical metric. */
void orc_mlp_baseline(double h0, const double cons[6], const double gup[6], double b[2]) {
  const double D = cons[0], q = cons[2] / D;
  static const int sym[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}}; /* xx xy xz yy yz zz */
  double r[3], r2 = 0.0;
  int i, j;
  for (i = 0; i < 3; ++i) r[i] = cons[3 + i] / D;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) r2 += gup[sym[i][j]] * r[i] * r[j];
  b[0] = log(h0) - 0.5 * log(h0 * h0 + r2);
  b[1] = -log(1.0 + q) + 0.5 * log(h0 * h0 + r2);
}

/* the roots as fractions of their upper bounds, in log space (log(mu_+ h0)
 * and log(mu / mu_+), both <= 0), less the baseline b */
void orc_mlp_targets(double h0, const double b[2], const double mu[2], double t[2]) {
  t[0] = log(mu[0] * h0) - b[0];
  t[1] = log(mu[1] / mu[0]) - b[1];
}

/* one sample through the network; keeps the intermediate values for backprop */
typedef struct {
  double xb[NI], a1[NH], h1b[NH], a2[NH], h2[NH], y[NO];
} mlp_trace;

static void forward_one(const double* prm, const float* x, int emulate, mlp_trace* t) {
  int n, k, o;
  for (k = 0; k < NI; ++k) {
    double z;
    if (emulate) {
      float zf = ((float)x[k] - (float)prm[OMEAN + k]) * (float)prm[OISTD + k];
      z = (double)orc_bf16(zf);
    } else {
      z = ((double)x[k] - prm[OMEAN + k]) * prm[OISTD + k];
    }
    t->xb[k] = z;
  }
  for (n = 0; n < NH; ++n) {
    double s = 0.0;
    for (k = 0; k < NI; ++k) s += q_bf(prm[OW1 + n * NI + k], emulate) * t->xb[k];
    s = q_f32(s, emulate);
    t->a1[n] = q_f32(s + prm[OB1 + n], emulate);
    t->h1b[n] = q_bf(t->a1[n] > 0.0 ? t->a1[n] : 0.0, emulate);
  }
  for (n = 0; n < NH; ++n) {
    double s = 0.0;
    for (k = 0; k < NH; ++k) s += q_bf(prm[OW2 + n * NH + k], emulate) * t->h1b[k];
    s = q_f32(s, emulate);
    t->a2[n] = q_f32(s + prm[OB2 + n], emulate);
    t->h2[n] = t->a2[n] > 0.0 ? t->a2[n] : 0.0;
  }
  for (o = 0; o < NO; ++o) {
    double s = 0.0;
    for (n = 0; n < NH; ++n) s += prm[OW3 + o * NH + n] * t->h2[n];
    t->y[o] = s + prm[OB3 + o];
  }
}

void orc_mlp_forward(const double* prm, const float* X, int64_t n, int emulate, double* Y) {
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < n; ++i) {
    mlp_trace t;
    if (isnan(X[i * NI])) {
      Y[i * NO] = Y[i * NO + 1] = NAN;
      continue;
    }
    forward_one(prm, X + i * NI, emulate, &t);
    Y[i * NO] = t.y[0];
    Y[i * NO + 1] = t.y[1];
  }
}

/* grad[0..NTRAIN) += dL/dtheta over the n samples; returns L */
double orc_mlp_grad(const double* prm, const float* X, const float* T, int64_t n, int emulate,
                    double* grad) {
  double loss = 0.0;
  int64_t i;
  for (i = 0; i < n; ++i) {
    mlp_trace t;
    double dy[NO], g2[NH], g1[NH];
    int o, j, k;
    if (isnan(X[i * NI])) continue;  /* rows without a state (atmosphere) carry no loss */
    forward_one(prm, X + i * NI, emulate, &t);
    for (o = 0; o < NO; ++o) {
      double r = t.y[o] - (double)T[i * NO + o];
      loss += 0.5 * r * r / (double)n;
      dy[o] = q_f32(r / (double)n, emulate);
    }
    for (o = 0; o < NO; ++o) {
      for (j = 0; j < NH; ++j) grad[OW3 + o * NH + j] += dy[o] * t.h2[j];
      grad[OB3 + o] += dy[o];
    }
    for (j = 0; j < NH; ++j) {
      double s = 0.0;
      for (o = 0; o < NO; ++o) s += dy[o] * prm[OW3 + o * NH + j];
      s = q_f32(s, emulate);
      g2[j] = t.a2[j] > 0.0 ? s : 0.0;
      grad[OB2 + j] += g2[j];
      g2[j] = q_bf(g2[j], emulate);
    }
    for (j = 0; j < NH; ++j)
      for (k = 0; k < NH; ++k) grad[OW2 + j * NH + k] += g2[j] * t.h1b[k];
    for (k = 0; k < NH; ++k) {
      double s = 0.0;
      for (j = 0; j < NH; ++j) s += g2[j] * q_bf(prm[OW2 + j * NH + k], emulate);
      s = q_f32(s, emulate);
      g1[k] = t.a1[k] > 0.0 ? s : 0.0;
      grad[OB1 + k] += g1[k];
      g1[k] = q_bf(g1[k], emulate);
    }
    for (k = 0; k < NH; ++k)
      for (j = 0; j < NI; ++j) grad[OW1 + k * NI + j] += g1[k] * t.xb[j];
  }
  return loss;
}

/* one Adam step on the trainable parameters; `step` counts from 1 */
void orc_mlp_adam(double* prm, const double* grad, double* m, double* v, int step, double lr,
                  double beta1, double beta2, double eps) {
  int i;
  double c1 = 1.0 - pow(beta1, step), c2 = 1.0 - pow(beta2, step);
  for (i = 0; i < NTRAIN; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
    prm[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}
