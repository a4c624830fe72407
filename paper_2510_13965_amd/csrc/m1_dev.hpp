// Device helpers of the grey M1 part shared by the RHS kernels (m1.hip) and
// the implicit collision solve (imex.hip): the Minerbo closure (Sec. 2.3),
// its root find in xi, and the Minerbo-interpolated speeds (App. B).
// Evaluated in one fixed order without FMA contraction.
#pragma once

#include "dev_common.hpp"

namespace mhd {

#pragma clang fp contract(off)

constexpr int kM1Closure = 0;  // workspace: P_ij of species s at 6 s + c
constexpr int kM1Flux = 18;    // fluxes and speed of (species s, axis d): 18 + 5 (3 s + d) + c, c = 4 speed
constexpr int kM1Fields = 63;
// with the number densities: their point fluxes (species s, axis d) at
// 63 + 3 s + d, and Gamma = W (E - F_i v^i)/J of species s at 72 + s
constexpr int kM1NFlux = 63;
constexpr int kM1Gamma = 72;
constexpr int kM1NFields = 75;

struct M1State {
  double E, F[3], Fu[3], F2, v[3], vd[3], W, vF;
};

__device__ __forceinline__ double m1_eddington(double xi) {
  return 1.0 / 3.0 + xi * xi * (6.0 - 2.0 * xi + 6.0 * xi * xi) / 15.0;
}

__device__ __forceinline__ void m1_state_init(M1State& s, double E, const double F[3], const double v[3], double W,
                                              const double gd[6], const double gu[6]) {
  s.E = E;
  s.W = W;
  s.F2 = 0.0;
  s.vF = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s.F[i] = F[i];
    s.v[i] = v[i];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s.Fu[i] = 0.0;
    s.vd[i] = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      s.Fu[i] += gu[sym(i, j)] * F[j];
      s.vd[i] += gd[sym(i, j)] * v[j];
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s.F2 += s.Fu[i] * F[i];
    s.vF += F[i] * v[i];
  }
}

// P_ij (symmetric storage), J, H_i and H_a H^a for Eddington factor chi
__device__ __forceinline__ void m1_closure_eval(const M1State& s, const double gd[6], const double gu[6], double chi,
                                                double P[6], double& J, double H[3], double& HH) {
  const double W = s.W, W2 = W * W;
  const double dthick = 1.5 * (1.0 - chi), dthin = 1.0 - dthick;
  const double Jth = 3.0 / (2.0 * W2 + 1.0) * ((2.0 * W2 - 1.0) * s.E - 2.0 * W2 * s.vF);
  double Hth[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    Hth[i] = s.F[i] / W + W * s.vd[i] / (2.0 * W2 + 1.0) * ((4.0 * W2 + 1.0) * s.vF - 4.0 * W2 * s.E);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const double thin = s.F2 > 0.0 ? s.E * s.F[i] * s.F[j] / s.F2 : 0.0;
      const double thick = 4.0 / 3.0 * Jth * W2 * s.vd[i] * s.vd[j] + W * (Hth[i] * s.vd[j] + Hth[j] * s.vd[i]) +
                           1.0 / 3.0 * Jth * gd[sym(i, j)];
      P[sym(i, j)] = dthin * thin + dthick * thick;
    }
  double Pv[3], vPv = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Pv[i] = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) Pv[i] += P[sym(i, j)] * s.v[j];
    vPv += s.v[i] * Pv[i];
  }
  J = W2 * (s.E - 2.0 * s.vF + vPv);
#pragma unroll
  for (int i = 0; i < 3; ++i) H[i] = W * (s.F[i] - Pv[i] - J * s.vd[i]);
  const double Hn = W * (J - s.E + s.vF);
  double hh = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) hh += gu[sym(i, j)] * H[i] * H[j];
  HH = hh - Hn * Hn;
}

// The root function of the closure, R(xi) = (xi^2 J^2 - H_a H^a)/E^2 with J
// and H of the closure at chi(xi), in closed form: P_ij is affine in d_thick
// (P = P^thin + d_thick (P^thick - P^thin)), and so are J, H_i and H_n, so
// J = Ja + d Jb and H_a H^a = c0 + c1 d + c2 d^2 with d = 3/2 (1 - chi(xi)).
// The coefficients are formed once per state; each evaluation is then a few
// operations instead of a closure evaluation (the same function up to
// rounding).
struct M1RCoef {
  double Ja, Jb, c0, c1, c2, E2;
};

__device__ __forceinline__ M1RCoef m1_rcoef(const M1State& s, const double gd[6], const double gu[6]) {
  const double W = s.W, W2 = W * W;
  const double Jth = 3.0 / (2.0 * W2 + 1.0) * ((2.0 * W2 - 1.0) * s.E - 2.0 * W2 * s.vF);
  double Hth[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    Hth[i] = s.F[i] / W + W * s.vd[i] / (2.0 * W2 + 1.0) * ((4.0 * W2 + 1.0) * s.vF - 4.0 * W2 * s.E);
  double Pa[6], Pb[6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const double thin = s.F2 > 0.0 ? s.E * s.F[i] * s.F[j] / s.F2 : 0.0;
      const double thick = 4.0 / 3.0 * Jth * W2 * s.vd[i] * s.vd[j] + W * (Hth[i] * s.vd[j] + Hth[j] * s.vd[i]) +
                           1.0 / 3.0 * Jth * gd[sym(i, j)];
      Pa[sym(i, j)] = thin;
      Pb[sym(i, j)] = thick - thin;
    }
  double Pva[3], Pvb[3], vPva = 0.0, vPvb = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Pva[i] = 0.0;
    Pvb[i] = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Pva[i] += Pa[sym(i, j)] * s.v[j];
      Pvb[i] += Pb[sym(i, j)] * s.v[j];
    }
    vPva += s.v[i] * Pva[i];
    vPvb += s.v[i] * Pvb[i];
  }
  M1RCoef c;
  c.Ja = W2 * (s.E - 2.0 * s.vF + vPva);
  c.Jb = W2 * vPvb;
  double Ha[3], Hb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Ha[i] = W * (s.F[i] - Pva[i] - c.Ja * s.vd[i]);
    Hb[i] = -W * (Pvb[i] + c.Jb * s.vd[i]);
  }
  const double Hna = W * (c.Ja - s.E + s.vF), Hnb = W * c.Jb;
  double aa = 0.0, ab = 0.0, bb = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      aa += gu[sym(i, j)] * Ha[i] * Ha[j];
      ab += gu[sym(i, j)] * Ha[i] * Hb[j];
      bb += gu[sym(i, j)] * Hb[i] * Hb[j];
    }
  c.c0 = aa - Hna * Hna;
  c.c1 = 2.0 * (ab - Hna * Hnb);
  c.c2 = bb - Hnb * Hnb;
  c.E2 = s.E * s.E;
  return c;
}

__device__ __forceinline__ double m1_R(const M1RCoef& c, double xi) {
  const double d = 1.5 * (1.0 - m1_eddington(xi));
  const double J = c.Ja + d * c.Jb;
  return (xi * xi * J * J - (c.c0 + d * (c.c1 + d * c.c2))) / c.E2;
}

// Brent's method on [a, b] with R(a) < 0 < R(b), to a bracket of a few ulp
__device__ double m1_brent(const M1RCoef& co, double a, double b, double fa, double fb) {
  double c = a, fc = fa, d = b - a, e = d;
  for (int it = 0; it < 200; ++it) {
    if ((fb > 0.0 && fc > 0.0) || (fb < 0.0 && fc < 0.0)) {
      c = a;
      fc = fa;
      d = b - a;
      e = d;
    }
    if (fabs(fc) < fabs(fb)) {
      a = b;
      b = c;
      c = a;
      fa = fb;
      fb = fc;
      fc = fa;
    }
    const double tol = 2.0 * 2.220446049250313e-16 * fabs(b) + 0.5 * 2.2250738585072014e-308;
    const double m = 0.5 * (c - b);
    if (fabs(m) <= tol || fb == 0.0) break;
    if (fabs(e) < tol || fabs(fa) <= fabs(fb)) {
      d = m;
      e = m;
    } else {
      double p, q, r, t = fb / fa;
      if (a == c) {
        p = 2.0 * m * t;
        q = 1.0 - t;
      } else {
        q = fa / fc;
        r = fb / fc;
        p = t * (2.0 * m * q * (q - r) - (b - a) * (r - 1.0));
        q = (q - 1.0) * (r - 1.0) * (t - 1.0);
      }
      if (p > 0.0) q = -q;
      else p = -p;
      t = e;
      e = d;
      if (2.0 * p < 3.0 * m * q - fabs(tol * q) && p < fabs(0.5 * t * q)) {
        d = p / q;
      } else {
        d = m;
        e = m;
      }
    }
    a = b;
    fa = fb;
    if (fabs(d) > tol) b += d;
    else b += (m > 0.0 ? tol : -tol);
    fb = m1_R(co, b);
  }
  return b;
}

// Eddington factor of the closure at this state
__device__ __forceinline__ double m1_closure_chi(const M1State& s, const double gd[6], const double gu[6]) {
  const M1RCoef co = m1_rcoef(s, gd, gu);
  const double r0 = m1_R(co, 0.0), r1 = m1_R(co, 1.0);
  double xi;
  if (r1 <= 0.0) xi = 1.0;
  else if (r0 >= 0.0) xi = 0.0;
  else xi = m1_brent(co, 0.0, 1.0, r0, r1);
  return m1_eddington(xi);
}

__device__ __forceinline__ double m1_speed(const M1State& s, const double gu[6], double chi, double alp, double bd,
                                           int d) {
  const double dthick = 1.5 * (1.0 - chi), dthin = 1.0 - dthick, W2 = s.W * s.W;
  double lthin = fabs(bd);
  if (s.F2 > 0.0) lthin += alp * fmax(fabs(s.Fu[d]) / sqrt(s.F2), s.E * fabs(s.Fu[d]) / s.F2);
  const double a = (2.0 * W2 + 1.0) * gu[sym(d, d)] - 2.0 * W2 * s.v[d] * s.v[d];
  const double lthick =
      fabs(bd) + alp * fmax((2.0 * W2 * fabs(s.v[d]) + sqrt(fmax(a, 0.0))) / (2.0 * W2 + 1.0), fabs(s.v[d]));
  return dthin * lthin + dthick * lthick;
}

__device__ __forceinline__ void m1_load_state(const double* __restrict__ U, const double* __restrict__ P, int64_t sf,
                                              int64_t p, int sp, const MetricR& m, M1State& s) {
  double F[3], v[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    F[i] = U[(33 + 4 * sp + i) * sf + p] / m.sqrtg;
    v[i] = P[(3 + i) * sf + p];
  }
  m1_state_init(s, U[(32 + 4 * sp) * sf + p] / m.sqrtg, F, v, P[6 * sf + p], m.gd, m.gu);
}

__device__ __forceinline__ void m1_metric(const double* __restrict__ U, int64_t sf, int64_t p, MetricR& m) {
  double gt[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) gt[c] = U[c * sf + p];
  metric_repro(gt, U[12 * sf + p], m);
}

}  // namespace mhd
