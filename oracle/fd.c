/*
 * Oracle (test infrastructure only): discrete operators of Sec. 3.2 and the
 * MP5 reconstruction of Sec. 3.3, at a single point of a strided array.
 * s is the element stride along the derivative direction, h the spacing.
 */
#include <math.h>
#include "orc.h"

/* 4th-order centred first derivative: (u_{-2} - 8u_{-1} + 8u_{+1} - u_{+2})/(12h),
 * summed as antisymmetric pairs so that constant data gives exactly zero. */
double orc_d1(const double* u, int64_t p, int64_t s, double h) {
  return (8.0 * (u[p + s] - u[p - s]) - (u[p + 2 * s] - u[p - 2 * s])) / (12.0 * h);
}

/* compact 4th-order second derivative: (-u_{-2} + 16u_{-1} - 30u_0 + 16u_{+1} - u_{+2})/(12h^2) */
double orc_d2(const double* u, int64_t p, int64_t s, double h) {
  return (16.0 * (u[p + s] + u[p - s]) - (u[p + 2 * s] + u[p - 2 * s]) - 30.0 * u[p]) / (12.0 * h * h);
}

/* mixed second derivative D_{xy} = D_y(D_x u) */
double orc_d11(const double* u, int64_t p, int64_t s1, int64_t s2, double h1, double h2) {
  double dm2 = orc_d1(u, p - 2 * s2, s1, h1);
  double dm1 = orc_d1(u, p - 1 * s2, s1, h1);
  double dp1 = orc_d1(u, p + 1 * s2, s1, h1);
  double dp2 = orc_d1(u, p + 2 * s2, s1, h1);
  return (8.0 * (dp1 - dm1) - (dp2 - dm2)) / (12.0 * h2);
}

/* one-sided 4th-order derivative for advection terms beta * d u:
 *   beta <  0: (-u_{-3} + 6u_{-2} - 18u_{-1} + 10u_0 + 3u_{+1})/(12h)
 *   beta >= 0: ( u_{+3} - 6u_{+2} + 18u_{+1} - 10u_0 - 3u_{-1})/(12h)
 * (beta = 0 takes the second form; the product with beta vanishes anyway). */
double orc_dup(const double* u, int64_t p, int64_t s, double h, double beta) {
  if (beta < 0.0)
    return (-u[p - 3 * s] + 6.0 * u[p - 2 * s] - 18.0 * u[p - s] + 10.0 * u[p] + 3.0 * u[p + s]) / (12.0 * h);
  return (u[p + 3 * s] - 6.0 * u[p + 2 * s] + 18.0 * u[p + s] - 10.0 * u[p] - 3.0 * u[p - s]) / (12.0 * h);
}

/* Kreiss-Oliger dissipation along one axis:
 *   sigma/(64h) (u_{-3} - 6u_{-2} + 15u_{-1} - 20u_0 + 15u_{+1} - 6u_{+2} + u_{+3}) */
double orc_ko(const double* u, int64_t p, int64_t s, double h, double sigma) {
  double q = (u[p + 3 * s] + u[p - 3 * s]) - 6.0 * (u[p + 2 * s] + u[p - 2 * s])
             + 15.0 * (u[p + s] + u[p - s]) - 20.0 * u[p];
  return sigma / (64.0 * h) * q;
}

static double sgn(double a) { return a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0); }

/* Minmod(a,b) = (sgn a + sgn b)/2 * min(|a|,|b|) */
static double minmod2(double a, double b) {
  return 0.5 * (sgn(a) + sgn(b)) * fmin(fabs(a), fabs(b));
}

/* four-argument minmod: common sign times the smallest magnitude, 0 if the
 * signs disagree (the natural extension of the two-argument form) */
static double minmod4(double a, double b, double c, double d) {
  double s = sgn(a);
  if (s == 0.0 || sgn(b) != s || sgn(c) != s || sgn(d) != s) return 0.0;
  return s * fmin(fmin(fabs(a), fabs(b)), fmin(fabs(c), fabs(d)));
}

/* Median(a,b,c) = a + Minmod(b-a, c-a) */
static double median3(double a, double b, double c) { return a + minmod2(b - a, c - a); }

static double min3(double a, double b, double c) { return fmin(a, fmin(b, c)); }
static double max3(double a, double b, double c) { return fmax(a, fmax(b, c)); }

/* MP5 reconstruction of the value at i+1/2 from f5 = (F_{i-2},...,F_{i+2}),
 * Suresh & Huynh with the bounds of Sec. 3.3. */
double orc_mp5(const double* f5, double alpha) {
  double fm2 = f5[0], fm1 = f5[1], f0 = f5[2], fp1 = f5[3], fp2 = f5[4];
  double funl = (2.0 * fm2 - 13.0 * fm1 + 47.0 * f0 + 27.0 * fp1 - 3.0 * fp2) / 60.0;
  double dplus = fp1 - f0;   /* Delta_{i+1/2} */
  double dminus = f0 - fm1;  /* Delta_{i-1/2} */
  double fmp = f0 + minmod2(dplus, alpha * dminus);
  if ((funl - f0) * (funl - fmp) < 0.0) return funl;
  {
    double dm1 = fm2 - 2.0 * fm1 + f0; /* d_{i-1} */
    double d0 = fm1 - 2.0 * f0 + fp1;  /* d_i */
    double dp1 = f0 - 2.0 * fp1 + fp2; /* d_{i+1} */
    double dm4_plus = minmod4(4.0 * d0 - dp1, 4.0 * dp1 - d0, d0, dp1);   /* d^M4_{i+1/2} */
    double dm4_minus = minmod4(4.0 * dm1 - d0, 4.0 * d0 - dm1, dm1, d0);  /* d^M4_{i-1/2} */
    double ful = f0 + alpha * dminus;
    double fmd = 0.5 * (f0 + fp1) - 0.5 * dm4_plus;
    double flc = f0 + 0.5 * dminus + 4.0 / 3.0 * dm4_minus;
    double fmin_ = fmax(min3(f0, fp1, fmd), min3(f0, ful, flc));
    double fmax_ = fmin(max3(f0, fp1, fmd), max3(f0, ful, flc));
    return median3(fmin_, funl, fmax_);
  }
}
