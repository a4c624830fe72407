/*
 * Oracle (test infrastructure only): conserved <-> primitive conversion.
 *
 * prim -> cons: the definitions of Sec. 2.2 (restated in App. D):
 *   D = rho W, DYe = rho W Ye,
 *   tau = h W^2 - p + B^2 - [(B.v)^2 + B^2/W^2]/2 - D,
 *   S_i = (h W^2 + B^2) v_i - (B.v) B_i,   h = rho(1+eps) + p,
 * densitized by sqrt(gamma).
 *
 * cons -> prim: App. D, following the two-root construction of Kastaun et al.
 *   step 1: q = tau/D, r_i = S_i/D, calB^i = B^i/sqrt(D), r^2, calB^2, (r.calB),
 *           calB^2 r_perp^2 = calB^2 r^2 - (r.calB)^2
 *   step 2: root mu_+ of f_a(mu) = mu sqrt(h0^2 + rbar^2(mu)) - 1 on (0, 1/h0]
 *   step 3: root mu of f(mu) = mu - 1/(nuhat + mu rbar^2(mu)) on (0, mu_+]
 *   step 4: primitives from mu; v^i = mu chi (r^i + mu (r.calB) calB^i)
 * both roots by Brent's method (R. P. Brent, Algorithms for Minimization
 * without Derivatives, 1973, ch. 4), run until the bracket is a few ulp wide,
 * followed by the error policy of App. D.
 */
#include <float.h>
#include <math.h>
#include <stddef.h>
#include "orc.h"

/* quantities fixed during the iterations (step 1) */
typedef struct {
  const orc_eos* e;
  double D, q, r2, B2, rB, B2rp2, v02, h0;
} c2p_ctx;

static double chi_of(const c2p_ctx* c, double mu) { return 1.0 / (1.0 + mu * c->B2); }

static double rbar2_of(const c2p_ctx* c, double mu) {
  double x = chi_of(c, mu);
  return c->r2 * x * x + mu * x * (1.0 + x) * c->rB * c->rB;
}

/* f_a(mu) = mu sqrt(h0^2 + rbar^2) - 1 */
static double f_a(const c2p_ctx* c, double mu) {
  return mu * sqrt(c->h0 * c->h0 + rbar2_of(c, mu)) - 1.0;
}

/* the step-3 intermediate quantities at mu; eps/rho clamped into the EoS range */
typedef struct {
  double x, rb2, qbar, v2, W, rho_raw, eps_raw, rho, eps, p, a;
} c2p_state;

static void state_at(const c2p_ctx* c, double mu, c2p_state* s) {
  const orc_eos* e = c->e;
  double emin;
  s->x = chi_of(c, mu);
  s->rb2 = rbar2_of(c, mu);
  s->qbar = c->q - 0.5 * c->B2 - 0.5 * mu * mu * s->x * s->x * c->B2rp2;
  s->v2 = fmin(mu * mu * s->rb2, c->v02);
  s->W = 1.0 / sqrt(1.0 - s->v2);
  s->rho_raw = c->D / s->W;
  s->eps_raw = s->W * (s->qbar - mu * s->rb2) + s->v2 * s->W * s->W / (1.0 + s->W);
  s->rho = fmax(fmin(e->rho_max, s->rho_raw), e->rho_min);
  emin = orc_eps_cold(e, s->rho);
  s->eps = fmax(fmin(e->eps_max, s->eps_raw), emin);
  s->p = orc_press(e, s->rho, s->eps);
  s->a = s->p / (s->rho * (1.0 + s->eps));
}

/* f(mu) = mu - 1/(nuhat + mu rbar^2), nuhat = max(nu_A, nu_B) */
static double f_main(const c2p_ctx* c, double mu) {
  c2p_state s;
  double nuA, nuB, nu;
  state_at(c, mu, &s);
  nuA = (1.0 + s.a) * (1.0 + s.eps) / s.W;
  nuB = (1.0 + s.a) * (1.0 + s.qbar - mu * s.rb2);
  nu = fmax(nuA, nuB);
  return mu - 1.0 / (nu + mu * s.rb2);
}

typedef double (*c2p_fn)(const c2p_ctx*, double);

/* Brent's root finder on a bracket [a,b] with f(a) f(b) <= 0.
 * Stops when half the bracket is <= 2 eps |b| (a few ulp), or after maxit. */
static double brent(c2p_fn f, const c2p_ctx* ctx, double a, double b, double fa, double fb,
                    int maxit, int* iters, int* ok) {
  double c = a, fc = fa, d = b - a, e = d;
  int it;
  *ok = 1;
  for (it = 0; it < maxit; ++it) {
    double tol, m, p, q, r, s;
    if ((fb > 0.0 && fc > 0.0) || (fb < 0.0 && fc < 0.0)) {
      c = a; fc = fa; d = b - a; e = d;
    }
    if (fabs(fc) < fabs(fb)) {
      a = b; b = c; c = a;
      fa = fb; fb = fc; fc = fa;
    }
    tol = 2.0 * DBL_EPSILON * fabs(b);
    m = 0.5 * (c - b);
    if (fabs(m) <= tol || fb == 0.0) {
      *iters = it;
      return b;
    }
    if (fabs(e) < tol || fabs(fa) <= fabs(fb)) {
      d = m; e = m;  /* bisection */
    } else {
      s = fb / fa;
      if (a == c) { /* secant */
        p = 2.0 * m * s;
        q = 1.0 - s;
      } else {      /* inverse quadratic interpolation */
        q = fa / fc;
        r = fb / fc;
        p = s * (2.0 * m * q * (q - r) - (b - a) * (r - 1.0));
        q = (q - 1.0) * (r - 1.0) * (s - 1.0);
      }
      if (p > 0.0) q = -q; else p = -p;
      s = e;
      e = d;
      if (2.0 * p < 3.0 * m * q - fabs(tol * q) && p < fabs(0.5 * s * q)) {
        d = p / q;
      } else {
        d = m; e = m;
      }
    }
    a = b;
    fa = fb;
    if (fabs(d) > tol) b += d;
    else b += (m > 0.0 ? tol : -tol);
    fb = f(ctx, b);
  }
  *iters = maxit;
  *ok = 0;
  return b;
}

static void lower(const double gdn[6], const double up[3], double dn[3]) {
  dn[0] = gdn[0] * up[0] + gdn[1] * up[1] + gdn[2] * up[2];
  dn[1] = gdn[1] * up[0] + gdn[3] * up[1] + gdn[4] * up[2];
  dn[2] = gdn[2] * up[0] + gdn[4] * up[1] + gdn[5] * up[2];
}

static void atmosphere(const orc_eos* e, double prim[8]) {
  prim[0] = e->rho_atm;
  prim[1] = orc_eps_cold(e, e->rho_atm);
  prim[2] = orc_press(e, prim[0], prim[1]);
  prim[3] = prim[4] = prim[5] = 0.0;
  prim[6] = 1.0;
  prim[7] = e->ye_atm;
}

/* step 1: the quantities fixed during the iterations; r^i and calB^i kept for step 4 */
static void setup_ctx(const orc_eos* e, const double cons[6], const double B[3], const double gdn[6],
                      const double gup[6], c2p_ctx* c, double r_up[3], double cB[3]) {
  double r_dn[3], cB_dn[3];
  int i;
  c->e = e;
  c->D = cons[0];
  c->h0 = e->h0;
  c->q = cons[2] / cons[0];
  for (i = 0; i < 3; ++i) {
    r_dn[i] = cons[3 + i] / cons[0];
    cB[i] = B[i] / sqrt(cons[0]);
  }
  r_up[0] = gup[0] * r_dn[0] + gup[1] * r_dn[1] + gup[2] * r_dn[2];
  r_up[1] = gup[1] * r_dn[0] + gup[3] * r_dn[1] + gup[4] * r_dn[2];
  r_up[2] = gup[2] * r_dn[0] + gup[4] * r_dn[1] + gup[5] * r_dn[2];
  lower(gdn, cB, cB_dn);
  c->r2 = r_up[0] * r_dn[0] + r_up[1] * r_dn[1] + r_up[2] * r_dn[2];
  c->B2 = cB[0] * cB_dn[0] + cB[1] * cB_dn[1] + cB[2] * cB_dn[2];
  c->rB = r_dn[0] * cB[0] + r_dn[1] * cB[1] + r_dn[2] * cB[2];
  c->B2rp2 = fmax(0.0, c->B2 * c->r2 - c->rB * c->rB);
  c->v02 = c->r2 / (c->h0 * c->h0 + c->r2);
}

/* steps 1-4 and the error policy; with mu_fixed != NULL, steps 2 and 3 are
 * skipped and the primitives are those at mu = *mu_fixed */
static unsigned c2p_point_impl(const orc_eos* e, const double cons[6], const double B[3],
                               const double gdn[6], const double gup[6], double alpha,
                               const double* mu_fixed, double prim[8], double mu_out[2], int* iters) {
  c2p_ctx c;
  c2p_state s;
  double r_up[3], cB[3];
  double mup, mu, fa_hi, f_lo, f_hi;
  int it1 = 0, it2 = 0, ok1 = 1, ok2 = 1, i;
  unsigned flags = 0;
  int low;
  double rho, eps, W, v[3], ye;

  if (mu_out) { mu_out[0] = 0.0; mu_out[1] = 0.0; }
  if (iters) *iters = 0;
  /* no positive rest mass above the threshold: atmosphere (rho = D/W <= D) */
  if (!(cons[0] >= e->rho_min)) {
    atmosphere(e, prim);
    return ORC_F_ATMO;
  }
  setup_ctx(e, cons, B, gdn, gup, &c, r_up, cB);

  if (mu_fixed) {
    mup = 0.0;
    mu = *mu_fixed;
  } else {
    /* step 2: mu_+ in (0, 1/h0] */
    fa_hi = f_a(&c, 1.0 / c.h0);
    if (fa_hi <= 0.0) mup = 1.0 / c.h0;
    else mup = brent(f_a, &c, 0.0, 1.0 / c.h0, -1.0, fa_hi, 200, &it1, &ok1);

    /* step 3: mu in (0, mu_+] */
    f_lo = f_main(&c, 0.0);
    f_hi = f_main(&c, mup);
    if (f_hi <= 0.0) mu = mup;
    else mu = brent(f_main, &c, 0.0, mup, f_lo, f_hi, 200, &it2, &ok2);
  }
  if (!(ok1 && ok2)) flags |= ORC_F_NOT_CONVERGED;
  if (iters) *iters = it1 + it2;
  if (mu_out) { mu_out[0] = mup; mu_out[1] = mu; }

  /* step 4: primitives at the root */
  state_at(&c, mu, &s);
  for (i = 0; i < 3; ++i) v[i] = mu * s.x * (r_up[i] + mu * c.rB * cB[i]);
  W = s.W;
  rho = s.rho_raw;
  eps = s.eps_raw;
  ye = cons[1] / cons[0];

  /* error policy (App. D) */
  low = (rho < e->rho_low) || (alpha < e->alpha_bh);
  if (rho < e->rho_min) {
    atmosphere(e, prim);
    return flags | ORC_F_ATMO;
  }
  if (rho > e->rho_max) {
    flags |= ORC_F_FATAL;
    rho = e->rho_max;
  }
  if (W > e->W_max) {
    if (low) {
      double vd[3], v2, vmax2 = 1.0 - 1.0 / (e->W_max * e->W_max), sc;
      lower(gdn, v, vd);
      v2 = v[0] * vd[0] + v[1] * vd[1] + v[2] * vd[2];
      sc = sqrt(vmax2 / v2);
      for (i = 0; i < 3; ++i) v[i] *= sc;
      W = e->W_max;
      rho = c.D / W;
      flags |= ORC_F_VEL_LIMIT;
    } else {
      flags |= ORC_F_FATAL;
    }
  }
  {
    double emin = orc_eps_cold(e, rho);
    if (eps < emin) {
      eps = emin;
      flags |= ORC_F_EPS_LO;
    } else if (eps > e->eps_max) {
      eps = e->eps_max;
      flags |= low ? ORC_F_EPS_HI : ORC_F_FATAL;
    }
  }
  if (ye < e->ye_min || ye > e->ye_max) {
    if (low) {
      ye = e->ye_atm;
      flags |= ORC_F_YE_RESET;
    } else {
      flags |= ORC_F_FATAL;
    }
  }
  prim[0] = rho;
  prim[1] = eps;
  prim[2] = orc_press(e, rho, eps);
  prim[3] = v[0];
  prim[4] = v[1];
  prim[5] = v[2];
  prim[6] = W;
  prim[7] = ye;
  return flags;
}

unsigned orc_c2p_point(const orc_eos* e, const double cons[6], const double B[3],
                       const double gdn[6], const double gup[6], double alpha,
                       double prim[8], double mu_out[2], int* iters) {
  return c2p_point_impl(e, cons, B, gdn, gup, alpha, NULL, prim, mu_out, iters);
}

/* ---------- grid-level drivers ---------- */

static void metric_at(const double* U, int64_t p, int64_t N, double gdn[6], double gup[6],
                      double* sqrtg) {
  double gt[6], chi, det, inv[6];
  int i;
  for (i = 0; i < 6; ++i) gt[i] = U[i * N + p];
  chi = U[12 * N + p];
  det = gt[0] * (gt[3] * gt[5] - gt[4] * gt[4]) - gt[1] * (gt[1] * gt[5] - gt[4] * gt[2])
        + gt[2] * (gt[1] * gt[4] - gt[3] * gt[2]);
  inv[0] = (gt[3] * gt[5] - gt[4] * gt[4]) / det;
  inv[1] = (gt[2] * gt[4] - gt[1] * gt[5]) / det;
  inv[2] = (gt[1] * gt[4] - gt[2] * gt[3]) / det;
  inv[3] = (gt[0] * gt[5] - gt[2] * gt[2]) / det;
  inv[4] = (gt[1] * gt[2] - gt[0] * gt[4]) / det;
  inv[5] = (gt[0] * gt[3] - gt[1] * gt[1]) / det;
  for (i = 0; i < 6; ++i) {
    gdn[i] = gt[i] / chi;
    gup[i] = chi * inv[i];
  }
  *sqrtg = sqrt(det / (chi * chi * chi));
}

/* undensitized conserved variables of one point from primitives */
static void p2c_point(const double gdn[6], const double prim[8], const double B[3],
                      double cons[6]) {
  double v[3] = {prim[3], prim[4], prim[5]}, vd[3], Bd[3];
  double v2, W, B2, Bv, h;
  int i;
  lower(gdn, v, vd);
  lower(gdn, B, Bd);
  v2 = v[0] * vd[0] + v[1] * vd[1] + v[2] * vd[2];
  W = 1.0 / sqrt(1.0 - v2);
  B2 = B[0] * Bd[0] + B[1] * Bd[1] + B[2] * Bd[2];
  Bv = B[0] * vd[0] + B[1] * vd[1] + B[2] * vd[2];
  h = prim[0] * (1.0 + prim[1]) + prim[2];
  cons[0] = prim[0] * W;
  cons[1] = prim[0] * W * prim[7];
  cons[2] = h * W * W - prim[2] + B2 - 0.5 * (Bv * Bv + B2 / (W * W)) - cons[0];
  for (i = 0; i < 3; ++i) cons[3 + i] = (h * W * W + B2) * vd[i] - Bv * Bd[i];
}

static int64_t npts(const orc_grid* g) {
  return (int64_t)(g->n[0] + 2 * g->ng) * (g->n[1] + 2 * g->ng) * (g->n[2] + 2 * g->ng);
}

void orc_prim2con(const orc_grid* g, const orc_eos* e, double* U, double* P,
                  const double* EM, int eps_mode) {
  int64_t N = npts(g), p;
  ORC_PHASE(ORC_PH_P2C);
#pragma omp parallel for schedule(static)
  for (p = 0; p < N; ++p) {
    double gdn[6], gup[6], sg, prim[8], B[3], cons[6], v[3], vd[3], v2;
    int i;
    metric_at(U, p, N, gdn, gup, &sg);
    for (i = 0; i < 8; ++i) prim[i] = P[i * N + p];
    if (eps_mode == 1) prim[1] += orc_eps_cold(e, prim[0]);
    prim[2] = orc_press(e, prim[0], prim[1]);
    v[0] = prim[3]; v[1] = prim[4]; v[2] = prim[5];
    lower(gdn, v, vd);
    v2 = v[0] * vd[0] + v[1] * vd[1] + v[2] * vd[2];
    prim[6] = 1.0 / sqrt(1.0 - v2);
    for (i = 0; i < 3; ++i) B[i] = EM[i * N + p];
    p2c_point(gdn, prim, B, cons);
    for (i = 0; i < 6; ++i) U[(22 + i) * N + p] = sg * cons[i];
    for (i = 0; i < 3; ++i) U[(28 + i) * N + p] = sg * B[i];
    U[31 * N + p] = sg * EM[3 * N + p];
    P[1 * N + p] = prim[1];
    P[2 * N + p] = prim[2];
    P[6 * N + p] = prim[6];
  }
  ORC_PHASE(ORC_PH_OTHER);
}

int64_t orc_con2prim(const orc_grid* g, const orc_eos* e, double* U, double* P,
                     uint8_t* flags, double* mu) {
  int64_t N = npts(g), p, nfatal = 0;
  ORC_PHASE(ORC_PH_C2P);
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : nfatal)
  for (p = 0; p < N; ++p) {
    double gdn[6], gup[6], sg, cons[6], B[3], prim[8], m[2];
    unsigned f;
    int i, it;
    metric_at(U, p, N, gdn, gup, &sg);
    for (i = 0; i < 6; ++i) cons[i] = U[(22 + i) * N + p] / sg;
    for (i = 0; i < 3; ++i) B[i] = U[(28 + i) * N + p] / sg;
    f = orc_c2p_point(e, cons, B, gdn, gup, U[18 * N + p], prim, m, &it);
    for (i = 0; i < 8; ++i) P[i * N + p] = prim[i];
    if (f & (ORC_F_ATMO | ORC_F_EPS_LO | ORC_F_EPS_HI | ORC_F_VEL_LIMIT | ORC_F_YE_RESET)) {
      p2c_point(gdn, prim, B, cons);
      for (i = 0; i < 6; ++i) U[(22 + i) * N + p] = sg * cons[i];
    }
    if (flags) flags[p] = (uint8_t)f;
    if (mu) { mu[p] = m[0]; mu[N + p] = m[1]; }
    if (f & ORC_F_FATAL) nfatal += 1;
  }
  ORC_PHASE(ORC_PH_OTHER);
  return nfatal;
}

/* Primitives (step 4 and the error policy) at a given mu per padded point,
 * mu[N] (undensitizing as orc_con2prim; U is not written).  For the tests'
 * condition estimates: how far the primitives move when mu moves. */
void orc_c2p_prims_at(const orc_grid* g, const orc_eos* e, const double* U, const double* mu,
                      double* P, uint8_t* flags) {
  int64_t N = npts(g), p;
#pragma omp parallel for schedule(static)
  for (p = 0; p < N; ++p) {
    double gdn[6], gup[6], sg, cons[6], B[3], prim[8], m = mu[p];
    unsigned f;
    int i;
    metric_at(U, p, N, gdn, gup, &sg);
    for (i = 0; i < 6; ++i) cons[i] = U[(22 + i) * N + p] / sg;
    for (i = 0; i < 3; ++i) B[i] = U[(28 + i) * N + p] / sg;
    f = c2p_point_impl(e, cons, B, gdn, gup, U[18 * N + p], &m, prim, NULL, NULL);
    for (i = 0; i < 8; ++i) P[i * N + p] = prim[i];
    if (flags) flags[p] = (uint8_t)f;
  }
}

/* f_a and f (steps 2 and 3) at a given mu per padded point, fa[N] and f[N]
 * (undensitizing as orc_con2prim).  For the tests: whether a mu found by
 * another solver is a root of the same functions. */
void orc_c2p_f_at(const orc_grid* g, const orc_eos* e, const double* U, const double* mu,
                  double* fa, double* f) {
  int64_t N = npts(g), p;
#pragma omp parallel for schedule(static)
  for (p = 0; p < N; ++p) {
    double gdn[6], gup[6], sg, cons[6], B[3], r_up[3], cB[3];
    c2p_ctx c;
    int i;
    metric_at(U, p, N, gdn, gup, &sg);
    for (i = 0; i < 6; ++i) cons[i] = U[(22 + i) * N + p] / sg;
    for (i = 0; i < 3; ++i) B[i] = U[(28 + i) * N + p] / sg;
    if (!(cons[0] >= e->rho_min)) {
      fa[p] = f[p] = NAN;
      continue;
    }
    setup_ctx(e, cons, B, gdn, gup, &c, r_up, cB);
    fa[p] = f_a(&c, mu[p]);
    f[p] = f_main(&c, mu[p]);
  }
}

void orc_c2p_features(const orc_grid* g, const orc_eos* e, const double* U, const double* mu,
                      float* X, float* T) {
  int64_t N = npts(g), p;
#pragma omp parallel for schedule(static)
  for (p = 0; p < N; ++p) {
    double gdn[6], gup[6], sg, cons[6], B[3], x[8], m[2], t[2], b[2];
    int i;
    metric_at(U, p, N, gdn, gup, &sg);
    for (i = 0; i < 6; ++i) cons[i] = U[(22 + i) * N + p] / sg;
    for (i = 0; i < 3; ++i) B[i] = U[(28 + i) * N + p] / sg;
    if (!(cons[0] >= e->rho_min)) {
      for (i = 0; i < 8; ++i) X[p * 8 + i] = (float)NAN;
      if (T) T[p * 2] = T[p * 2 + 1] = (float)NAN;
      continue;
    }
    orc_mlp_features(cons, B, gdn, gup, x);
    for (i = 0; i < 8; ++i) X[p * 8 + i] = (float)x[i];
    if (T && mu) {
      m[0] = mu[p];
      m[1] = mu[N + p];
      orc_mlp_baseline(e->h0, cons, gup, b);
      orc_mlp_targets(e->h0, b, m, t);
      T[p * 2] = (float)t[0];
      T[p * 2 + 1] = (float)t[1];
    }
  }
}
