/*
 * Oracle (test infrastructure only): grey M1 neutrino moments.
 *
 * Per species the evolved fields are the densitized energy and flux
 * (Ebar, Fbar_i) = sqrt(gamma) (E, F_i), at U indices 32 + 4 s (s = 0, 1, 2).
 * Per point and species the auxiliary inputs are kappa_a, kappa_s and eta at
 * aux[(3 s + c) N + p], c = 0, 1, 2.
 *
 *   closure    Minerbo (Sec. 2.3): P_ij = d_thin P^thin_ij + d_thick P^thick_ij,
 *              d_thick = 3(1 - chi)/2, chi(xi) = 1/3 + xi^2 (6 - 2 xi + 6 xi^2)/15,
 *              xi the root on [0, 1] of R(xi) = (xi^2 J^2 - H_a H^a)/E^2, with J and
 *              H from the fluid-frame projections; Brent's method to full precision
 *   fluxes     d_k-flux of Ebar: -beta^k Ebar + alpha Fbar^k; of Fbar_i:
 *              -beta^k Fbar_i + alpha Pbar^k_i (Sec. 2.3)
 *   speeds     Minerbo interpolation of the thin and thick speeds (App. B)
 *   interfaces HO/LO flux splitting with the limiter Phi, the opacity switch
 *              A = tanh(1/(kappa dx)) and the odd-even fix (Sec. 3.4)
 *   sources    geometric terms of the Ebar, Fbar_i equations and the collision
 *              terms alpha sqrt(gamma) (S_n, S_i); the fluid loses what the
 *              radiation gains (tau and S_i get -alpha sqrt(gamma) sum S)
 *   matter     E, S_i, S_ij of the radiation for the CCZ4 matter terms
 *
 * Readings (where the text is silent or garbled): the low-order flux is the
 * Lax-Friedrichs flux 1/2 (F_i + F_i+1) - lambda/2 (u_i+1 - u_i); lambda at an
 * interface is the larger of the two point speeds; Phi = 0 when u_i+1 = u_i;
 * Phi and the odd-even test act per field; P^thin and the thin speed are dropped
 * when F_k F^k = 0; xi = 1 when R(1) <= 0 and xi = 0 when R(0) >= 0; a negative
 * argument of the thick-speed square root counts as 0; kappa = 0 gives A = 1.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include "orc.h"

static const int S6m[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

typedef struct {
  double gdn[3][3], gup[3][3], sqrtg, chi;
} m1_metric;

static void m1_metric_at(const double* U, int64_t N, int64_t p, m1_metric* m) {
  double g[3][3], gi[3][3], det;
  int i, j;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) g[i][j] = U[S6m[i][j] * N + p];
  m->chi = U[12 * N + p];
  det = g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1]) - g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0]) +
        g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
  gi[0][0] = (g[1][1] * g[2][2] - g[1][2] * g[2][1]) / det;
  gi[0][1] = (g[0][2] * g[2][1] - g[0][1] * g[2][2]) / det;
  gi[0][2] = (g[0][1] * g[1][2] - g[0][2] * g[1][1]) / det;
  gi[1][1] = (g[0][0] * g[2][2] - g[0][2] * g[2][0]) / det;
  gi[1][2] = (g[0][2] * g[1][0] - g[0][0] * g[1][2]) / det;
  gi[2][2] = (g[0][0] * g[1][1] - g[0][1] * g[1][0]) / det;
  gi[1][0] = gi[0][1];
  gi[2][0] = gi[0][2];
  gi[2][1] = gi[1][2];
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      m->gdn[i][j] = g[i][j] / m->chi;
      m->gup[i][j] = m->chi * gi[i][j];
    }
  m->sqrtg = sqrt(det / (m->chi * m->chi * m->chi));
}

/* one species at one point, undensitized */
typedef struct {
  double E, F[3], Fu[3], F2, v[3], vd[3], W, vF;
  double gdn[3][3], gup[3][3];
} m1_state;

double orc_m1_eddington(double xi) { return 1.0 / 3.0 + xi * xi * (6.0 - 2.0 * xi + 6.0 * xi * xi) / 15.0; }

/* P_ij, J, H_i (lower), H.n and H_a H^a for the Eddington factor chi */
static void closure_eval(const m1_state* s, double chi, double P[3][3], double* J, double H[3], double* Hn,
                         double* HH) {
  const double W = s->W, W2 = W * W;
  const double dthick = 1.5 * (1.0 - chi), dthin = 1.0 - dthick;
  double Jth, Hth[3], Pv[3], vPv = 0.0, hh = 0.0;
  int i, j;
  Jth = 3.0 / (2.0 * W2 + 1.0) * ((2.0 * W2 - 1.0) * s->E - 2.0 * W2 * s->vF);
  for (i = 0; i < 3; ++i)
    Hth[i] = s->F[i] / W + W * s->vd[i] / (2.0 * W2 + 1.0) * ((4.0 * W2 + 1.0) * s->vF - 4.0 * W2 * s->E);
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      double thin = s->F2 > 0.0 ? s->E * s->F[i] * s->F[j] / s->F2 : 0.0;
      double thick = 4.0 / 3.0 * Jth * W2 * s->vd[i] * s->vd[j] + W * (Hth[i] * s->vd[j] + Hth[j] * s->vd[i]) +
                     1.0 / 3.0 * Jth * s->gdn[i][j];
      P[i][j] = dthin * thin + dthick * thick;
    }
  for (i = 0; i < 3; ++i) {
    Pv[i] = 0.0;
    for (j = 0; j < 3; ++j) Pv[i] += P[i][j] * s->v[j];
    vPv += s->v[i] * Pv[i];
  }
  *J = W2 * (s->E - 2.0 * s->vF + vPv);
  for (i = 0; i < 3; ++i) H[i] = W * (s->F[i] - Pv[i] - *J * s->vd[i]);
  *Hn = W * (*J - s->E + s->vF);
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) hh += s->gup[i][j] * H[i] * H[j];
  *HH = hh - *Hn * *Hn;
}

static double R_of(const m1_state* s, double xi) {
  double P[3][3], J, H[3], Hn, HH;
  closure_eval(s, orc_m1_eddington(xi), P, &J, H, &Hn, &HH);
  return (xi * xi * J * J - HH) / (s->E * s->E);
}

/* Brent's method (Brent 1973, ch. 4) for R on [a, b] with R(a) < 0 < R(b) */
static double brent_xi(const m1_state* s, double a, double b, double fa, double fb, int* iters) {
  double c = a, fc = fa, d = b - a, e = d;
  int it;
  for (it = 0; it < 200; ++it) {
    double tol, m, p, q, r, t;
    if ((fb > 0.0 && fc > 0.0) || (fb < 0.0 && fc < 0.0)) {
      c = a; fc = fa; d = b - a; e = d;
    }
    if (fabs(fc) < fabs(fb)) {
      a = b; b = c; c = a;
      fa = fb; fb = fc; fc = fa;
    }
    tol = 2.0 * DBL_EPSILON * fabs(b) + 0.5 * DBL_MIN;
    m = 0.5 * (c - b);
    if (fabs(m) <= tol || fb == 0.0) break;
    if (fabs(e) < tol || fabs(fa) <= fabs(fb)) {
      d = m; e = m;
    } else {
      t = fb / fa;
      if (a == c) {
        p = 2.0 * m * t;
        q = 1.0 - t;
      } else {
        q = fa / fc;
        r = fb / fc;
        p = t * (2.0 * m * q * (q - r) - (b - a) * (r - 1.0));
        q = (q - 1.0) * (r - 1.0) * (t - 1.0);
      }
      if (p > 0.0) q = -q; else p = -p;
      t = e;
      e = d;
      if (2.0 * p < 3.0 * m * q - fabs(tol * q) && p < fabs(0.5 * t * q)) {
        d = p / q;
      } else {
        d = m; e = m;
      }
    }
    a = b;
    fa = fb;
    if (fabs(d) > tol) b += d;
    else b += (m > 0.0 ? tol : -tol);
    fb = R_of(s, b);
  }
  if (iters) *iters = it;
  return b;
}

static void state_init(m1_state* s, double E, const double F[3], const double v[3], double W,
                       const double gdn[3][3], const double gup[3][3]) {
  int i, j;
  s->E = E;
  s->W = W;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      s->gdn[i][j] = gdn[i][j];
      s->gup[i][j] = gup[i][j];
    }
  s->F2 = 0.0;
  s->vF = 0.0;
  for (i = 0; i < 3; ++i) {
    s->F[i] = F[i];
    s->v[i] = v[i];
  }
  for (i = 0; i < 3; ++i) {
    s->Fu[i] = 0.0;
    s->vd[i] = 0.0;
    for (j = 0; j < 3; ++j) {
      s->Fu[i] += gup[i][j] * F[j];
      s->vd[i] += gdn[i][j] * v[j];
    }
  }
  for (i = 0; i < 3; ++i) {
    s->F2 += s->Fu[i] * F[i];
    s->vF += F[i] * v[i];
  }
}

/* xi of the closure, and P_ij, J, H_i at it */
static double closure(const m1_state* s, double P[3][3], double* J, double H[3], double* chi_out, int* iters) {
  double xi, r0, r1, Hn, HH;
  if (iters) *iters = 0;
  r0 = R_of(s, 0.0);
  r1 = R_of(s, 1.0);
  if (r1 <= 0.0) xi = 1.0;
  else if (r0 >= 0.0) xi = 0.0;
  else xi = brent_xi(s, 0.0, 1.0, r0, r1, iters);
  *chi_out = orc_m1_eddington(xi);
  closure_eval(s, *chi_out, P, J, H, &Hn, &HH);
  return xi;
}

double orc_m1_closure(double E, const double F[3], const double v[3], double W, const double gdn6[6],
                      const double gup6[6], double P6[6], double* J, double H[3], double* chi, int* iters) {
  double gdn[3][3], gup[3][3], P[3][3], xi;
  m1_state s;
  int i, j;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      gdn[i][j] = gdn6[S6m[i][j]];
      gup[i][j] = gup6[S6m[i][j]];
    }
  state_init(&s, E, F, v, W, gdn, gup);
  xi = closure(&s, P, J, H, chi, iters);
  for (i = 0; i < 3; ++i)
    for (j = i; j < 3; ++j) P6[S6m[i][j]] = P[i][j];
  return xi;
}

/* point speed along axis d (Minerbo interpolation of the thin and thick speeds) */
static double speed(const m1_state* s, double chi, double alp, double beta_d, int d) {
  const double dthick = 1.5 * (1.0 - chi), dthin = 1.0 - dthick, W2 = s->W * s->W;
  double lthin = fabs(beta_d), lthick, a;
  if (s->F2 > 0.0) lthin += alp * fmax(fabs(s->Fu[d]) / sqrt(s->F2), s->E * fabs(s->Fu[d]) / s->F2);
  a = (2.0 * W2 + 1.0) * s->gup[d][d] - 2.0 * W2 * s->v[d] * s->v[d];
  lthick = fabs(beta_d) +
           alp * fmax((2.0 * W2 * fabs(s->v[d]) + sqrt(fmax(a, 0.0))) / (2.0 * W2 + 1.0), fabs(s->v[d]));
  return dthin * lthin + dthick * lthick;
}

/* interface value between p and p + st of one field (HO/LO splitting) */
static double holo(const double* u, const double* f, const double* lam, const double* ka, const double* ks,
                   int64_t p, int64_t st, double h) {
  const double um = u[p - st], u0 = u[p], u1 = u[p + st], u2 = u[p + 2 * st];
  const double fho = 0.5 * (f[p] + f[p + st]);
  const double lh = fmax(lam[p], lam[p + st]);
  const double flo = fho - 0.5 * lh * (u1 - u0);
  const double du = u1 - u0;
  double phi = 0.0, A, kap;
  if (du != 0.0) phi = fmax(0.0, fmin(1.0, fmin(2.0 * (u0 - um) / du, 2.0 * (u2 - u1) / du)));
  kap = 0.5 * (ka[p] + ka[p + st] + ks[p] + ks[p + st]);
  A = kap > 0.0 ? tanh(1.0 / (kap * h)) : 1.0;
  if ((u0 - um) * du < 0.0 && du * (u2 - u1) < 0.0) A = 1.0;
  return fho - A * (1.0 - phi) * (fho - flo);
}

static int64_t npts(const orc_grid* g) {
  return (int64_t)(g->n[0] + 2 * g->ng) * (g->n[1] + 2 * g->ng) * (g->n[2] + 2 * g->ng);
}

static void point_state(const double* U, const double* P, int64_t N, int64_t p, int sp, const m1_metric* m,
                        m1_state* s) {
  double F[3], v[3];
  int i;
  for (i = 0; i < 3; ++i) {
    F[i] = U[(33 + 4 * sp + i) * N + p] / m->sqrtg;
    v[i] = P[(3 + i) * N + p];
  }
  state_init(s, U[(32 + 4 * sp) * N + p] / m->sqrtg, F, v, P[6 * N + p], m->gdn, m->gup);
}

/* radiation part of the CCZ4 matter terms at p: E, S_i, S_ij are incremented */
void orc_m1_matter(const double* U, const double* P, int64_t N, int64_t p, double* E, double S[3],
                   double Sij[3][3]) {
  m1_metric m;
  int sp, i, j;
  m1_metric_at(U, N, p, &m);
  for (sp = 0; sp < 3; ++sp) {
    m1_state s;
    double Pij[3][3], J, H[3], chi;
    point_state(U, P, N, p, sp, &m, &s);
    ORC_PHASE(ORC_PH_M1_RECL); /* the closure itself belongs to the M1 point step */
    closure(&s, Pij, &J, H, &chi, NULL);
    ORC_PHASE(ORC_PH_CCZ4);
    *E += s.E;
    for (i = 0; i < 3; ++i) {
      S[i] += s.F[i];
      for (j = 0; j < 3; ++j) Sij[i][j] += Pij[i][j];
    }
  }
}

/* M1 part of L(U) at interior points: rhs[32..43] written; the collision
 * exchange is subtracted from rhs[24] (taubar) and rhs[25..27] (Sbar_i), which
 * must already hold the fluid part.  max_speed (may be NULL) gets the max of
 * the M1 point speeds. */
static void m1_rhs_impl(const orc_grid* g, const orc_par* par, const double* U, const double* P,
                        const double* aux, double* rhs, double* stiff, double* max_speed) {
  const int ng = g->ng;
  const int nrad = par->evolve_m1n ? 15 : 12; /* stiff slots of the radiation (and number densities) */
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = npts(g);
  const int64_t st[3] = {1, Nx, Nx * Ny};
  /* per species and axis: 4 point fluxes and the point speed */
  double* FL = (double*)malloc(sizeof(double) * 3 * 3 * 4 * N);
  double* LM = (double*)malloc(sizeof(double) * 3 * 3 * N);
  double vmax = 0.0;
  int64_t p;

  ORC_PHASE(ORC_PH_M1_POINT);
#pragma omp parallel for schedule(static)
  for (p = 0; p < N; ++p) {
    m1_metric m;
    int sp, d, i, j;
    const double alp = U[18 * N + p];
    m1_metric_at(U, N, p, &m);
    for (sp = 0; sp < 3; ++sp) {
      m1_state s;
      double Pij[3][3], J, H[3], chi;
      const double Eb = U[(32 + 4 * sp) * N + p];
      point_state(U, P, N, p, sp, &m, &s);
      closure(&s, Pij, &J, H, &chi, NULL);
      for (d = 0; d < 3; ++d) {
        const double bd = U[(19 + d) * N + p];
        double* f = FL + ((sp * 3 + d) * 4) * N;
        f[p] = -bd * Eb + alp * m.sqrtg * s.Fu[d];
        for (i = 0; i < 3; ++i) {
          double Pdi = 0.0;
          for (j = 0; j < 3; ++j) Pdi += m.gup[d][j] * Pij[j][i];
          f[(1 + i) * N + p] = -bd * U[(33 + 4 * sp + i) * N + p] + alp * m.sqrtg * Pdi;
        }
        LM[(sp * 3 + d) * N + p] = speed(&s, chi, alp, bd, d);
      }
    }
  }

  ORC_PHASE(ORC_PH_M1_UPD);
#pragma omp parallel for collapse(2) schedule(static) reduction(max : vmax)
  for (int64_t k = ng; k < Nz - ng; ++k)
    for (int64_t j = ng; j < Ny - ng; ++j)
      for (int64_t i = ng; i < Nx - ng; ++i) {
        const int64_t q = i + Nx * (j + Ny * k);
        const double alp = U[18 * N + q], Kh = U[13 * N + q], Th = U[14 * N + q];
        m1_metric m;
        double dalp[3], dchi[3], dbeta[3][3], dgt[3][3][3];
        int sp, d, c, a, b, e2;
        m1_metric_at(U, N, q, &m);
        for (d = 0; d < 3; ++d) {
          dalp[d] = orc_d1(U + 18 * N, q, st[d], g->dx[d]);
          dchi[d] = orc_d1(U + 12 * N, q, st[d], g->dx[d]);
          for (a = 0; a < 3; ++a) dbeta[d][a] = orc_d1(U + (19 + a) * N, q, st[d], g->dx[d]);
          for (a = 0; a < 3; ++a)
            for (b = 0; b < 3; ++b) dgt[d][a][b] = orc_d1(U + S6m[a][b] * N, q, st[d], g->dx[d]);
        }
        for (sp = 0; sp < 3; ++sp) {
          double out[4] = {0.0, 0.0, 0.0, 0.0};
          m1_state s;
          double Pij[3][3], J, H[3], chi, Pbu[3][3], trP = 0.0, Fbu[3], Sn, Si[3];
          const double ka = aux[(3 * sp) * N + q], ks = aux[(3 * sp + 1) * N + q], eta = aux[(3 * sp + 2) * N + q];
          const double Eb = U[(32 + 4 * sp) * N + q];
          for (d = 0; d < 3; ++d) {
            const double* lam = LM + (sp * 3 + d) * N;
            vmax = fmax(vmax, lam[q]);
            for (c = 0; c < 4; ++c) {
              const double* u = U + (32 + 4 * sp + c) * N;
              const double* f = FL + ((sp * 3 + d) * 4 + c) * N;
              const double* kap = aux + (3 * sp) * N;
              const double* kas = aux + (3 * sp + 1) * N;
              double fr, fl;
              ORC_PHASE(ORC_PH_M1_HOLO);
              fr = holo(u, f, lam, kap, kas, q, st[d], g->dx[d]);
              fl = holo(u, f, lam, kap, kas, q - st[d], st[d], g->dx[d]);
              ORC_PHASE(ORC_PH_M1_UPD);
              out[c] -= (fr - fl) / g->dx[d];
            }
          }
          /* geometric sources */
          ORC_PHASE(ORC_PH_M1_RECL);
          point_state(U, P, N, q, sp, &m, &s);
          closure(&s, Pij, &J, H, &chi, NULL);
          ORC_PHASE(ORC_PH_M1_UPD);
          for (a = 0; a < 3; ++a)
            for (b = 0; b < 3; ++b) {
              double t = 0.0;
              for (c = 0; c < 3; ++c)
                for (e2 = 0; e2 < 3; ++e2) t += m.gup[a][c] * m.gup[b][e2] * Pij[c][e2];
              Pbu[a][b] = m.sqrtg * t;
            }
          for (a = 0; a < 3; ++a)
            for (b = 0; b < 3; ++b) trP += m.gdn[a][b] * Pbu[a][b];
          for (a = 0; a < 3; ++a) {
            Fbu[a] = 0.0;
            for (b = 0; b < 3; ++b) Fbu[a] += m.gup[a][b] * U[(33 + 4 * sp + b) * N + q];
          }
          {
            double r = 0.0;
            for (a = 0; a < 3; ++a)
              for (b = 0; b < 3; ++b) r += alp / m.chi * Pbu[a][b] * U[(6 + S6m[a][b]) * N + q];
            r += alp / 3.0 * trP * (Kh + 2.0 * Th);
            for (a = 0; a < 3; ++a) r -= Fbu[a] * dalp[a];
            out[0] += r;
          }
          for (a = 0; a < 3; ++a) {
            double r = 0.0;
            for (b = 0; b < 3; ++b)
              for (c = 0; c < 3; ++c) r += Pbu[b][c] * dgt[a][b][c];
            r = alp / (2.0 * m.chi) * (r - trP * dchi[a]);
            for (b = 0; b < 3; ++b) r += U[(33 + 4 * sp + b) * N + q] * dbeta[a][b];
            r -= Eb * dalp[a];
            out[1 + a] += r;
          }
          /* collisions, and the opposite exchange with the fluid */
          Sn = s.W * ((eta + ks * J) - (ka + ks) * (s.E - s.vF));
          for (a = 0; a < 3; ++a) Si[a] = s.W * (eta - ka * J) * s.vd[a] - (ka + ks) * H[a];
          if (stiff) {
            stiff[(4 * sp) * N + q] = alp * m.sqrtg * Sn;
            for (a = 0; a < 3; ++a) stiff[(4 * sp + 1 + a) * N + q] = alp * m.sqrtg * Si[a];
          } else {
            out[0] += alp * m.sqrtg * Sn;
            for (a = 0; a < 3; ++a) out[1 + a] += alp * m.sqrtg * Si[a];
          }
          if (stiff && par->couple_exchange) {
            /* the fluid's share in the stiff part too: slots nrad (tau), nrad + 1..3 (S_i) */
            double* fs = stiff + (int64_t)nrad * N + q;
            fs[0] = (sp == 0 ? 0.0 : fs[0]) - alp * m.sqrtg * Sn;
            for (a = 0; a < 3; ++a) fs[(1 + a) * N] = (sp == 0 ? 0.0 : fs[(1 + a) * N]) - alp * m.sqrtg * Si[a];
          } else {
            rhs[24 * N + q] -= alp * m.sqrtg * Sn;
            for (a = 0; a < 3; ++a) rhs[(25 + a) * N + q] -= alp * m.sqrtg * Si[a];
          }
          for (c = 0; c < 4; ++c) rhs[(32 + 4 * sp + c) * N + q] = out[c];
        }
      }
  ORC_PHASE(ORC_PH_OTHER);
  free(FL);
  free(LM);
  if (max_speed) *max_speed = fmax(*max_speed, vmax);
}

void orc_m1_rhs(const orc_grid* g, const orc_par* par, const double* U, const double* P, const double* aux,
                double* rhs, double* max_speed) {
  m1_rhs_impl(g, par, U, P, aux, rhs, NULL, max_speed);
}

/* as orc_m1_rhs, but the radiation's collision terms (the stiff part of the
 * IMEX splitting) go to stiff (12 fields) instead of rhs; the fluid's opposite
 * exchange stays in rhs (explicit), or with par->couple_exchange goes to the
 * stiff slots after the radiation's (tau, then S_i; orc_imex_stiff_fields) */
void orc_m1_rhs_split(const orc_grid* g, const orc_par* par, const double* U, const double* P,
                      const double* aux, double* rhs, double* stiff, double* max_speed) {
  m1_rhs_impl(g, par, U, P, aux, rhs, stiff, max_speed);
}

/* G(V) = V - V* - adt alpha (S_n, S_i)(V) of one species at one point, undensitized,
 * with the closure's Eddington factor frozen at chi */
static void implicit_residual(const m1_state* s0, double chi, const double V[4], const double Vs[4], double adt,
                              double alp, double ka, double ks, double eta, double G[4]) {
  m1_state s;
  double P[3][3], J, H[3], Hn, HH, Sn, Si[3];
  int a;
  state_init(&s, V[0], V + 1, s0->v, s0->W, s0->gdn, s0->gup);
  closure_eval(&s, chi, P, &J, H, &Hn, &HH);
  Sn = s.W * ((eta + ks * J) - (ka + ks) * (s.E - s.vF));
  for (a = 0; a < 3; ++a) Si[a] = s.W * (eta - ka * J) * s.vd[a] - (ka + ks) * H[a];
  G[0] = V[0] - Vs[0] - adt * alp * Sn;
  for (a = 0; a < 3; ++a) G[1 + a] = V[1 + a] - Vs[1 + a] - adt * alp * Si[a];
}

/* dG/dV = I - adt calJ with calJ = d(alpha (S_n, S_i))/d(E, F_j) as App. C
 * prints it: J and H_i of the Minerbo closure with the Eddington factor chi
 * frozen, written as functions of (E, F_i), and their derivatives
 *   dJ/dE     = W^2 + d_thin (v.fh)^2 W^2 + d_thick (3 - 2W^2)(W^2 - 1)/(1 + 2W^2)
 *   dJ/dF_j   = 2W^2 (-1 + d_thin E (v.fh)/F + 2 d_thick (W^2-1)/(1+2W^2)) v^j
 *               - 2 d_thin W^2 E (v.fh)^2 / F fh^j
 *   dH_i/dE   = W^3 (-1 - d_thin (v.fh)^2 + d_thick (2W^2-3)/(1+2W^2)) v_i
 *               - d_thin W (v.fh) fh_i
 *   dH_i/dF_j = W (1 - d_thin E (v.fh)/F - d_thick v^2) delta_i^j
 *               + 2W^3 [1 - d_thin E (v.fh)/F - d_thick (v^2 + 1/(2W^2 (1+2W^2)))] v_i v^j
 *               + 2 d_thin W E (v.fh)/F fh_i fh^j + 2 d_thin W^3 E (v.fh)^2/F v_i fh^j
 *               - d_thin W E/F fh_i v^j
 * with F = sqrt(F_k F^k), fh_i = F_i/F, kappa_as = kappa_a + kappa_s, and
 *   calJ_00 = -alpha W (kappa_as - kappa_s dJ/dE)
 *   calJ_0j = alpha W (kappa_s dJ/dF_j + kappa_as v^j)
 *   calJ_i0 = -alpha (kappa_as dH_i/dE + W kappa_a dJ/dE v_i)
 *   calJ_ij = -alpha (kappa_as dH_i/dF_j + W kappa_a v_i dJ/dF_j).
 * Where F_k F^k = 0 the thin terms with fh are dropped (the closure drops
 * P^thin there). */
static void implicit_jacobian(const m1_state* s, double chi, double adt, double alp, double ka, double ks,
                              double Jm[4][4]) {
  const double W = s->W, W2 = W * W, W3 = W2 * W;
  const double dthick = 1.5 * (1.0 - chi), dthin = 1.0 - dthick;
  const double kas = ka + ks;
  const double F = sqrt(s->F2);
  double fh[3] = {0.0, 0.0, 0.0}, fhu[3] = {0.0, 0.0, 0.0}, vfh = 0.0, v2 = 0.0;
  double dJdE, dJdF[3], dHdE[3], dHdF[3][3], cal[4][4];
  int i, j;
  for (i = 0; i < 3; ++i) v2 += s->v[i] * s->vd[i];
  if (F > 0.0) {
    for (i = 0; i < 3; ++i) {
      fh[i] = s->F[i] / F;
      fhu[i] = s->Fu[i] / F;
    }
    vfh = s->vF / F;
  }
  {
    const double tE = F > 0.0 ? s->E * vfh / F : 0.0;       /* E (v.fh)/F */
    const double tE2 = F > 0.0 ? s->E * vfh * vfh / F : 0.0; /* E (v.fh)^2/F */
    const double tE0 = F > 0.0 ? s->E / F : 0.0;             /* E/F */
    dJdE = W2 + dthin * vfh * vfh * W2 + dthick * (3.0 - 2.0 * W2) * (W2 - 1.0) / (1.0 + 2.0 * W2);
    for (j = 0; j < 3; ++j)
      dJdF[j] = 2.0 * W2 * (-1.0 + dthin * tE + 2.0 * dthick * (W2 - 1.0) / (1.0 + 2.0 * W2)) * s->v[j] -
                2.0 * dthin * W2 * tE2 * fhu[j];
    for (i = 0; i < 3; ++i)
      dHdE[i] = W3 * (-1.0 - dthin * vfh * vfh + dthick * (2.0 * W2 - 3.0) / (1.0 + 2.0 * W2)) * s->vd[i] -
                dthin * W * vfh * fh[i];
    for (i = 0; i < 3; ++i)
      for (j = 0; j < 3; ++j)
        dHdF[i][j] = W * (1.0 - dthin * tE - dthick * v2) * (i == j ? 1.0 : 0.0) +
                     2.0 * W3 * (1.0 - dthin * tE - dthick * (v2 + 1.0 / (2.0 * W2 * (1.0 + 2.0 * W2)))) *
                         s->vd[i] * s->v[j] +
                     2.0 * dthin * W * tE * fh[i] * fhu[j] + 2.0 * dthin * W3 * tE2 * s->vd[i] * fhu[j] -
                     dthin * W * tE0 * fh[i] * s->v[j];
  }
  cal[0][0] = -alp * W * (kas - ks * dJdE);
  for (j = 0; j < 3; ++j) cal[0][1 + j] = alp * W * (ks * dJdF[j] + kas * s->v[j]);
  for (i = 0; i < 3; ++i) {
    cal[1 + i][0] = -alp * (kas * dHdE[i] + W * ka * dJdE * s->vd[i]);
    for (j = 0; j < 3; ++j) cal[1 + i][1 + j] = -alp * (kas * dHdF[i][j] + W * ka * s->vd[i] * dJdF[j]);
  }
  for (i = 0; i < 4; ++i)
    for (j = 0; j < 4; ++j) Jm[i][j] = (i == j ? 1.0 : 0.0) - adt * cal[i][j];
}

/* Residual and App. C Jacobian of the implicit M1 equation at one point, for
 * the pins: metric gdn (6 components xx,xy,xz,yy,yz,zz), fluid v^i and W, the
 * trial V = (E, F_i) and V*, the frozen Eddington factor chi. */
void orc_m1_implicit_point(const double gd6[6], const double v[3], double W, const double V[4], const double Vs[4],
                           double chi, double adt, double alp, double ka, double ks, double eta, double G[4],
                           double Jac[16]) {
  double gdn[3][3], gup[3][3], det, Jm[4][4];
  m1_state s;
  int i, j;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) gdn[i][j] = gd6[S6m[i][j]];
  det = gdn[0][0] * (gdn[1][1] * gdn[2][2] - gdn[1][2] * gdn[2][1]) -
        gdn[0][1] * (gdn[1][0] * gdn[2][2] - gdn[1][2] * gdn[2][0]) +
        gdn[0][2] * (gdn[1][0] * gdn[2][1] - gdn[1][1] * gdn[2][0]);
  gup[0][0] = (gdn[1][1] * gdn[2][2] - gdn[1][2] * gdn[2][1]) / det;
  gup[0][1] = (gdn[0][2] * gdn[2][1] - gdn[0][1] * gdn[2][2]) / det;
  gup[0][2] = (gdn[0][1] * gdn[1][2] - gdn[0][2] * gdn[1][1]) / det;
  gup[1][1] = (gdn[0][0] * gdn[2][2] - gdn[0][2] * gdn[2][0]) / det;
  gup[1][2] = (gdn[0][2] * gdn[1][0] - gdn[0][0] * gdn[1][2]) / det;
  gup[2][2] = (gdn[0][0] * gdn[1][1] - gdn[0][1] * gdn[1][0]) / det;
  gup[1][0] = gup[0][1];
  gup[2][0] = gup[0][2];
  gup[2][1] = gup[1][2];
  {
    m1_state s0;
    state_init(&s0, Vs[0], Vs + 1, v, W, gdn, gup);
    implicit_residual(&s0, chi, V, Vs, adt, alp, ka, ks, eta, G);
  }
  state_init(&s, V[0], V + 1, v, W, gdn, gup);
  implicit_jacobian(&s, chi, adt, alp, ka, ks, Jm);
  for (i = 0; i < 4; ++i)
    for (j = 0; j < 4; ++j) Jac[4 * i + j] = Jm[i][j];
}

/* solve the 4x4 system A x = b by Gaussian elimination with partial pivoting */
static int solve4(double A[4][4], double b[4], double x[4]) {
  int i, j, k;
  for (k = 0; k < 4; ++k) {
    int piv = k;
    for (i = k + 1; i < 4; ++i)
      if (fabs(A[i][k]) > fabs(A[piv][k])) piv = i;
    if (A[piv][k] == 0.0) return 0;
    if (piv != k) {
      for (j = 0; j < 4; ++j) {
        double t = A[k][j];
        A[k][j] = A[piv][j];
        A[piv][j] = t;
      }
      {
        double t = b[k];
        b[k] = b[piv];
        b[piv] = t;
      }
    }
    for (i = k + 1; i < 4; ++i) {
      double f = A[i][k] / A[k][k];
      for (j = k; j < 4; ++j) A[i][j] -= f * A[k][j];
      b[i] -= f * b[k];
    }
  }
  for (i = 3; i >= 0; --i) {
    double t = b[i];
    for (j = i + 1; j < 4; ++j) t -= A[i][j] * x[j];
    x[i] = t / A[i][i];
  }
  return 1;
}

/* Implicit M1 update of an IMEX stage (App. C): at every interior point and
 * species, V = (E, F_i) solves V = V* + adt alpha (S_n, S_i)(V) with V* the
 * radiation fields on input (densitized in U; the equations are solved
 * undensitized), the fluid state from P and the closure's Eddington factor
 * frozen at its value for V*.  Newton's method with App. C's Jacobian
 * (implicit_jacobian), at most 60 iterations.  Converged when |dV| <= 1e-15 (E + |F|), or
 * when an update no larger than 1e-9 (E + |F|) is not below half of the one
 * before it: Newton has stopped contracting and rounding decides the last
 * digits (App. C leaves the stopping rule open).  A solve that does not
 * converge keeps the first Newton iterate, which is App. C's linearised
 * implicit update about V' = V* (one solve with the Jacobian at V*).  Returns
 * the number of solves that did not converge. */
int64_t orc_m1_implicit(const orc_grid* g, double* U, const double* P, const double* aux, double adt) {
  return orc_m1_implicit_x(g, U, P, aux, adt, 0);
}

/* as orc_m1_implicit; with couple != 0 the fluid's taubar and Sbar_i then lose
 * what each species' Ebar and Fbar_i gained in its solve (the stiff exchange
 * taken implicitly by both sides, as it is evaluated in the stiff slots of
 * the split right-hand side) */
int64_t orc_m1_implicit_x(const orc_grid* g, double* U, const double* P, const double* aux, double adt,
                          int couple) {
  const int ng = g->ng;
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = npts(g);
  int64_t bad = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : bad)
  for (int64_t k = ng; k < Nz - ng; ++k)
    for (int64_t j = ng; j < Ny - ng; ++j)
      for (int64_t i = ng; i < Nx - ng; ++i) {
        const int64_t q = i + Nx * (j + Ny * k);
        const double alp = U[18 * N + q];
        m1_metric m;
        int sp;
        m1_metric_at(U, N, q, &m);
        for (sp = 0; sp < 3; ++sp) {
          const double ka = aux[(3 * sp) * N + q], ks = aux[(3 * sp + 1) * N + q], eta = aux[(3 * sp + 2) * N + q];
          m1_state s0;
          double Pij[3][3], J, H[3], chi, Vs[4], V[4];
          int it, a, ok = 0;
          point_state(U, P, N, q, sp, &m, &s0);
          closure(&s0, Pij, &J, H, &chi, NULL);
          Vs[0] = s0.E;
          for (a = 0; a < 3; ++a) Vs[1 + a] = s0.F[a];
          for (a = 0; a < 4; ++a) V[a] = Vs[a];
          double prev = HUGE_VAL, V1[4];
          for (a = 0; a < 4; ++a) V1[a] = Vs[a];
          for (it = 0; it < 60; ++it) {
            double G[4], Jm[4][4], dV[4], scale = fabs(V[0]) + fabs(V[1]) + fabs(V[2]) + fabs(V[3]), nrm = 0.0;
            implicit_residual(&s0, chi, V, Vs, adt, alp, ka, ks, eta, G);
            {
              m1_state sv;
              state_init(&sv, V[0], V + 1, s0.v, s0.W, s0.gdn, s0.gup);
              implicit_jacobian(&sv, chi, adt, alp, ka, ks, Jm);
            }
            for (a = 0; a < 4; ++a) G[a] = -G[a];
            if (!solve4(Jm, G, dV)) break;
            for (a = 0; a < 4; ++a) {
              V[a] += dV[a];
              nrm += fabs(dV[a]);
            }
            if (it == 0)
              for (a = 0; a < 4; ++a) V1[a] = V[a];
            if (nrm <= 1e-15 * scale || (nrm <= 1e-9 * scale && nrm >= 0.5 * prev)) {
              ok = 1;
              break;
            }
            prev = nrm;
          }
          if (!ok) {
            bad += 1;
            for (a = 0; a < 4; ++a) V[a] = V1[a];
          }
          {
            const double E0 = U[(32 + 4 * sp) * N + q];
            U[(32 + 4 * sp) * N + q] = m.sqrtg * V[0];
            if (couple) U[24 * N + q] -= U[(32 + 4 * sp) * N + q] - E0;
          }
          for (a = 0; a < 3; ++a) {
            const double F0 = U[(33 + 4 * sp + a) * N + q];
            U[(33 + 4 * sp + a) * N + q] = m.sqrtg * V[1 + a];
            if (couple) U[(25 + a) * N + q] -= U[(33 + 4 * sp + a) * N + q] - F0;
          }
        }
      }
  return bad;
}

/* ---- neutrino number densities (Sec. 2.3; App. C) --------------------------
 * Per species s the evolved field is Nbar = sqrt(gamma) N at U index 44 + s;
 * the number absorption coefficient kappa0_a and emissivity eta0 sit at
 * aux[(9 + 2 s) N + p] and aux[(10 + 2 s) N + p].  With J and H_i of the
 * Minerbo closure at the point, the number current N^a = n (u^a + H^a/J)
 * gives the d_k-flux
 *   Fbar_N^k = (-W beta^k + alpha W v^k + alpha H^k/J) Nbar/Gamma,
 *   Gamma = W (E - F_i v^i)/J,
 * where H^k is the spatial component of the four-vector
 * H^a = -(H^b n_b) n^a + gamma^a_b H^b, i.e. H^k = gamma^kj H_j + H_n beta^k/alpha
 * with H_n = H^b n_b = W (J - E + F_i v^i) (the relations below the M1
 * equations in Sec. 2.3);
 * and the source alpha sqrt(gamma) C with C = eta0 - kappa0_a N/Gamma.  The
 * electron fraction gains -alpha sqrt(gamma) m_b (C_0 - C_1) (species 0 the
 * electron neutrino, 1 its antineutrino).
 * Readings: H^k as above (with the spatial projection alone the shift term
 * would not reduce to -beta^k Nbar); Nbar's interfaces take the HO/LO splitting of the energy moments
 * (Sec. 3.4) with the species' point speed and its kappa_a + kappa_s in the
 * opacity switch (the text gives one scheme for the radiation fields); the
 * electron-fraction source stays explicit, as the fluid's energy and momentum
 * exchange does. */
void orc_m1n_rhs(const orc_grid* g, const orc_par* par, const double* U, const double* P, const double* aux,
                 double* rhs, double* stiff) {
  const int ng = g->ng;
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = npts(g);
  const int64_t st[3] = {1, Nx, Nx * Ny};
  double* FN = (double*)malloc(sizeof(double) * 3 * 3 * N);
  double* LM = (double*)malloc(sizeof(double) * 3 * 3 * N);
  double* GM = (double*)malloc(sizeof(double) * 3 * N);
  int64_t p;

#pragma omp parallel for schedule(static)
  for (p = 0; p < N; ++p) {
    m1_metric m;
    int sp, d, j;
    const double alp = U[18 * N + p];
    m1_metric_at(U, N, p, &m);
    for (sp = 0; sp < 3; ++sp) {
      m1_state s;
      double Pij[3][3], J, H[3], chi, Hu[3], gam;
      const double Nb = U[(44 + sp) * N + p];
      point_state(U, P, N, p, sp, &m, &s);
      closure(&s, Pij, &J, H, &chi, NULL);
      for (d = 0; d < 3; ++d) {
        Hu[d] = s.W * (J - s.E + s.vF) * U[(19 + d) * N + p] / alp;
        for (j = 0; j < 3; ++j) Hu[d] += m.gup[d][j] * H[j];
      }
      gam = s.W * (s.E - s.vF) / J;
      GM[sp * N + p] = gam;
      for (d = 0; d < 3; ++d) {
        const double bd = U[(19 + d) * N + p];
        FN[(sp * 3 + d) * N + p] = (-s.W * bd + alp * s.W * s.v[d] + alp * Hu[d] / J) * Nb / gam;
        LM[(sp * 3 + d) * N + p] = speed(&s, chi, alp, bd, d);
      }
    }
  }

#pragma omp parallel for collapse(2) schedule(static)
  for (int64_t k = ng; k < Nz - ng; ++k)
    for (int64_t j = ng; j < Ny - ng; ++j)
      for (int64_t i = ng; i < Nx - ng; ++i) {
        const int64_t q = i + Nx * (j + Ny * k);
        const double alp = U[18 * N + q];
        m1_metric m;
        double C[3];
        int sp, d;
        m1_metric_at(U, N, q, &m);
        for (sp = 0; sp < 3; ++sp) {
          const double* u = U + (44 + sp) * N;
          const double* kap = aux + (3 * sp) * N;
          const double* kas = aux + (3 * sp + 1) * N;
          const double k0 = aux[(9 + 2 * sp) * N + q], e0 = aux[(10 + 2 * sp) * N + q];
          double out = 0.0;
          for (d = 0; d < 3; ++d) {
            const double* f = FN + (sp * 3 + d) * N;
            const double* lam = LM + (sp * 3 + d) * N;
            const double fr = holo(u, f, lam, kap, kas, q, st[d], g->dx[d]);
            const double fl = holo(u, f, lam, kap, kas, q - st[d], st[d], g->dx[d]);
            out -= (fr - fl) / g->dx[d];
          }
          C[sp] = e0 - k0 * (u[q] / m.sqrtg) / GM[sp * N + q];
          if (stiff)
            stiff[(12 + sp) * N + q] = alp * m.sqrtg * C[sp];
          else
            out += alp * m.sqrtg * C[sp];
          rhs[(44 + sp) * N + q] = out;
        }
        if (stiff && par->couple_exchange)
          stiff[(15 + 4) * N + q] = -alp * m.sqrtg * par->m_b * (C[0] - C[1]);
        else
          rhs[23 * N + q] -= alp * m.sqrtg * par->m_b * (C[0] - C[1]);
      }
  free(FN);
  free(LM);
  free(GM);
}

/* After the stage's E and F_i are updated: per interior point and species,
 * N = (N* + adt alpha eta0)/(1 + adt alpha kappa0_a/Gamma), with N* the number
 * density on input (undensitized) and Gamma from the updated E, F_i and their
 * closure (App. C). */
void orc_m1n_implicit(const orc_grid* g, double* U, const double* P, const double* aux, double adt) {
  orc_m1n_implicit_x(g, U, P, aux, adt, 0, 0.0);
}

/* as orc_m1n_implicit; with couple != 0, DYebar then changes by -m_b times
 * the change of (Nbar_nue - Nbar_nuebar), the electron fraction's stiff source
 * taken implicitly with the number densities */
void orc_m1n_implicit_x(const orc_grid* g, double* U, const double* P, const double* aux, double adt, int couple,
                        double m_b) {
  const int ng = g->ng;
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = npts(g);
#pragma omp parallel for collapse(2) schedule(static)
  for (int64_t k = ng; k < Nz - ng; ++k)
    for (int64_t j = ng; j < Ny - ng; ++j)
      for (int64_t i = ng; i < Nx - ng; ++i) {
        const int64_t q = i + Nx * (j + Ny * k);
        const double alp = U[18 * N + q];
        m1_metric m;
        double dN[3];
        int sp;
        m1_metric_at(U, N, q, &m);
        for (sp = 0; sp < 3; ++sp) {
          m1_state s;
          double Pij[3][3], J, H[3], chi, gam, Ns;
          const double k0 = aux[(9 + 2 * sp) * N + q], e0 = aux[(10 + 2 * sp) * N + q];
          point_state(U, P, N, q, sp, &m, &s);
          closure(&s, Pij, &J, H, &chi, NULL);
          gam = s.W * (s.E - s.vF) / J;
          Ns = U[(44 + sp) * N + q] / m.sqrtg;
          dN[sp] = -U[(44 + sp) * N + q];
          U[(44 + sp) * N + q] = m.sqrtg * (Ns + adt * alp * e0) / (1.0 + adt * alp * k0 / gam);
          dN[sp] += U[(44 + sp) * N + q];
        }
        if (couple) U[23 * N + q] -= m_b * (dN[0] - dN[1]);
      }
}
