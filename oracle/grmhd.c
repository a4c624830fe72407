/*
 * Oracle (test infrastructure only): GRMHD part of the right-hand side,
 * Sec. 2.2 (balance laws with divergence cleaning, eq. for Dbar ... phibar),
 * Sec. 3.3 (conservative form, Lax-Friedrichs splitting F^pm = (F +- lambda U)/2,
 * MP5 on F^+ (left) and mirrored on F^- (right), Fhat = F^L + F^R),
 * App. B (fast-magnetosonic bound for normal propagation).
 *
 * Readings:
 *   - lambda at interface i+1/2 is the maximum of the point speeds over the
 *     six reconstruction points i-2..i+3; the point speed is the largest of
 *     |lambda_fast^+-| and |-beta^k +- alpha c_b sqrt(gamma^kk)| (the cleaning
 *     mode), and one lambda serves all 10 fields;
 *   - c_s^2 for a general p(rho,eps) (the printed Gamma p/h is the ideal gas case);
 *   - a negative radicand in the fast speed (rounding) is taken as zero;
 *   - metric derivatives in the sources are the centred 4th-order ones.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"

void orc_matter_point(const double* U, const double* P, int64_t N, int64_t p,
                      const double gdn[3][3], double sqrtg, double* E, double S[3],
                      double Sij[3][3]);

static const int S6[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

typedef struct {
  double gt[3][3], gtu[3][3], chi, gdn[3][3], gup[3][3], sqrtg, det;
} metric_t;

static void metric(const double* U, int64_t N, int64_t p, metric_t* m) {
  int i, j;
  double (*g)[3] = m->gt;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) g[i][j] = U[S6[i][j] * N + p];
  m->chi = U[12 * N + p];
  m->det = g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1]) - g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0])
           + g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
  m->gtu[0][0] = (g[1][1] * g[2][2] - g[1][2] * g[2][1]) / m->det;
  m->gtu[0][1] = (g[0][2] * g[2][1] - g[0][1] * g[2][2]) / m->det;
  m->gtu[0][2] = (g[0][1] * g[1][2] - g[0][2] * g[1][1]) / m->det;
  m->gtu[1][1] = (g[0][0] * g[2][2] - g[0][2] * g[2][0]) / m->det;
  m->gtu[1][2] = (g[0][2] * g[1][0] - g[0][0] * g[1][2]) / m->det;
  m->gtu[2][2] = (g[0][0] * g[1][1] - g[0][1] * g[1][0]) / m->det;
  m->gtu[1][0] = m->gtu[0][1];
  m->gtu[2][0] = m->gtu[0][2];
  m->gtu[2][1] = m->gtu[1][2];
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      m->gdn[i][j] = g[i][j] / m->chi;
      m->gup[i][j] = m->chi * m->gtu[i][j];
    }
  m->sqrtg = sqrt(m->det / (m->chi * m->chi * m->chi));
}

/* point flux along direction d of the 10 densitized MHD fields, and the point speed */
static void point_flux(const orc_par* par, const orc_eos* e, const double* U, const double* P,
                       int64_t N, int64_t p, int d, double F[10], double* lam) {
  metric_t m;
  double alp, beta[3], v[3], vd[3], B[3], Bd[3], Sbar[3], Sij[3][3], E, Sm[3];
  double B2 = 0.0, Bv = 0.0, v2 = 0.0, rho, eps, pr, W, h, b2, cs2, ca2, a2;
  double Dbar, DYbar, taubar, phibar, Sup_d, vk;
  int i, j;
  metric(U, N, p, &m);
  alp = U[18 * N + p];
  for (i = 0; i < 3; ++i) {
    beta[i] = U[(19 + i) * N + p];
    v[i] = P[(3 + i) * N + p];
    B[i] = U[(28 + i) * N + p] / m.sqrtg;
    Sbar[i] = U[(25 + i) * N + p];
  }
  for (i = 0; i < 3; ++i) {
    vd[i] = 0.0;
    Bd[i] = 0.0;
    for (j = 0; j < 3; ++j) {
      vd[i] += m.gdn[i][j] * v[j];
      Bd[i] += m.gdn[i][j] * B[j];
    }
  }
  for (i = 0; i < 3; ++i) {
    B2 += B[i] * Bd[i];
    Bv += B[i] * vd[i];
    v2 += v[i] * vd[i];
  }
  Dbar = U[22 * N + p];
  DYbar = U[23 * N + p];
  taubar = U[24 * N + p];
  phibar = U[31 * N + p];
  vk = v[d];
  orc_matter_point(U, P, N, p, m.gdn, m.sqrtg, &E, Sm, Sij);

  F[0] = (-beta[d] + alp * vk) * Dbar;
  F[1] = (-beta[d] + alp * vk) * DYbar;
  Sup_d = 0.0;
  for (j = 0; j < 3; ++j) Sup_d += m.gup[d][j] * Sbar[j];
  F[2] = -beta[d] * taubar + alp * (Sup_d - Dbar * vk);
  for (i = 0; i < 3; ++i) {
    double Smix = 0.0; /* S^d_i = gamma^{dj} S_ji, densitized */
    for (j = 0; j < 3; ++j) Smix += m.gup[d][j] * Sij[j][i];
    F[3 + i] = -beta[d] * Sbar[i] + alp * m.sqrtg * Smix;
  }
  for (i = 0; i < 3; ++i) {
    double Bbar_i = U[(28 + i) * N + p], Bbar_d = U[(28 + d) * N + p];
    F[6 + i] = Bbar_i * (alp * vk - beta[d]) - Bbar_d * (alp * v[i] - beta[i])
               + alp * m.chi * m.gtu[d][i] * phibar;
  }
  F[9] = -beta[d] * phibar + alp * par->c_b * par->c_b * U[(28 + d) * N + p];

  /* speeds (App. B) */
  rho = P[0 * N + p];
  eps = P[1 * N + p];
  pr = P[2 * N + p];
  W = P[6 * N + p];
  h = rho * (1.0 + eps) + pr;
  b2 = B2 / (W * W) + Bv * Bv;
  cs2 = orc_cs2(e, rho, eps);
  ca2 = b2 / (h + b2);
  a2 = cs2 + ca2 - cs2 * ca2;
  {
    double gdd = m.gup[d][d];
    double rad = a2 * (1.0 - v2) * ((1.0 - v2 * a2) * gdd - (1.0 - a2) * vk * vk);
    double sq = sqrt(fmax(rad, 0.0));
    double lp = -beta[d] + alp / (1.0 - v2 * a2) * ((1.0 - a2) * vk + sq);
    double lm = -beta[d] + alp / (1.0 - v2 * a2) * ((1.0 - a2) * vk - sq);
    double cp = -beta[d] + alp * par->c_b * sqrt(gdd);
    double cm = -beta[d] - alp * par->c_b * sqrt(gdd);
    *lam = fmax(fmax(fabs(lp), fabs(lm)), fmax(fabs(cp), fabs(cm)));
  }
}

static int64_t npts(const orc_grid* g) {
  return (int64_t)(g->n[0] + 2 * g->ng) * (g->n[1] + 2 * g->ng) * (g->n[2] + 2 * g->ng);
}

/* numerical flux at interface between p and p+s (i.e. i+1/2 with i = p) */
static double iface_flux(const double* Ff, const double* Uf, const double* lam, int64_t p,
                         int64_t s, double alpha_mp5) {
  double l = 0.0, fp[5], fm[5], r;
  int m;
  ORC_PHASE(ORC_PH_MHD_RECON);
  for (m = -2; m <= 3; ++m) l = fmax(l, lam[p + m * s]);
  for (m = 0; m < 5; ++m) {
    int64_t q = p + (m - 2) * s;        /* i-2 .. i+2 */
    int64_t r = p + (3 - m) * s;        /* i+3 .. i-1 */
    fp[m] = 0.5 * (Ff[q] + l * Uf[q]);
    fm[m] = 0.5 * (Ff[r] - l * Uf[r]);
  }
  r = orc_mp5(fp, alpha_mp5) + orc_mp5(fm, alpha_mp5);
  ORC_PHASE(ORC_PH_MHD_UPD);
  return r;
}

/* GRMHD contribution for all interior points: rhs[22..31] (overwritten). */
void orc_grmhd_rhs(const orc_grid* g, const orc_par* par, const orc_eos* e, const double* U,
                   const double* P, double* rhs, double* max_speed) {
  const int ng = g->ng;
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = npts(g);
  const int64_t st[3] = {1, Nx, Nx * Ny};
  double* F = (double*)malloc(sizeof(double) * 30 * N);
  double* lam = (double*)malloc(sizeof(double) * 3 * N);
  double vmax = 0.0;
  int64_t p;
  int d;

  ORC_PHASE(ORC_PH_MHD_POINT);
#pragma omp parallel for schedule(static)
  for (p = 0; p < N; ++p) {
    int dd, f;
    for (dd = 0; dd < 3; ++dd) {
      double Fp[10], l;
      point_flux(par, e, U, P, N, p, dd, Fp, &l);
      for (f = 0; f < 10; ++f) F[(dd * 10 + f) * N + p] = Fp[f];
      lam[dd * N + p] = l;
    }
  }

  ORC_PHASE(ORC_PH_MHD_UPD);
#pragma omp parallel for collapse(2) schedule(static) reduction(max : vmax)
  for (int64_t k = ng; k < Nz - ng; ++k)
    for (int64_t j = ng; j < Ny - ng; ++j)
      for (int64_t i = ng; i < Nx - ng; ++i) {
        int64_t q = i + Nx * (j + Ny * k);
        double out[10];
        double h[3] = {g->dx[0], g->dx[1], g->dx[2]};
        int f, dd;
        for (f = 0; f < 10; ++f) out[f] = 0.0;
        for (dd = 0; dd < 3; ++dd) {
          vmax = fmax(vmax, lam[dd * N + q]);
          for (f = 0; f < 10; ++f) {
            const double* Ff = F + (dd * 10 + f) * N;
            const double* Uf = U + (22 + f) * N;
            double fr = iface_flux(Ff, Uf, lam + dd * N, q, st[dd], par->alpha_mp5);
            double fl = iface_flux(Ff, Uf, lam + dd * N, q - st[dd], st[dd], par->alpha_mp5);
            out[f] -= (fr - fl) / h[dd];
          }
        }
        /* sources */
        {
          metric_t m;
          double alp = U[18 * N + q], Kh = U[13 * N + q], Th = U[14 * N + q];
          double dalp[3], dbeta[3][3], dgt[3][3][3], dchi[3], Gt[3], Z[3], Gh[3];
          double E, Sm[3], Sij[3][3], Supup[3][3], trS = 0.0, Sup[3];
          double Dbar = U[22 * N + q], taubar = U[24 * N + q], phibar = U[31 * N + q];
          double Bbar[3], Sbar[3], cb2 = par->c_b * par->c_b;
          int i2, j2, k2, l2;
          metric(U, N, q, &m);
          for (dd = 0; dd < 3; ++dd) {
            dalp[dd] = orc_d1(U + 18 * N, q, st[dd], h[dd]);
            dchi[dd] = orc_d1(U + 12 * N, q, st[dd], h[dd]);
            for (i2 = 0; i2 < 3; ++i2) dbeta[dd][i2] = orc_d1(U + (19 + i2) * N, q, st[dd], h[dd]);
            for (i2 = 0; i2 < 3; ++i2)
              for (j2 = 0; j2 < 3; ++j2) dgt[dd][i2][j2] = orc_d1(U + S6[i2][j2] * N, q, st[dd], h[dd]);
          }
          for (i2 = 0; i2 < 3; ++i2) {
            Gh[i2] = U[(15 + i2) * N + q];
            Bbar[i2] = U[(28 + i2) * N + q];
            Sbar[i2] = U[(25 + i2) * N + q];
            Gt[i2] = 0.0;
            for (j2 = 0; j2 < 3; ++j2)
              for (k2 = 0; k2 < 3; ++k2)
                for (l2 = 0; l2 < 3; ++l2) Gt[i2] += m.gtu[i2][j2] * m.gtu[k2][l2] * dgt[l2][j2][k2];
            Z[i2] = 0.5 * m.chi * (Gh[i2] - Gt[i2]);
          }
          orc_matter_point(U, P, N, q, m.gdn, m.sqrtg, &E, Sm, Sij);
          /* Sbar^{ij} = sqrt(gamma) gamma^{ik} gamma^{jl} S_kl ; trSbar = gamma_jk Sbar^{jk} */
          for (i2 = 0; i2 < 3; ++i2)
            for (j2 = 0; j2 < 3; ++j2) {
              double s = 0.0;
              for (k2 = 0; k2 < 3; ++k2)
                for (l2 = 0; l2 < 3; ++l2) s += m.gup[i2][k2] * m.gup[j2][l2] * Sij[k2][l2];
              Supup[i2][j2] = m.sqrtg * s;
            }
          for (i2 = 0; i2 < 3; ++i2)
            for (j2 = 0; j2 < 3; ++j2) trS += m.gdn[i2][j2] * Supup[i2][j2];
          for (i2 = 0; i2 < 3; ++i2) {
            Sup[i2] = 0.0;
            for (j2 = 0; j2 < 3; ++j2) Sup[i2] += m.gup[i2][j2] * Sbar[j2];
          }
          /* taubar */
          {
            double s = 0.0;
            for (i2 = 0; i2 < 3; ++i2)
              for (j2 = 0; j2 < 3; ++j2) s += alp / m.chi * Supup[i2][j2] * U[(6 + S6[i2][j2]) * N + q];
            s += alp / 3.0 * trS * (Kh + 2.0 * Th);
            for (j2 = 0; j2 < 3; ++j2) s -= Sup[j2] * dalp[j2];
            out[2] += s;
          }
          /* Sbar_i */
          for (i2 = 0; i2 < 3; ++i2) {
            double s = 0.0;
            for (j2 = 0; j2 < 3; ++j2)
              for (k2 = 0; k2 < 3; ++k2) s += Supup[j2][k2] * dgt[i2][j2][k2];
            s = alp / (2.0 * m.chi) * (s - trS * dchi[i2]);
            for (j2 = 0; j2 < 3; ++j2) s += Sbar[j2] * dbeta[i2][j2];
            s -= (taubar + Dbar) * dalp[i2];
            out[3 + i2] += s;
          }
          /* Bbar^i */
          for (i2 = 0; i2 < 3; ++i2) {
            double s = -alp * (m.chi * Gh[i2] - 2.0 * Z[i2]);
            for (k2 = 0; k2 < 3; ++k2)
              s += m.gtu[k2][i2] * (-0.5 * alp * dchi[k2] + m.chi / cb2 * dalp[k2]);
            out[6 + i2] += phibar * s;
          }
          /* phibar */
          {
            double s = -alp * cb2 * phibar * (Kh + 2.0 * Th) - alp * par->kappa_b * phibar;
            for (k2 = 0; k2 < 3; ++k2) s += cb2 * Bbar[k2] * dalp[k2];
            out[9] += s;
          }
        }
        for (f = 0; f < 10; ++f) rhs[(22 + f) * N + q] = out[f];
      }
  ORC_PHASE(ORC_PH_OTHER);
  free(F);
  free(lam);
  if (max_speed) *max_speed = vmax;
  (void)d;
}
