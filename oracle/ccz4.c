/*
 * Oracle (test infrastructure only): CCZ4 right-hand side at one interior point,
 * Sec. 2.1 of the paper:
 *   evolution equations for gt_ij, At_ij, chi, Khat, Theta, Ghat^i,
 *   Ricci split R_ij + 2 D_(i Z_j) = Rhat_ij + Rhat^chi_ij,
 *   Laplacian of the lapse, gauge (1+log / harmonic slicing, Gamma-freezing shift),
 *   matter projections tau (= n n T), S_i, S_ij (Sec. 2.2 for the fluid part).
 * Centred 4th-order derivatives everywhere except advection terms beta^k d_k,
 * which use the one-sided operator (Sec. 3.2); Kreiss-Oliger dissipation is
 * added on all 22 fields.
 *
 * Readings where the paper is not explicit:
 *   - the conformal trace is At = gt^{ij} At_ij (trace w.r.t. the conformal metric);
 *   - Gt^i (tilde) is computed from derivatives of gt_ij as printed,
 *     Gt^i = gt^{ij} gt^{kl} d_l gt_jk; Ghat^i is the evolved field;
 *   - D_i D_j alpha = d_i d_j alpha - Gamma^k_ij d_k alpha with the physical
 *     Christoffels from the conformal ones and chi;
 *   - the CCZ4 energy density is tau_ccz4 = (taubar + Dbar)/sqrt(gamma);
 *   - kappa_2 is a free parameter (default 0).
 */
#include <math.h>
#include "orc.h"

static const int S6[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

static double fld(const double* U, int f, int64_t N, int64_t p) { return U[f * N + p]; }

static double dd(const double* u, int64_t p, const int64_t st[3], const double h[3], int k, int l) {
  if (k == l) return orc_d2(u, p, st[k], h[k]);
  return orc_d11(u, p, st[k], st[l], h[k], h[l]);
}

/* matter projections of the magnetized fluid at point p (Sec. 2.2):
 * energy density E = tau + D, momentum S_i, stress S_ij (lower indices) */
void orc_matter_point(const double* U, const double* P, int64_t N, int64_t p,
                      const double gdn[3][3], double sqrtg, double* E, double S[3],
                      double Sij[3][3]) {
  double v[3], vd[3], B[3], Bd[3], B2 = 0.0, Bv = 0.0, W, pr;
  int i, j;
  for (i = 0; i < 3; ++i) {
    v[i] = P[(3 + i) * N + p];
    B[i] = U[(28 + i) * N + p] / sqrtg;
    S[i] = U[(25 + i) * N + p] / sqrtg;
  }
  for (i = 0; i < 3; ++i) {
    vd[i] = 0.0;
    Bd[i] = 0.0;
    for (j = 0; j < 3; ++j) {
      vd[i] += gdn[i][j] * v[j];
      Bd[i] += gdn[i][j] * B[j];
    }
  }
  for (i = 0; i < 3; ++i) {
    B2 += B[i] * Bd[i];
    Bv += B[i] * vd[i];
  }
  W = P[6 * N + p];
  pr = P[2 * N + p];
  *E = (U[24 * N + p] + U[22 * N + p]) / sqrtg;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j)
      Sij[i][j] = 0.5 * (vd[i] * S[j] + vd[j] * S[i]) + gdn[i][j] * pr
                  - 0.5 / (W * W) * (2.0 * Bd[i] * Bd[j] - gdn[i][j] * B2)
                  - 0.5 * Bv * (Bd[i] * vd[j] + Bd[j] * vd[i] - gdn[i][j] * Bv);
}

void orc_ccz4_point(const orc_par* par, const double* U, const double* P, int64_t N,
                    int64_t p, const int64_t st[3], const double h[3], double out[22]) {
  const double PI = 3.14159265358979323846;
  double gt[3][3], At[3][3], chi, Kh, Th, Gh[3], alp, beta[3];
  double dgt[3][3][3], dchi[3], dKh[3], dTh[3], dGh[3][3], dalp[3], dbeta[3][3];
  double ddgt[3][3][3][3], ddchi[3][3], ddalp[3][3], ddbeta[3][3][3];
  double adv[22];
  double det, gtu[3][3], c1[3][3][3], c2[3][3][3], Gt[3], Z[3];
  double Atu[3][3], Amix[3][3], trA, AA;
  double Rh[3][3], Rchi[3][3], Rs[3][3], Rtr;
  double Gphys[3][3][3], DDa[3][3], lapA;
  double gdn[3][3], gup[3][3], sqrtg;
  double E = 0.0, Sm[3] = {0, 0, 0}, Sij[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, Str = 0.0;
  double divb, Kfull, falpha;
  int i, j, k, l, m, n, f;

  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      gt[i][j] = fld(U, S6[i][j], N, p);
      At[i][j] = fld(U, 6 + S6[i][j], N, p);
    }
  chi = fld(U, 12, N, p);
  Kh = fld(U, 13, N, p);
  Th = fld(U, 14, N, p);
  for (i = 0; i < 3; ++i) {
    Gh[i] = fld(U, 15 + i, N, p);
    beta[i] = fld(U, 19 + i, N, p);
  }
  alp = fld(U, 18, N, p);

  /* centred first and second derivatives */
  for (k = 0; k < 3; ++k) {
    for (i = 0; i < 3; ++i)
      for (j = 0; j < 3; ++j) dgt[k][i][j] = orc_d1(U + S6[i][j] * N, p, st[k], h[k]);
    dchi[k] = orc_d1(U + 12 * N, p, st[k], h[k]);
    dKh[k] = orc_d1(U + 13 * N, p, st[k], h[k]);
    dTh[k] = orc_d1(U + 14 * N, p, st[k], h[k]);
    for (i = 0; i < 3; ++i) dGh[k][i] = orc_d1(U + (15 + i) * N, p, st[k], h[k]);
    dalp[k] = orc_d1(U + 18 * N, p, st[k], h[k]);
    for (i = 0; i < 3; ++i) dbeta[k][i] = orc_d1(U + (19 + i) * N, p, st[k], h[k]);
  }
  for (k = 0; k < 3; ++k)
    for (l = 0; l < 3; ++l) {
      for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) ddgt[k][l][i][j] = dd(U + S6[i][j] * N, p, st, h, k, l);
      ddchi[k][l] = dd(U + 12 * N, p, st, h, k, l);
      ddalp[k][l] = dd(U + 18 * N, p, st, h, k, l);
      for (i = 0; i < 3; ++i) ddbeta[k][l][i] = dd(U + (19 + i) * N, p, st, h, k, l);
    }
  /* advection terms beta^k d_k u with the one-sided operator */
  for (f = 0; f < 22; ++f) {
    adv[f] = 0.0;
    for (k = 0; k < 3; ++k) adv[f] += beta[k] * orc_dup(U + f * N, p, st[k], h[k], beta[k]);
  }

  /* conformal metric inverse and Christoffels */
  det = gt[0][0] * (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1])
        - gt[0][1] * (gt[1][0] * gt[2][2] - gt[1][2] * gt[2][0])
        + gt[0][2] * (gt[1][0] * gt[2][1] - gt[1][1] * gt[2][0]);
  gtu[0][0] = (gt[1][1] * gt[2][2] - gt[1][2] * gt[2][1]) / det;
  gtu[0][1] = (gt[0][2] * gt[2][1] - gt[0][1] * gt[2][2]) / det;
  gtu[0][2] = (gt[0][1] * gt[1][2] - gt[0][2] * gt[1][1]) / det;
  gtu[1][1] = (gt[0][0] * gt[2][2] - gt[0][2] * gt[2][0]) / det;
  gtu[1][2] = (gt[0][2] * gt[1][0] - gt[0][0] * gt[1][2]) / det;
  gtu[2][2] = (gt[0][0] * gt[1][1] - gt[0][1] * gt[1][0]) / det;
  gtu[1][0] = gtu[0][1];
  gtu[2][0] = gtu[0][2];
  gtu[2][1] = gtu[1][2];

  for (k = 0; k < 3; ++k)
    for (i = 0; i < 3; ++i)
      for (j = 0; j < 3; ++j)
        c1[k][i][j] = 0.5 * (dgt[j][k][i] + dgt[i][k][j] - dgt[k][i][j]);
  for (k = 0; k < 3; ++k)
    for (i = 0; i < 3; ++i)
      for (j = 0; j < 3; ++j) {
        c2[k][i][j] = 0.0;
        for (l = 0; l < 3; ++l) c2[k][i][j] += gtu[k][l] * c1[l][i][j];
      }
  for (i = 0; i < 3; ++i) {
    Gt[i] = 0.0;
    for (j = 0; j < 3; ++j)
      for (k = 0; k < 3; ++k)
        for (l = 0; l < 3; ++l) Gt[i] += gtu[i][j] * gtu[k][l] * dgt[l][j][k];
    Z[i] = 0.5 * chi * (Gh[i] - Gt[i]);
  }

  /* physical metric */
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      gdn[i][j] = gt[i][j] / chi;
      gup[i][j] = chi * gtu[i][j];
    }
  sqrtg = sqrt(det / (chi * chi * chi));

  /* At with raised indices, trace and square */
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      Amix[i][j] = 0.0;
      for (k = 0; k < 3; ++k) Amix[i][j] += gtu[i][k] * At[k][j];
    }
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      Atu[i][j] = 0.0;
      for (k = 0; k < 3; ++k) Atu[i][j] += Amix[i][k] * gtu[k][j];
    }
  trA = 0.0;
  AA = 0.0;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      trA += gtu[i][j] * At[i][j];
      AA += At[i][j] * Atu[i][j];
    }

  /* Rhat_ij */
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      double r = 0.0;
      for (m = 0; m < 3; ++m)
        for (n = 0; n < 3; ++n) r += -0.5 * gtu[m][n] * ddgt[m][n][i][j];
      for (k = 0; k < 3; ++k) r += 0.5 * (gt[k][i] * dGh[j][k] + gt[k][j] * dGh[i][k]);
      for (k = 0; k < 3; ++k) r += Gh[k] * 0.5 * (c1[i][j][k] + c1[j][i][k]);
      for (m = 0; m < 3; ++m)
        for (n = 0; n < 3; ++n)
          for (k = 0; k < 3; ++k)
            r += gtu[m][n] * (c2[k][m][i] * c1[j][k][n] + c2[k][m][j] * c1[i][k][n]
                              + c2[k][m][i] * c1[k][n][j]);
      Rh[i][j] = r;
    }
  /* Rhat^chi_ij (the printed expression is chi * Rhat^chi_ij) */
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      double r = 0.5 * ddchi[i][j] - 0.25 / chi * dchi[i] * dchi[j];
      double tr = 0.0;
      for (k = 0; k < 3; ++k) {
        r += -0.5 * c2[k][i][j] * dchi[k];
        r += 1.0 / chi * Z[k] * (gt[k][i] * dchi[j] + gt[k][j] * dchi[i]);
      }
      for (k = 0; k < 3; ++k) {
        for (m = 0; m < 3; ++m) tr += gtu[k][m] * (ddchi[k][m] - 1.5 / chi * dchi[k] * dchi[m]);
        tr -= Gh[k] * dchi[k];
      }
      r += 0.5 * gt[i][j] * tr;
      Rchi[i][j] = r / chi;
    }
  Rtr = 0.0;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      Rs[i][j] = Rh[i][j] + Rchi[i][j];
      Rtr += gup[i][j] * Rs[i][j];
    }

  /* physical Christoffels and D_i D_j alpha; Laplacian as printed */
  for (k = 0; k < 3; ++k)
    for (i = 0; i < 3; ++i)
      for (j = 0; j < 3; ++j) {
        double t = (k == i ? dchi[j] : 0.0) + (k == j ? dchi[i] : 0.0);
        for (l = 0; l < 3; ++l) t -= gt[i][j] * gtu[k][l] * dchi[l];
        Gphys[k][i][j] = c2[k][i][j] - 0.5 / chi * t;
      }
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      DDa[i][j] = ddalp[i][j];
      for (k = 0; k < 3; ++k) DDa[i][j] -= Gphys[k][i][j] * dalp[k];
    }
  lapA = 0.0;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j)
      lapA += chi * gtu[i][j] * ddalp[i][j] - 0.5 * gtu[i][j] * dalp[i] * dchi[j];
  for (k = 0; k < 3; ++k) lapA -= chi * Gt[k] * dalp[k];

  /* matter */
  if (par->couple_matter) {
    orc_matter_point(U, P, N, p, gdn, sqrtg, &E, Sm, Sij);
    if (par->evolve_m1) orc_m1_matter(U, P, N, p, &E, Sm, Sij);
    for (i = 0; i < 3; ++i)
      for (j = 0; j < 3; ++j) Str += gup[i][j] * Sij[i][j];
  }

  divb = dbeta[0][0] + dbeta[1][1] + dbeta[2][2];
  Kfull = Kh + 2.0 * Th;

  /* d_t gt_ij */
  for (i = 0; i < 3; ++i)
    for (j = i; j < 3; ++j) {
      double r = adv[S6[i][j]];
      for (k = 0; k < 3; ++k) r += gt[i][k] * dbeta[j][k] + gt[k][j] * dbeta[i][k];
      r += -2.0 / 3.0 * gt[i][j] * divb;
      r += -2.0 * alp * (At[i][j] - 1.0 / 3.0 * gt[i][j] * trA);
      r += -alp / 3.0 * par->kappa_c * gt[i][j] * log(det);
      out[S6[i][j]] = r;
    }
  /* d_t At_ij */
  {
    double X[3][3], trX = 0.0;
    for (i = 0; i < 3; ++i)
      for (j = 0; j < 3; ++j) X[i][j] = alp * (Rs[i][j] - 8.0 * PI * Sij[i][j]) - DDa[i][j];
    for (i = 0; i < 3; ++i)
      for (j = 0; j < 3; ++j) trX += gtu[i][j] * X[i][j];
    for (i = 0; i < 3; ++i)
      for (j = i; j < 3; ++j) {
        double r = adv[6 + S6[i][j]];
        double AikAkj = 0.0;
        for (k = 0; k < 3; ++k) r += At[i][k] * dbeta[j][k] + At[k][j] * dbeta[i][k];
        r += -2.0 / 3.0 * At[i][j] * divb;
        r += -alp / 3.0 * par->kappa_c * gt[i][j] * trA;
        r += chi * (X[i][j] - 1.0 / 3.0 * gt[i][j] * trX);
        for (k = 0; k < 3; ++k) AikAkj += At[i][k] * Amix[k][j];
        r += alp * (Kh * At[i][j] - 2.0 * AikAkj);
        out[6 + S6[i][j]] = r;
      }
  }
  /* d_t chi */
  out[12] = adv[12] + 2.0 / 3.0 * chi * (alp * Kfull - divb);
  /* d_t Khat */
  {
    double r = adv[13] - lapA;
    r += alp * (1.0 / 3.0 * Kfull * Kfull + AA + 4.0 * PI * (E + Str)
                + par->kappa_z * (1.0 - par->kappa_2) * Th);
    for (i = 0; i < 3; ++i) r += 2.0 * Z[i] * dalp[i];
    out[13] = r;
  }
  /* d_t Theta */
  {
    double r = adv[14];
    r += 0.5 * alp * (Rtr + 2.0 / 3.0 * Kh * Kh + 2.0 / 3.0 * Th * (Kh - 2.0 * Th) - AA);
    for (i = 0; i < 3; ++i) r -= Z[i] * dalp[i];
    r -= alp * (8.0 * PI * E + par->kappa_z * (2.0 + par->kappa_2) * Th);
    out[14] = r;
  }
  /* d_t Ghat^i */
  for (i = 0; i < 3; ++i) {
    double r = adv[15 + i], t1 = 0.0, t2 = 0.0;
    for (j = 0; j < 3; ++j) {
      r += -Gh[j] * dbeta[j][i];
      for (k = 0; k < 3; ++k) r += gtu[j][k] * ddbeta[j][k][i];
      for (k = 0; k < 3; ++k) r += 1.0 / 3.0 * gtu[i][j] * ddbeta[j][k][k];
      r += -2.0 * Atu[i][j] * dalp[j];
    }
    r += 2.0 / 3.0 * Gh[i] * divb;
    for (j = 0; j < 3; ++j) {
      for (k = 0; k < 3; ++k) t1 += c2[i][j][k] * Atu[j][k];
      t1 += -1.5 / chi * Atu[i][j] * dchi[j];
      t1 += -2.0 / 3.0 * gtu[i][j] * dKh[j];
      t1 += -8.0 * PI * gtu[i][j] * Sm[j];
    }
    r += 2.0 * alp * t1;
    for (j = 0; j < 3; ++j) t2 += -gtu[i][j] * (1.0 / 3.0 * dTh[j] + Th / alp * dalp[j]);
    t2 += -1.0 / chi * Z[i] * (par->kappa_z + 2.0 / 3.0 * Kfull);
    r += 2.0 * alp * t2;
    out[15 + i] = r;
  }
  /* gauge */
  falpha = (par->f_alpha_kind == 1) ? 0.5 * alp : 1.0;
  out[18] = adv[18] - 2.0 * alp * falpha * Kh;
  for (i = 0; i < 3; ++i)
    out[19 + i] = adv[19 + i] + 0.75 * par->f_beta * Gh[i] - par->eta * (beta[i] - par->beta0[i]);

  /* Kreiss-Oliger dissipation on all 22 fields */
  for (f = 0; f < 22; ++f)
    for (k = 0; k < 3; ++k) out[f] += orc_ko(U + f * N, p, st[k], h[k], par->sigma_ko);
}
