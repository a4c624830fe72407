/*
 * Oracle (test infrastructure only): constraint monitors of the evolution
 * (Sec. 2.1 constraints Theta = 0, Z_i = 0 and the energy and momentum
 * constraints they integrate; Sec. 5 accuracy checks: L2 norms of the energy
 * and momentum constraint residuals, total baryonic mass as the integral of the
 * conserved density, the Z4 variables Theta and Z, and the cleaning field phi
 * against |B|).
 *
 * The paper names these monitors without writing out the residuals; this file
 * uses the textbook 3+1 constraints of the physical metric:
 *   H   = R + K^2 - K_ij K^ij - 16 pi E,
 *   M_i = D_j K^j_i - D_i K - 8 pi S_i,
 * with gamma_ij = gt_ij / chi, K_ij = (At_ij + gt_ij K / 3) / chi,
 * K = Khat + 2 Theta (the physical trace), E = (taubar + Dbar)/sqrt(gamma),
 * S_i = Sbar_i / sqrt(gamma); R_ij is the Ricci tensor of gamma_ij from its
 * definition through the Christoffel symbols,
 *   R_ij = d_k G^k_ij - d_j G^k_ik + G^k_kl G^l_ij - G^k_jl G^l_ik,
 * and d_m G^k_ij follows from the first and second derivatives of gamma_ij.
 * Every derivative of a product is taken by the product rule from the 4th-order
 * centred derivatives of the evolved fields (the same operators as the
 * right-hand side).  Z^i = chi (Ghat^i - Gt^i) / 2 with Gt^i from the metric
 * derivatives, as in the definition of Ghat^i.
 */
#include <math.h>
#include "orc.h"

static const int S6[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

static void inv3(const double a[3][3], double inv[3][3], double* det) {
  double d = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0])
             + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  inv[0][0] = (a[1][1] * a[2][2] - a[1][2] * a[2][1]) / d;
  inv[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) / d;
  inv[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) / d;
  inv[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) / d;
  inv[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) / d;
  inv[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) / d;
  inv[1][0] = inv[0][1];
  inv[2][0] = inv[0][2];
  inv[2][1] = inv[1][2];
  *det = d;
}

static double dd(const double* u, int64_t p, const int64_t st[3], const double h[3], int k, int l) {
  if (k == l) return orc_d2(u, p, st[k], h[k]);
  return orc_d11(u, p, st[k], st[l], h[k], h[l]);
}

/* H, M_i, Z_i Z^i at padded point p; also sqrt(gamma) and gamma_ij */
void orc_constraints_point(const double* U, int64_t N, int64_t p, const int64_t st[3], const double h[3],
                           double out[5], double* sqrtg_out, double gdn_out[3][3]) {
  const double PI = 3.14159265358979323846;
  double gt[3][3], dgt[3][3][3], ddgt[3][3][3][3], chi, dchi[3], ddchi[3][3];
  double At[3][3], dAt[3][3][3], Kt, dK[3];
  double g[3][3], dg[3][3][3], ddg[3][3][3][3], gu[3][3], det;
  double c1[3][3][3], c2[3][3][3], dc2[3][3][3][3], dgu[3][3][3];
  double R, Kdn[3][3], dKdn[3][3][3], Kup[3][3], KK, E, S[3], sqrtg;
  double gtu[3][3], dett, Gt[3], Zu[3], Z2;
  int i, j, k, l, m;

  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      gt[i][j] = U[S6[i][j] * N + p];
      At[i][j] = U[(6 + S6[i][j]) * N + p];
    }
  chi = U[12 * N + p];
  Kt = U[13 * N + p] + 2.0 * U[14 * N + p];
  for (k = 0; k < 3; ++k) {
    for (i = 0; i < 3; ++i)
      for (j = 0; j < 3; ++j) {
        dgt[k][i][j] = orc_d1(U + S6[i][j] * N, p, st[k], h[k]);
        dAt[k][i][j] = orc_d1(U + (6 + S6[i][j]) * N, p, st[k], h[k]);
      }
    dchi[k] = orc_d1(U + 12 * N, p, st[k], h[k]);
    dK[k] = orc_d1(U + 13 * N, p, st[k], h[k]) + 2.0 * orc_d1(U + 14 * N, p, st[k], h[k]);
  }
  for (k = 0; k < 3; ++k)
    for (l = 0; l < 3; ++l) {
      for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) ddgt[k][l][i][j] = dd(U + S6[i][j] * N, p, st, h, k, l);
      ddchi[k][l] = dd(U + 12 * N, p, st, h, k, l);
    }

  /* physical metric and its derivatives, gamma = gt / chi, by the quotient rule */
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      g[i][j] = gt[i][j] / chi;
      for (k = 0; k < 3; ++k) dg[k][i][j] = dgt[k][i][j] / chi - gt[i][j] * dchi[k] / (chi * chi);
      for (k = 0; k < 3; ++k)
        for (l = 0; l < 3; ++l)
          ddg[k][l][i][j] = ddgt[k][l][i][j] / chi - (dgt[k][i][j] * dchi[l] + dgt[l][i][j] * dchi[k]) / (chi * chi)
                            - gt[i][j] * ddchi[k][l] / (chi * chi)
                            + 2.0 * gt[i][j] * dchi[k] * dchi[l] / (chi * chi * chi);
    }
  inv3(g, gu, &det);
  sqrtg = sqrt(det);

  /* Christoffels: first kind c1[k][i][j] = G_kij, second kind c2[k][i][j] = G^k_ij */
  for (k = 0; k < 3; ++k)
    for (i = 0; i < 3; ++i)
      for (j = 0; j < 3; ++j) c1[k][i][j] = 0.5 * (dg[i][k][j] + dg[j][k][i] - dg[k][i][j]);
  for (k = 0; k < 3; ++k)
    for (i = 0; i < 3; ++i)
      for (j = 0; j < 3; ++j) {
        c2[k][i][j] = 0.0;
        for (l = 0; l < 3; ++l) c2[k][i][j] += gu[k][l] * c1[l][i][j];
      }
  /* d_m gamma^{kl} = -gamma^{ka} gamma^{lb} d_m gamma_ab */
  for (m = 0; m < 3; ++m)
    for (k = 0; k < 3; ++k)
      for (l = 0; l < 3; ++l) {
        double s = 0.0;
        for (i = 0; i < 3; ++i)
          for (j = 0; j < 3; ++j) s -= gu[k][i] * gu[l][j] * dg[m][i][j];
        dgu[m][k][l] = s;
      }
  /* d_m G^k_ij = d_m gamma^{kl} G_lij + gamma^{kl} d_m G_lij */
  for (m = 0; m < 3; ++m)
    for (k = 0; k < 3; ++k)
      for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) {
          double s = 0.0;
          for (l = 0; l < 3; ++l)
            s += dgu[m][k][l] * c1[l][i][j]
                 + gu[k][l] * 0.5 * (ddg[m][i][l][j] + ddg[m][j][l][i] - ddg[m][l][i][j]);
          dc2[m][k][i][j] = s;
        }
  /* Ricci tensor and scalar */
  R = 0.0;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      double r = 0.0;
      for (k = 0; k < 3; ++k) {
        r += dc2[k][k][i][j] - dc2[j][k][i][k];
        for (l = 0; l < 3; ++l) r += c2[k][k][l] * c2[l][i][j] - c2[k][j][l] * c2[l][i][k];
      }
      R += gu[i][j] * r;
    }

  /* extrinsic curvature K_ij = (At_ij + gt_ij K/3)/chi and its derivatives */
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      const double num = At[i][j] + gt[i][j] * Kt / 3.0;
      Kdn[i][j] = num / chi;
      for (k = 0; k < 3; ++k) {
        const double dnum = dAt[k][i][j] + dgt[k][i][j] * Kt / 3.0 + gt[i][j] * dK[k] / 3.0;
        dKdn[k][i][j] = dnum / chi - num * dchi[k] / (chi * chi);
      }
    }
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) {
      Kup[i][j] = 0.0;
      for (k = 0; k < 3; ++k)
        for (l = 0; l < 3; ++l) Kup[i][j] += gu[i][k] * gu[j][l] * Kdn[k][l];
    }
  KK = 0.0;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) KK += Kdn[i][j] * Kup[i][j];

  /* matter: E = (taubar + Dbar)/sqrt(gamma), S_i = Sbar_i/sqrt(gamma) */
  E = (U[24 * N + p] + U[22 * N + p]) / sqrtg;
  for (i = 0; i < 3; ++i) S[i] = U[(25 + i) * N + p] / sqrtg;

  out[0] = R + Kt * Kt - KK - 16.0 * PI * E;
  /* M_i = gamma^{jk} D_k K_ji - d_i K - 8 pi S_i,
   * D_k K_ji = d_k K_ji - G^l_kj K_li - G^l_ki K_jl */
  for (i = 0; i < 3; ++i) {
    double s = 0.0;
    for (j = 0; j < 3; ++j)
      for (k = 0; k < 3; ++k) {
        double DK = dKdn[k][j][i];
        for (l = 0; l < 3; ++l) DK -= c2[l][k][j] * Kdn[l][i] + c2[l][k][i] * Kdn[j][l];
        s += gu[j][k] * DK;
      }
    out[1 + i] = s - dK[i] - 8.0 * PI * S[i];
  }

  /* Z^i = chi (Ghat^i - Gt^i)/2, Gt^i = gt^{ij} gt^{kl} d_l gt_jk; Z_i Z^i with gamma_ij */
  inv3(gt, gtu, &dett);
  for (i = 0; i < 3; ++i) {
    Gt[i] = 0.0;
    for (j = 0; j < 3; ++j)
      for (k = 0; k < 3; ++k)
        for (l = 0; l < 3; ++l) Gt[i] += gtu[i][j] * gtu[k][l] * dgt[l][j][k];
    Zu[i] = 0.5 * chi * (U[(15 + i) * N + p] - Gt[i]);
  }
  Z2 = 0.0;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) Z2 += g[i][j] * Zu[i] * Zu[j];
  out[4] = Z2;
  *sqrtg_out = sqrtg;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) gdn_out[i][j] = g[i][j];
}

/* Over the interior: C (5 fields of the padded layout, interior points
 * written) = H, M_1, M_2, M_3, Z_i Z^i; sums (7 (nz + 1) doubles): for each
 * interior plane k, sums[7 + 7 k + q] = the plane's sum times the cell volume
 * of
 *   q = 0: H^2, 1: M_1^2 + M_2^2 + M_3^2, 2: Dbar (baryonic mass),
 *   3: Theta^2, 4: Z_i Z^i, 5: phi^2 = (phibar / sqrt(gamma))^2,
 *   6: gamma_ij B^i B^j with B^i = Bbar^i / sqrt(gamma),
 * and sums[q] the total over the planes in order. */
void orc_constraints(const orc_grid* g, const double* U, double* C, double* sums) {
  const int ng = g->ng, nx = g->n[0], ny = g->n[1], nz = g->n[2];
  const int64_t Nx = nx + 2 * ng, Ny = ny + 2 * ng, Nz = nz + 2 * ng, N = Nx * Ny * Nz;
  const int64_t st[3] = {1, Nx, Nx * Ny};
  const double h[3] = {g->dx[0], g->dx[1], g->dx[2]};
  const double dV = h[0] * h[1] * h[2];
  int i, j, k, q, a, b;
  for (q = 0; q < 7; ++q) sums[q] = 0.0;
  for (k = 0; k < nz; ++k) {
    double pl[7] = {0, 0, 0, 0, 0, 0, 0};
    for (j = 0; j < ny; ++j)
      for (i = 0; i < nx; ++i) {
        const int64_t p = (i + ng) + Nx * ((j + ng) + Ny * (int64_t)(k + ng));
        double o[5], sg, gd[3][3], B[3], B2 = 0.0, phi;
        orc_constraints_point(U, N, p, st, h, o, &sg, gd);
        for (q = 0; q < 5; ++q) C[q * N + p] = o[q];
        for (a = 0; a < 3; ++a) B[a] = U[(28 + a) * N + p] / sg;
        for (a = 0; a < 3; ++a)
          for (b = 0; b < 3; ++b) B2 += gd[a][b] * B[a] * B[b];
        phi = U[31 * N + p] / sg;
        pl[0] += o[0] * o[0] * dV;
        pl[1] += (o[1] * o[1] + o[2] * o[2] + o[3] * o[3]) * dV;
        pl[2] += U[22 * N + p] * dV;
        pl[3] += U[14 * N + p] * U[14 * N + p] * dV;
        pl[4] += o[4] * dV;
        pl[5] += phi * phi * dV;
        pl[6] += B2 * dV;
      }
    for (q = 0; q < 7; ++q) {
      sums[7 + 7 * k + q] = pl[q];
      sums[q] += pl[q];
    }
  }
}
