/*
 * Oracle (test infrastructure only): the gradient sub-grid-scale (LES) term
 * of the induction equation, App. A, with the paper's default coefficients
 * (C_M = 8 for the magnetic field; the others 0).
 *
 * The flux of Bbar^i along k gains -alpha G_B^{ki},
 *   G_B^{ki} = -C_M xi sqrt(gamma) H_M^{ki},   xi = gamma^{1/3} Delta^2 / 24,
 *   H_M^{ki} = 2 B^[i H_v^k] + 4 grad B^[i . grad v^k]
 *            = B^i H_v^k - B^k H_v^i + 2 (grad B^i . grad v^k - grad B^k . grad v^i),
 * so the right-hand side of Bbar^i gains d_k (alpha G_B^{ki}).
 *
 * H_v is the velocity part of the second-order response of the primitive
 * recovery that the gradient model expands: filtering the conserved fields
 * C(P) gives C + xi lap C, and lap C = C_P lap P + C_PP(grad P, grad P), so the
 * primitives recovered from the filtered conserved fields differ from the
 * filtered primitives by xi dP with C_P dP = C_PP(grad P, grad P):
 *   H_P = -(C_P)^{-1} C_PP(grad P, grad P),
 * C = (D, S_i, tau) of Sec. 2.2 as functions of P = (rho, eps, v^i) at the
 * point's metric, with B^i (itself conserved) entering C_PP through its
 * gradients.  C_PP(grad P, grad P) = gamma^{jl} C_PP(d_j P, d_l P) is taken as
 * a sum of second directional derivatives along the columns of the Cholesky
 * factor of gamma^{jl}, each by second-order Taylor arithmetic; C_P by
 * first-order Taylor arithmetic; the 5x5 system by Gaussian elimination with
 * partial pivoting.  (App. A prints H_v in closed form through Psi_v, H_Theta
 * and H_p; as read, that form misses this leading-order term on smooth
 * magnetised fields by a few per cent, e.g. in its rho-gradient times
 * v-gradient terms, so the definition itself is evaluated.)
 *
 * Readings: grad a . grad b = gamma^{jl} d_j a d_l b with the physical metric;
 * Delta^2 = (dx dy dz)^{2/3}; the metric is taken as locally constant in the
 * expansion (only the fluid fields are filtered); first derivatives of the
 * primitives (rho, eps, v^i from P, B^i = Bbar^i/sqrt(gamma)) by the 4th-order
 * centred operator, so alpha G_B is formed at the interior points and one
 * point beyond, and its divergence by the 2nd-order centred operator (three
 * ghost points suffice).
 */
#include <math.h>
#include <stdlib.h>
#include "orc.h"

/* second-order Taylor numbers a0 + a1 t + a2 t^2 */
typedef struct {
  double a0, a1, a2;
} jet;

static jet jc(double c) { jet r = {c, 0.0, 0.0}; return r; }
static jet jadd(jet a, jet b) { jet r = {a.a0 + b.a0, a.a1 + b.a1, a.a2 + b.a2}; return r; }
static jet jsub(jet a, jet b) { jet r = {a.a0 - b.a0, a.a1 - b.a1, a.a2 - b.a2}; return r; }
static jet jmul(jet a, jet b) {
  jet r = {a.a0 * b.a0, a.a0 * b.a1 + a.a1 * b.a0, a.a0 * b.a2 + a.a1 * b.a1 + a.a2 * b.a0};
  return r;
}
static jet jscale(double s, jet a) { jet r = {s * a.a0, s * a.a1, s * a.a2}; return r; }
static jet jdiv(jet a, jet b) {
  jet r;
  r.a0 = a.a0 / b.a0;
  r.a1 = (a.a1 - r.a0 * b.a1) / b.a0;
  r.a2 = (a.a2 - r.a0 * b.a2 - r.a1 * b.a1) / b.a0;
  return r;
}
static jet jsqrt(jet a) {
  jet r;
  r.a0 = sqrt(a.a0);
  r.a1 = a.a1 / (2.0 * r.a0);
  r.a2 = (a.a2 - r.a1 * r.a1) / (2.0 * r.a0);
  return r;
}
/* a^e for a0 > 0 */
static jet jpow(jet a, double e) {
  jet r;
  const double p = pow(a.a0, e);
  r.a0 = p;
  r.a1 = e * p / a.a0 * a.a1;
  r.a2 = e * p / a.a0 * a.a2 + 0.5 * e * (e - 1.0) * p / (a.a0 * a.a0) * a.a1 * a.a1;
  return r;
}

/* pressure of the hybrid EoS, p = K_i rho^G_i + (G_th - 1) rho (eps - eps_cold(rho)),
 * with the piece chosen by rho's value */
static jet eos_p(const orc_eos* e, jet rho, jet eps) {
  int i = 0, b;
  jet pc, ec;
  for (b = 0; b < e->npieces - 1; ++b)
    if (rho.a0 >= e->rho_b[b]) i = b + 1;
  if (e->K[i] == 0.0) {
    pc = jc(0.0);
    ec = jc(e->a[i]);
  } else {
    pc = jscale(e->K[i], jpow(rho, e->Gamma[i]));
    ec = jadd(jc(e->a[i]), jscale(e->K[i] / (e->Gamma[i] - 1.0), jpow(rho, e->Gamma[i] - 1.0)));
  }
  return jadd(pc, jscale(e->Gamma_th - 1.0, jmul(rho, jsub(eps, ec))));
}

/* undensitized D, S_i, tau of Sec. 2.2 at the metric gdn */
static void cons_jet(const orc_eos* e, const double gdn[3][3], jet rho, jet eps, const jet v[3], const jet B[3],
                     jet C[5]) {
  jet vd[3], Bd[3], v2 = jc(0.0), B2 = jc(0.0), vB = jc(0.0), W, W2, hW2, p;
  int i, j;
  for (i = 0; i < 3; ++i) {
    vd[i] = jc(0.0);
    Bd[i] = jc(0.0);
    for (j = 0; j < 3; ++j) {
      vd[i] = jadd(vd[i], jscale(gdn[i][j], v[j]));
      Bd[i] = jadd(Bd[i], jscale(gdn[i][j], B[j]));
    }
  }
  for (i = 0; i < 3; ++i) {
    v2 = jadd(v2, jmul(v[i], vd[i]));
    B2 = jadd(B2, jmul(B[i], Bd[i]));
    vB = jadd(vB, jmul(B[i], vd[i]));
  }
  W = jdiv(jc(1.0), jsqrt(jsub(jc(1.0), v2)));
  W2 = jmul(W, W);
  p = eos_p(e, rho, eps);
  hW2 = jmul(jadd(jmul(rho, jadd(jc(1.0), eps)), p), W2);
  C[0] = jmul(rho, W);
  for (i = 0; i < 3; ++i) C[1 + i] = jsub(jmul(jadd(hW2, B2), vd[i]), jmul(vB, Bd[i]));
  C[4] = jsub(jsub(jadd(jsub(hW2, p), B2), jscale(0.5, jadd(jmul(vB, vB), jdiv(B2, W2)))), C[0]);
}

static int solve5(double A[5][5], double b[5], double x[5]) {
  int i, j, k;
  for (k = 0; k < 5; ++k) {
    int piv = k;
    for (i = k + 1; i < 5; ++i)
      if (fabs(A[i][k]) > fabs(A[piv][k])) piv = i;
    if (A[piv][k] == 0.0) return 0;
    if (piv != k) {
      double t;
      for (j = 0; j < 5; ++j) {
        t = A[k][j];
        A[k][j] = A[piv][j];
        A[piv][j] = t;
      }
      t = b[k];
      b[k] = b[piv];
      b[piv] = t;
    }
    for (i = k + 1; i < 5; ++i) {
      const double f = A[i][k] / A[k][k];
      for (j = k; j < 5; ++j) A[i][j] -= f * A[k][j];
      b[i] -= f * b[k];
    }
  }
  for (i = 4; i >= 0; --i) {
    double t = b[i];
    for (j = i + 1; j < 5; ++j) t -= A[i][j] * x[j];
    x[i] = t / A[i][i];
  }
  return 1;
}

static const int S6l[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

typedef struct {
  double gdn[3][3], gup[3][3], sqrtg, det;
} lmetric;

static void lmetric_at(const double* U, int64_t N, int64_t p, lmetric* m) {
  double g[3][3], gi[3][3], det, chi = U[12 * N + p];
  int i, j;
  for (i = 0; i < 3; ++i)
    for (j = 0; j < 3; ++j) g[i][j] = U[S6l[i][j] * N + p];
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
      m->gdn[i][j] = g[i][j] / chi;
      m->gup[i][j] = chi * gi[i][j];
    }
  m->det = det / (chi * chi * chi);
  m->sqrtg = sqrt(m->det);
}

/* 4th-order centred first derivative of field f at p along stride st, spacing h */
static double d1(const double* f, int64_t p, int64_t st, double h) {
  return (8.0 * (f[p + st] - f[p - st]) - (f[p + 2 * st] - f[p - 2 * st])) / (12.0 * h);
}

/* H_v^k and H_M^{ki} (k < i: xy, xz, yz) at padded point p from the primitives
 * P (rho, eps, v^i) and B^i = Bbar^i/sqrt(gamma); needs two points around p */
static void les_point(const orc_grid* g, const orc_eos* e, const double* U, const double* P, int64_t N, int64_t p,
                      const int64_t st[3], const lmetric* m, double Hv[3], double HM[3]) {
  double Pv[8], dP[3][8], L[3][3], gd[3][8];
  int a, b, c, d, i, k;
  /* the primitives at p and their coordinate derivatives */
  for (a = 0; a < 8; ++a) {
    for (d = 0; d < 3; ++d) dP[d][a] = 0.0;
  }
  Pv[0] = P[p];
  Pv[1] = P[N + p];
  for (i = 0; i < 3; ++i) Pv[2 + i] = P[(3 + i) * N + p];
  for (i = 0; i < 3; ++i) Pv[5 + i] = U[(28 + i) * N + p] / m->sqrtg;
  for (d = 0; d < 3; ++d) {
    double tmp[5];
    int64_t q;
    for (a = 0; a < 2; ++a) dP[d][a] = d1(P + (int64_t)a * N, p, st[d], g->dx[d]);
    for (i = 0; i < 3; ++i) dP[d][2 + i] = d1(P + (int64_t)(3 + i) * N, p, st[d], g->dx[d]);
    /* B^i = Bbar^i / sqrt(gamma) at the five stencil points */
    for (i = 0; i < 3; ++i) {
      for (c = -2; c <= 2; ++c) {
        lmetric mq;
        q = p + c * st[d];
        lmetric_at(U, N, q, &mq);
        tmp[c + 2] = U[(28 + i) * N + q] / mq.sqrtg;
      }
      dP[d][5 + i] = (8.0 * (tmp[3] - tmp[1]) - (tmp[4] - tmp[0])) / (12.0 * g->dx[d]);
    }
  }
  /* Cholesky factor of gamma^{jl}: gamma^{jl} = sum_a L[j][a] L[l][a] */
  for (i = 0; i < 3; ++i)
    for (k = 0; k < 3; ++k) L[i][k] = 0.0;
  for (k = 0; k < 3; ++k) {
    double s = m->gup[k][k];
    for (a = 0; a < k; ++a) s -= L[k][a] * L[k][a];
    L[k][k] = sqrt(s);
    for (i = k + 1; i < 3; ++i) {
      double t = m->gup[i][k];
      for (a = 0; a < k; ++a) t -= L[i][a] * L[k][a];
      L[i][k] = t / L[k][k];
    }
  }
  /* derivatives along the factor's columns: gd[a][.] = sum_j L[j][a] d_j P */
  for (a = 0; a < 3; ++a)
    for (b = 0; b < 8; ++b) {
      gd[a][b] = 0.0;
      for (d = 0; d < 3; ++d) gd[a][b] += L[d][a] * dP[d][b];
    }
  {
    double rhs[5] = {0, 0, 0, 0, 0}, Jm[5][5], x[5];
    jet Cj[5], v[3], B[3];
    /* C_PP(grad P, grad P) = sum_a d^2/dt^2 C(P + t gd_a) */
    for (a = 0; a < 3; ++a) {
      jet rho = {Pv[0], gd[a][0], 0.0}, eps = {Pv[1], gd[a][1], 0.0};
      for (i = 0; i < 3; ++i) {
        v[i].a0 = Pv[2 + i], v[i].a1 = gd[a][2 + i], v[i].a2 = 0.0;
        B[i].a0 = Pv[5 + i], B[i].a1 = gd[a][5 + i], B[i].a2 = 0.0;
      }
      cons_jet(e, m->gdn, rho, eps, v, B, Cj);
      for (c = 0; c < 5; ++c) rhs[c] += 2.0 * Cj[c].a2;
    }
    /* C_P by unit first-order directions in (rho, eps, v^i), B held */
    for (b = 0; b < 5; ++b) {
      jet rho = {Pv[0], b == 0 ? 1.0 : 0.0, 0.0}, eps = {Pv[1], b == 1 ? 1.0 : 0.0, 0.0};
      for (i = 0; i < 3; ++i) {
        v[i].a0 = Pv[2 + i], v[i].a1 = (b == 2 + i) ? 1.0 : 0.0, v[i].a2 = 0.0;
        B[i] = jc(Pv[5 + i]);
      }
      cons_jet(e, m->gdn, rho, eps, v, B, Cj);
      for (c = 0; c < 5; ++c) Jm[c][b] = Cj[c].a1;
    }
    if (!solve5(Jm, rhs, x)) x[2] = x[3] = x[4] = 0.0;
    for (k = 0; k < 3; ++k) Hv[k] = -x[2 + k];
  }
  {
    /* grad B^i . grad v^k = sum_a gd_a(B^i) gd_a(v^k) */
    static const int KI[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (c = 0; c < 3; ++c) {
      const int kk = KI[c][0], ii = KI[c][1];
      double bv = 0.0, vb = 0.0;
      for (a = 0; a < 3; ++a) {
        bv += gd[a][5 + ii] * gd[a][2 + kk];
        vb += gd[a][5 + kk] * gd[a][2 + ii];
      }
      HM[c] = Pv[5 + ii] * Hv[kk] - Pv[5 + kk] * Hv[ii] + 2.0 * (bv - vb);
    }
  }
}

void orc_les_point_fields(const orc_grid* g, const orc_eos* e, const double* U, const double* P, double* out) {
  /* out: 6 fields (H_v^x, H_v^y, H_v^z, H_M^xy, H_M^xz, H_M^yz) at the points
   * two or more from the patch edge (others untouched) */
  const int64_t Nx = g->n[0] + 2 * g->ng, Ny = g->n[1] + 2 * g->ng, Nz = g->n[2] + 2 * g->ng;
  const int64_t N = Nx * Ny * Nz, st[3] = {1, Nx, Nx * Ny};
  int64_t k;
#pragma omp parallel for schedule(static)
  for (k = 2; k < Nz - 2; ++k)
    for (int64_t j = 2; j < Ny - 2; ++j)
      for (int64_t i = 2; i < Nx - 2; ++i) {
        const int64_t p = i + Nx * (j + Ny * k);
        lmetric m;
        double Hv[3], HM[3];
        int c;
        lmetric_at(U, N, p, &m);
        les_point(g, e, U, P, N, p, st, &m, Hv, HM);
        for (c = 0; c < 3; ++c) {
          out[c * N + p] = Hv[c];
          out[(3 + c) * N + p] = HM[c];
        }
      }
}

/* rhs of Bbar^i (fields 28..30) += d_k (alpha G_B^{ki}) at the interior points */
void orc_les_rhs(const orc_grid* g, const orc_par* par, const orc_eos* e, const double* U, const double* P,
                 double* rhs) {
  const int ng = g->ng;
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = Nx * Ny * Nz, st[3] = {1, Nx, Nx * Ny};
  const double D2 = pow(g->dx[0] * g->dx[1] * g->dx[2], 2.0 / 3.0);
  double* AG = (double*)calloc(3 * N, sizeof(double)); /* alpha G_B^{ki}: xy, xz, yz */
  int64_t k;
  if (par->les_cm == 0.0) {
    free(AG);
    return;
  }
#pragma omp parallel for schedule(static)
  for (k = ng - 1; k < Nz - ng + 1; ++k)
    for (int64_t j = ng - 1; j < Ny - ng + 1; ++j)
      for (int64_t i = ng - 1; i < Nx - ng + 1; ++i) {
        const int64_t p = i + Nx * (j + Ny * k);
        lmetric m;
        double Hv[3], HM[3], xi;
        int c;
        lmetric_at(U, N, p, &m);
        les_point(g, e, U, P, N, p, st, &m, Hv, HM);
        xi = cbrt(m.det) * D2 / 24.0;
        for (c = 0; c < 3; ++c) AG[c * N + p] = U[18 * N + p] * (-par->les_cm * xi * m.sqrtg * HM[c]);
      }
#pragma omp parallel for schedule(static)
  for (k = ng; k < Nz - ng; ++k)
    for (int64_t j = ng; j < Ny - ng; ++j)
      for (int64_t i = ng; i < Nx - ng; ++i) {
        const int64_t p = i + Nx * (j + Ny * k);
        /* antisymmetric G^{ki}: G^{xy} = AG0, G^{xz} = AG1, G^{yz} = AG2, G^{yx} = -AG0, ... */
        const double *gxy = AG, *gxz = AG + N, *gyz = AG + 2 * N;
        const double dx2 = 2.0 * g->dx[0], dy2 = 2.0 * g->dx[1], dz2 = 2.0 * g->dx[2];
        /* i = x: d_y G^{yx} + d_z G^{zx} = -d_y G^{xy} - d_z G^{xz} */
        rhs[28 * N + p] += -(gxy[p + st[1]] - gxy[p - st[1]]) / dy2 - (gxz[p + st[2]] - gxz[p - st[2]]) / dz2;
        /* i = y: d_x G^{xy} + d_z G^{zy} = d_x G^{xy} - d_z G^{yz} */
        rhs[29 * N + p] += (gxy[p + st[0]] - gxy[p - st[0]]) / dx2 - (gyz[p + st[2]] - gyz[p - st[2]]) / dz2;
        /* i = z: d_x G^{xz} + d_y G^{yz} */
        rhs[30 * N + p] += (gxz[p + st[0]] - gxz[p - st[0]]) / dx2 + (gyz[p + st[1]] - gyz[p - st[1]]) / dy2;
      }
  free(AG);
}
