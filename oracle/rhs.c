/*
 * Oracle (test infrastructure only): full method-of-lines right-hand side
 * L(U) on one patch (Sec. 3, eq. d_t U = L(U)), Runge-Kutta stage update
 * (Table I, explicit RK4) and periodic ghost filling.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"
#ifdef _OPENMP
#include <omp.h>
#endif

/* threads of the oracle's parallel loops (for timing it on a given core count) */
void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

void orc_ccz4_point(const orc_par* par, const double* U, const double* P, int64_t N,
                    int64_t p, const int64_t st[3], const double h[3], double out[22]);
void orc_grmhd_rhs(const orc_grid* g, const orc_par* par, const orc_eos* e, const double* U,
                   const double* P, double* rhs, double* max_speed);

static int64_t npts(const orc_grid* g) {
  return (int64_t)(g->n[0] + 2 * g->ng) * (g->n[1] + 2 * g->ng) * (g->n[2] + 2 * g->ng);
}

/* rhs is written at interior points only (fields 0..31); ghost entries untouched */
void orc_rhs(const orc_grid* g, const orc_par* par, const orc_eos* e, const double* U,
             const double* P, double* rhs, double* max_speed) {
  const int ng = g->ng;
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = npts(g);
  const int64_t st[3] = {1, Nx, Nx * Ny};
  const double h[3] = {g->dx[0], g->dx[1], g->dx[2]};
  int64_t k;
  ORC_PHASE(ORC_PH_CCZ4);
#pragma omp parallel for schedule(static)
  for (k = ng; k < Nz - ng; ++k)
    for (int64_t j = ng; j < Ny - ng; ++j)
      for (int64_t i = ng; i < Nx - ng; ++i) {
        int64_t p = i + Nx * (j + Ny * k);
        double out[22];
        int f;
        if (par->evolve_st) {
          orc_ccz4_point(par, U, P, N, p, st, h, out);
        } else {
          for (f = 0; f < 22; ++f) out[f] = 0.0;
        }
        for (f = 0; f < 22; ++f) rhs[f * N + p] = out[f];
      }
  ORC_PHASE(ORC_PH_OTHER);
  if (par->evolve_mhd) {
    orc_grmhd_rhs(g, par, e, U, P, rhs, max_speed);
    if (par->les_cm != 0.0) orc_les_rhs(g, par, e, U, P, rhs);
  } else {
#pragma omp parallel for schedule(static)
    for (k = ng; k < Nz - ng; ++k)
      for (int64_t j = ng; j < Ny - ng; ++j)
        for (int64_t i = ng; i < Nx - ng; ++i) {
          int64_t p = i + Nx * (j + Ny * k);
          int f;
          for (f = 22; f < 32; ++f) rhs[f * N + p] = 0.0;
        }
    if (max_speed) *max_speed = 0.0;
  }
}

void orc_rhs_full(const orc_grid* g, const orc_par* par, const orc_eos* e, const double* U, const double* P,
                  const double* aux, double* rhs, double* max_speed) {
  orc_rhs(g, par, e, U, P, rhs, max_speed);
  if (par->evolve_m1) orc_m1_rhs(g, par, U, P, aux, rhs, max_speed);
  if (par->evolve_m1 && par->evolve_m1n) orc_m1n_rhs(g, par, U, P, aux, rhs, NULL);
}

/* Explicit RK4 of Table I (c = 0, 1/2, 1/2, 1; b = 1/6, 1/3, 1/3, 1/6),
 * written with an accumulator:
 *   stage s: acc  = (s == 0 ? 0 : acc) + b_s k_s
 *            s < 3: Unext = Un + dt a_{s+1,s} k_s
 *            s = 3: Unext = Un + dt acc                               */
static const double RK4_A[3] = {0.5, 0.5, 1.0};
static const double RK4_B[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};

static void stage_point(int stage, double dt, int64_t p, const double* Un, const double* k,
                        double* acc, double* Unext) {
  double a = (stage == 0 ? 0.0 : acc[p]) + RK4_B[stage] * k[p];
  if (stage < 3) {
    acc[p] = a;
    Unext[p] = Un[p] + dt * RK4_A[stage] * k[p];
  } else {
    Unext[p] = Un[p] + dt * a;
  }
}

void orc_rk4_stage(int stage, double dt, int64_t n, const double* Un, const double* k,
                   double* acc, double* Unext) {
  int64_t p;
  ORC_PHASE(ORC_PH_RK);
  for (p = 0; p < n; ++p) stage_point(stage, dt, p, Un, k, acc, Unext);
  ORC_PHASE(ORC_PH_OTHER);
}

/* SSP-RK(3,3) of Shu and Osher (Sec. 3.1, explicit half of IMEX(3,3,2)) in
 * its Butcher form: with K[j] the right-hand sides of the earlier stages,
 * stage s = 0, 1 gives the next stage state Un + dt sum_{j<=s} a_{s+1,j} K[j],
 * s = 2 the step Un + dt sum_j b_j K[j], at the interior points. */
static const double SSP_A[3][3] = {{0.0, 0.0, 0.0}, {1.0, 0.0, 0.0}, {0.25, 0.25, 0.0}};
static const double SSP_B[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};

void orc_ssprk3_tableau(double A[9], double b[3]) {
  int i, j;
  for (i = 0; i < 3; ++i) {
    for (j = 0; j < 3; ++j) A[3 * i + j] = SSP_A[i][j];
    b[i] = SSP_B[i];
  }
}

void orc_ssprk3_combine(const orc_grid* g, int nfields, int stage, double dt, const double* Un,
                        const double* K0, const double* K1, const double* K2, double* Unext) {
  const int ng = g->ng;
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = npts(g);
  const double* K[3] = {K0, K1, K2};
  int f, j;
  for (f = 0; f < nfields; ++f)
    for (int64_t kk = ng; kk < Nz - ng; ++kk)
      for (int64_t jj = ng; jj < Ny - ng; ++jj)
        for (int64_t i = ng; i < Nx - ng; ++i) {
          const int64_t p = f * N + i + Nx * (jj + Ny * kk);
          double s = 0.0;
          for (j = 0; j <= stage; ++j) s += (stage < 2 ? SSP_A[stage + 1][j] : SSP_B[j]) * K[j][p];
          Unext[p] = Un[p] + dt * s;
        }
}

void orc_rk4_stage_interior(const orc_grid* g, int nfields, int stage, double dt,
                            const double* Un, const double* k, double* acc, double* Unext) {
  const int ng = g->ng;
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = npts(g);
  int f;
  ORC_PHASE(ORC_PH_RK);
  for (f = 0; f < nfields; ++f) {
    int64_t kk;
#pragma omp parallel for schedule(static)
    for (kk = ng; kk < Nz - ng; ++kk)
      for (int64_t j = ng; j < Ny - ng; ++j)
        for (int64_t i = ng; i < Nx - ng; ++i)
          stage_point(stage, dt, f * N + i + Nx * (j + Ny * kk), Un, k, acc, Unext);
  }
  ORC_PHASE(ORC_PH_OTHER);
}

/* periodic ghost fill: each ghost point takes the value of the interior point
 * an integer number of periods away (edges and corners included) */
void orc_fill_periodic(const orc_grid* g, double* U, int nfields) {
  const int ng = g->ng;
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = npts(g);
  int f;
  for (f = 0; f < nfields; ++f) {
    double* u = U + f * N;
    int64_t k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < Nz; ++k)
      for (int64_t j = 0; j < Ny; ++j)
        for (int64_t i = 0; i < Nx; ++i) {
          int64_t ii = ((i - ng) % g->n[0] + g->n[0]) % g->n[0] + ng;
          int64_t jj = ((j - ng) % g->n[1] + g->n[1]) % g->n[1] + ng;
          int64_t kk = ((k - ng) % g->n[2] + g->n[2]) % g->n[2] + ng;
          if (ii != i || jj != j || kk != k) u[i + Nx * (j + Ny * k)] = u[ii + Nx * (jj + Ny * kk)];
        }
  }
}

/* ---------------------------------------------------------------- IMEX(4,4,2)
 * Table I: explicit RK4 tableau (AE, BE) for the non-stiff part and the
 * implicit I42L tableau (AI, BI) for the stiff part, the collision terms of
 * the radiation.  Stage i: every field gets Un + dt sum_j AE[i][j] F_j, the
 * radiation fields also + dt sum_j AI[i][j] R_j (= V*); con2prim; if AI[i][i]
 * is not zero, the implicit solve V = V* + AI[i][i] dt R(V); then F_i, R_i at
 * the stage state.  Final: Un + dt sum_i (BE[i] F_i + BI[i] R_i) (radiation)
 * and Un + dt sum_i BE[i] F_i (all other fields).  Interior points only; ghost
 * values are frozen unless `periodic` is set. */
static const double IM_AE[4][4] = {{0, 0, 0, 0}, {0.5, 0, 0, 0}, {0, 0.5, 0, 0}, {0, 0, 1.0, 0}};
static const double IM_AI[4][4] = {{0, 0, 0, 0}, {0.25, 0.25, 0, 0}, {0, 1.0 / 6.0, 1.0 / 3.0, 0},
                                   {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0}};
static const double IM_BE[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
static const double IM_BI[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};

void orc_m1_rhs_split(const orc_grid* g, const orc_par* par, const double* U, const double* P,
                      const double* aux, double* rhs, double* stiff, double* max_speed);
int64_t orc_m1_implicit(const orc_grid* g, double* U, const double* P, const double* aux, double adt);

/* explicit part F (all 44 fields) and stiff part R (12 radiation fields) */
void orc_rhs_split(const orc_grid* g, const orc_par* par, const orc_eos* e, const double* U, const double* P,
                   const double* aux, double* F, double* R, double* max_speed) {
  orc_rhs(g, par, e, U, P, F, max_speed);
  orc_m1_rhs_split(g, par, U, P, aux, F, R, max_speed);
  if (par->evolve_m1n) orc_m1n_rhs(g, par, U, P, aux, F, R);
}

/* ---------------------------------------------------------------- IMEX(3,3,2)
 * Table II pairs the explicit SSP-RK(3,3) of Shu and Osher (c = (0, 1, 1/2),
 * A = ((0), (1), (1/4, 1/4)), b = (1/6, 1/6, 2/3)) with an L-stable implicit
 * I32L.  As printed, the implicit rows sum to (0, 1, 1) while its c column is
 * (0, 1, 1/2); with c the row sums (Sec. 3.1 defines c that way) the
 * printed tableau fails the second-order condition sum_i b_i c_i = 1/2
 * (it gives 5/6).  The tableau used here is re-derived from Sec. 3.1's
 * conditions keeping the printed structure: an explicit first stage (first
 * row 0), the printed c = (0, 1, 1/2) (equal to the explicit c, so every
 * coupling condition of order 2 holds with b equal to the explicit b) and the
 * printed b = (1/6, 1/6, 2/3).  Rows 2 and 3 then sum to 1 and 1/2, and
 * the stability function R(z) = 1 + z b^T (I - z A)^{-1} 1 is a cubic over
 * 6 (1 - a22 z)(1 - a33 z); L-stability (R bounded and R -> 0 as z -> -inf)
 * makes its z^3 and z^2 coefficients vanish:
 *   6 a22 a33 - 2 a22 + 4 a32 - a33 = 0,   (1 - a22)(1 - a33) = 1/2.
 * With equal diagonal entries a22 = a33 = gamma, gamma = 1 - 1/sqrt(2) (the
 * root in (0, 1)), a32 = 3 gamma (1 - 2 gamma)/4, a31 = 1/2 - gamma - a32,
 * a21 = 1 - gamma; then R(z) = (1 + (1 - 2 gamma) z)/(1 - gamma z)^2 and
 * |R(iy)|^2 <= 1 (A-stable).  (The printed second row (1/2, 1/2) admits no
 * L-stable completion: with a22 = 1/2 the second condition forces a33 = 0.) */
static void imex332_tableau(double AE[4][4], double AI[4][4], double BE[4], double BI[4]) {
  const double gam = 1.0 - sqrt(0.5);
  const double a32 = 3.0 * gam * (1.0 - 2.0 * gam) / 4.0;
  int i, j;
  for (i = 0; i < 4; ++i) {
    BE[i] = BI[i] = 0.0;
    for (j = 0; j < 4; ++j) AE[i][j] = AI[i][j] = 0.0;
  }
  AE[1][0] = 1.0;
  AE[2][0] = 0.25;
  AE[2][1] = 0.25;
  AI[1][0] = 1.0 - gam;
  AI[1][1] = gam;
  AI[2][0] = 0.5 - gam - a32;
  AI[2][1] = a32;
  AI[2][2] = gam;
  BE[0] = BI[0] = 1.0 / 6.0;
  BE[1] = BI[1] = 1.0 / 6.0;
  BE[2] = BI[2] = 2.0 / 3.0;
}

void orc_imex_tableau(int scheme, double AE[16], double AI[16], double BE[4], double BI[4], int* stages) {
  double ae[4][4], ai[4][4], be[4], bi[4];
  int i, j;
  if (scheme == 1) {
    imex332_tableau(ae, ai, be, bi);
    *stages = 3;
  } else {
    for (i = 0; i < 4; ++i) {
      be[i] = IM_BE[i];
      bi[i] = IM_BI[i];
      for (j = 0; j < 4; ++j) {
        ae[i][j] = IM_AE[i][j];
        ai[i][j] = IM_AI[i][j];
      }
    }
    *stages = 4;
  }
  for (i = 0; i < 4; ++i) {
    BE[i] = be[i];
    BI[i] = bi[i];
    for (j = 0; j < 4; ++j) {
      AE[4 * i + j] = ae[i][j];
      AI[4 * i + j] = ai[i][j];
    }
  }
}

/* one IMEX step of `scheme` (0: IMEX(4,4,2) of Table I, 1: IMEX(3,3,2) with
 * the re-derived I32L above) */
/* stiff fields of the split right-hand side: the radiation's 12 (15 with the
 * number densities), then with par->couple_exchange the fluid's share of the
 * exchange, tau and S_i (and DYe with the number densities) */
int orc_imex_stiff_fields(const orc_par* par) {
  const int nrad = par->evolve_m1n ? 15 : 12;
  return par->couple_exchange ? nrad + 4 + (par->evolve_m1n ? 1 : 0) : nrad;
}

/* stiff slot of evolved field f, or -1 */
static int stiff_slot(const orc_par* par, int f) {
  const int nrad = par->evolve_m1n ? 15 : 12;
  if (f >= 32) return f - 32;
  if (!par->couple_exchange) return -1;
  if (f >= 24 && f <= 27) return nrad + f - 24;
  if (f == 23 && par->evolve_m1n) return nrad + 4;
  return -1;
}

int64_t orc_imex_step_scheme(const orc_grid* g, const orc_par* par, const orc_eos* e, double* U, const double* aux,
                             double dt, int periodic, int scheme) {
  const int ng = g->ng, nf = par->evolve_m1n ? 47 : 44, nr = orc_imex_stiff_fields(par);
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = npts(g);
  double AE[16], AI[16], BE[4], BI[4];
  int ns;
  double* Un = (double*)malloc(sizeof(double) * nf * N);
  double* Ui = (double*)malloc(sizeof(double) * nf * N);
  double* P = (double*)calloc(8 * N, sizeof(double));
  double* F[4];
  double* R[4];
  int64_t bad = 0;
  int st, f;
  orc_imex_tableau(scheme, AE, AI, BE, BI, &ns);
  memcpy(Un, U, sizeof(double) * nf * N);
  for (st = 0; st < ns; ++st) {
    F[st] = (double*)calloc(nf * N, sizeof(double));
    R[st] = (double*)calloc(nr * N, sizeof(double));
  }
  for (st = 0; st < ns; ++st) {
    memcpy(Ui, Un, sizeof(double) * nf * N);
    for (f = 0; f < nf; ++f) {
      const int rs = stiff_slot(par, f);
      int64_t k;
#pragma omp parallel for schedule(static)
      for (k = ng; k < Nz - ng; ++k)
        for (int64_t j = ng; j < Ny - ng; ++j)
          for (int64_t i = ng; i < Nx - ng; ++i) {
            const int64_t p = f * N + i + Nx * (j + Ny * k);
            double v = Un[p];
            int jj;
            for (jj = 0; jj < st; ++jj) v += dt * AE[4 * st + jj] * F[jj][p];
            if (rs >= 0)
              for (jj = 0; jj < st; ++jj) v += dt * AI[4 * st + jj] * R[jj][rs * N + (p - f * N)];
            Ui[p] = v;
          }
    }
    if (periodic) orc_fill_periodic(g, Ui, nf);
    orc_con2prim(g, e, Ui, P, NULL, NULL);
    if (AI[4 * st + st] != 0.0) {
      bad += orc_m1_implicit_x(g, Ui, P, aux, AI[4 * st + st] * dt, par->couple_exchange);
      if (par->evolve_m1n)
        orc_m1n_implicit_x(g, Ui, P, aux, AI[4 * st + st] * dt, par->couple_exchange, par->m_b);
      if (periodic) orc_fill_periodic(g, Ui, nf);
    }
    orc_rhs_split(g, par, e, Ui, P, aux, F[st], R[st], NULL);
  }
  for (f = 0; f < nf; ++f) {
    const int rs = stiff_slot(par, f);
    int64_t k;
#pragma omp parallel for schedule(static) private(st)
    for (k = ng; k < Nz - ng; ++k)
      for (int64_t j = ng; j < Ny - ng; ++j)
        for (int64_t i = ng; i < Nx - ng; ++i) {
          const int64_t p = f * N + i + Nx * (j + Ny * k);
          double v = Un[p];
          for (st = 0; st < ns; ++st) v += dt * BE[st] * F[st][p];
          if (rs >= 0)
            for (st = 0; st < ns; ++st) v += dt * BI[st] * R[st][rs * N + (p - f * N)];
          U[p] = v;
        }
  }
  if (periodic) orc_fill_periodic(g, U, nf);
  for (st = 0; st < ns; ++st) {
    free(F[st]);
    free(R[st]);
  }
  free(Un);
  free(Ui);
  free(P);
  return bad;
}

int64_t orc_imex_step(const orc_grid* g, const orc_par* par, const orc_eos* e, double* U, const double* aux,
                      double dt, int periodic) {
  return orc_imex_step_scheme(g, par, e, U, aux, dt, periodic, 0);
}
