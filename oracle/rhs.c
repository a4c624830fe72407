/*
 * Oracle (test infrastructure only): full method-of-lines right-hand side
 * L(U) on one patch (Sec. 3, eq. d_t U = L(U)), Runge-Kutta stage update
 * (Table I, explicit RK4) and periodic ghost filling.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"

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

int64_t orc_imex_step(const orc_grid* g, const orc_par* par, const orc_eos* e, double* U, const double* aux,
                      double dt, int periodic) {
  const int ng = g->ng, nf = par->evolve_m1n ? 47 : 44, nr = nf - 32;
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = npts(g);
  double* Un = (double*)malloc(sizeof(double) * nf * N);
  double* Ui = (double*)malloc(sizeof(double) * nf * N);
  double* P = (double*)calloc(8 * N, sizeof(double));
  double* F[4];
  double* R[4];
  int64_t bad = 0;
  int st, f;
  memcpy(Un, U, sizeof(double) * nf * N);
  for (st = 0; st < 4; ++st) {
    F[st] = (double*)calloc(nf * N, sizeof(double));
    R[st] = (double*)calloc(nr * N, sizeof(double));
  }
  for (st = 0; st < 4; ++st) {
    memcpy(Ui, Un, sizeof(double) * nf * N);
    for (f = 0; f < nf; ++f) {
      int64_t k;
#pragma omp parallel for schedule(static)
      for (k = ng; k < Nz - ng; ++k)
        for (int64_t j = ng; j < Ny - ng; ++j)
          for (int64_t i = ng; i < Nx - ng; ++i) {
            const int64_t p = f * N + i + Nx * (j + Ny * k);
            double v = Un[p];
            int jj;
            for (jj = 0; jj < st; ++jj) v += dt * IM_AE[st][jj] * F[jj][p];
            if (f >= 32)
              for (jj = 0; jj < st; ++jj) v += dt * IM_AI[st][jj] * R[jj][(f - 32) * N + (p - f * N)];
            Ui[p] = v;
          }
    }
    if (periodic) orc_fill_periodic(g, Ui, nf);
    orc_con2prim(g, e, Ui, P, NULL, NULL);
    if (IM_AI[st][st] != 0.0) {
      bad += orc_m1_implicit(g, Ui, P, aux, IM_AI[st][st] * dt);
      if (par->evolve_m1n) orc_m1n_implicit(g, Ui, P, aux, IM_AI[st][st] * dt);
      if (periodic) orc_fill_periodic(g, Ui, nf);
    }
    orc_rhs_split(g, par, e, Ui, P, aux, F[st], R[st], NULL);
  }
  for (f = 0; f < nf; ++f) {
    int64_t k;
#pragma omp parallel for schedule(static)
    for (k = ng; k < Nz - ng; ++k)
      for (int64_t j = ng; j < Ny - ng; ++j)
        for (int64_t i = ng; i < Nx - ng; ++i) {
          const int64_t p = f * N + i + Nx * (j + Ny * k);
          double v = Un[p];
          for (st = 0; st < 4; ++st) v += dt * IM_BE[st] * F[st][p];
          if (f >= 32)
            for (st = 0; st < 4; ++st) v += dt * IM_BI[st] * R[st][(f - 32) * N + (p - f * N)];
          U[p] = v;
        }
  }
  if (periodic) orc_fill_periodic(g, U, nf);
  for (st = 0; st < 4; ++st) {
    free(F[st]);
    free(R[st]);
  }
  free(Un);
  free(Ui);
  free(P);
  return bad;
}
