/*
 * Plain FP64 oracle of the mesh-refinement glue (Sec. 4.2 prolongation and
 * restriction; Sec. 3.1 dense output of RK4 for sub-cycling in time).
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h): it checks the HIP library and is no
 * code path of it.
 *
 * Index convention shared by prolongation and restriction (2:1 vertex-centred
 * refinement): fine padded index I and coarse padded index i coincide when
 * I = 2 i + off (per axis; off may be any integer).  A fine point with I - off
 * odd lies half-way between coarse points i = (I - off - 1)/2 and i + 1.
 */
#include <math.h>
#include <stdint.h>

#include "orc.h"

static int64_t npts_of(const orc_grid* g) {
  return (int64_t)(g->n[0] + 2 * g->ng) * (g->n[1] + 2 * g->ng) * (g->n[2] + 2 * g->ng);
}

/* floor division (negative numerators round down) */
static int64_t fdiv2(int64_t t) { return t >= 0 ? t / 2 : -((-t + 1) / 2); }

/* Lagrange basis at x = 1/2 for the nodes x_m = m - 2, m = 0..5 (three on each
 * side): l_j(x) = prod_{m != j} (x - x_m) / (x_j - x_m), written out as the
 * definition (Sec. 4.2) */
void orc_lagrange_half(double w[6]) {
  int j, m;
  for (j = 0; j < 6; ++j) {
    double num = 1.0, den = 1.0;
    for (m = 0; m < 6; ++m) {
      if (m == j) continue;
      num *= 0.5 - (double)(m - 2);
      den *= (double)(j - 2) - (double)(m - 2);
    }
    w[j] = num / den;
  }
}

/* value of field array A (strides of grid g) at coarse padded (i, j, k) */
static double at(const orc_grid* g, const double* A, int64_t i, int64_t j, int64_t k) {
  const int64_t Nx = g->n[0] + 2 * g->ng, Ny = g->n[1] + 2 * g->ng;
  return A[i + Nx * (j + Ny * k)];
}

/* interpolation along one axis at half-index t (fine units relative to the
 * coarse origin): coincident points copy, half points take the six-point sum */
static void nodes_of(int64_t t, int64_t* first, int* count) {
  if (t % 2 == 0) {
    *first = fdiv2(t);
    *count = 1;
  } else {
    *first = fdiv2(t - 1) - 2;
    *count = 6;
  }
}

/* Fill the fine padded index box [lo, hi) of every field of Uf from Uc by the
 * tensor product of the one-dimensional interpolation: along x first, then y,
 * then z.  Returns 0, or -1 if a needed coarse point lies outside Uc. */
int orc_prolong(const orc_grid* gc, const double* Uc, const orc_grid* gf, double* Uf, int nfields,
                const int off[3], const int lo[3], const int hi[3]) {
  const int64_t Ncx = gc->n[0] + 2 * gc->ng, Ncy = gc->n[1] + 2 * gc->ng, Ncz = gc->n[2] + 2 * gc->ng;
  const int64_t Nfx = gf->n[0] + 2 * gf->ng, Nfy = gf->n[1] + 2 * gf->ng;
  const int64_t Nc = npts_of(gc), Nf = npts_of(gf);
  double w[6];
  int f;
  int64_t I, J, K;
  orc_lagrange_half(w);
  for (K = lo[2]; K < hi[2]; ++K)
    for (J = lo[1]; J < hi[1]; ++J)
      for (I = lo[0]; I < hi[0]; ++I) {
        int64_t fx, fy, fz;
        int nx, ny, nz, a, b, c;
        nodes_of(I - off[0], &fx, &nx);
        nodes_of(J - off[1], &fy, &ny);
        nodes_of(K - off[2], &fz, &nz);
        if (fx < 0 || fy < 0 || fz < 0 || fx + nx > Ncx || fy + ny > Ncy || fz + nz > Ncz) return -1;
        for (f = 0; f < nfields; ++f) {
          const double* A = Uc + (int64_t)f * Nc;
          double vz[6];
          for (c = 0; c < nz; ++c) {
            double vy[6];
            for (b = 0; b < ny; ++b) {
              double s = 0.0;
              if (nx == 1) {
                s = at(gc, A, fx, fy + b, fz + c);
              } else {
                for (a = 0; a < 6; ++a) s += w[a] * at(gc, A, fx + a, fy + b, fz + c);
              }
              vy[b] = s;
            }
            if (ny == 1) {
              vz[c] = vy[0];
            } else {
              double s = 0.0;
              for (b = 0; b < 6; ++b) s += w[b] * vy[b];
              vz[c] = s;
            }
          }
          {
            double s = 0.0;
            if (nz == 1) {
              s = vz[0];
            } else {
              for (c = 0; c < 6; ++c) s += w[c] * vz[c];
            }
            Uf[(int64_t)f * Nf + I + Nfx * (J + Nfy * K)] = s;
          }
        }
      }
  return 0;
}

/* Restriction by direct copy (Sec. 4.2): coarse padded box [lo, hi) of every
 * field takes the coincident fine values, Uc(i) = Uf(2 i + off).  Returns 0,
 * or -1 if a needed fine point lies outside Uf. */
int orc_restrict(const orc_grid* gf, const double* Uf, const orc_grid* gc, double* Uc, int nfields,
                 const int off[3], const int lo[3], const int hi[3]) {
  const int64_t Nfx = gf->n[0] + 2 * gf->ng, Nfy = gf->n[1] + 2 * gf->ng, Nfz = gf->n[2] + 2 * gf->ng;
  const int64_t Ncx = gc->n[0] + 2 * gc->ng, Ncy = gc->n[1] + 2 * gc->ng;
  const int64_t Nc = npts_of(gc), Nf = npts_of(gf);
  int f;
  int64_t i, j, k;
  for (k = lo[2]; k < hi[2]; ++k)
    for (j = lo[1]; j < hi[1]; ++j)
      for (i = lo[0]; i < hi[0]; ++i) {
        const int64_t I = 2 * i + off[0], J = 2 * j + off[1], K = 2 * k + off[2];
        if (I < 0 || J < 0 || K < 0 || I >= Nfx || J >= Nfy || K >= Nfz) return -1;
        for (f = 0; f < nfields; ++f) Uc[(int64_t)f * Nc + i + Ncx * (j + Ncy * k)] = Uf[(int64_t)f * Nf + I + Nfx * (J + Nfy * K)];
      }
  return 0;
}

/* Dense output of RK4 (Sec. 3.1): the weights b_j(theta) of
 * U(t^n + theta dt) = U^n + sum_j b_j(theta) k_j, and their m-th derivatives
 * in theta (m = 0..3), written out from the polynomials. */
void orc_dense_weights(double theta, int m, double b[4]) {
  const double t = theta, t2 = t * t, t3 = t2 * t;
  if (m == 0) {
    b[0] = t - 1.5 * t2 + 2.0 / 3.0 * t3;
    b[1] = t2 - 2.0 / 3.0 * t3;
    b[2] = b[1];
    b[3] = -0.5 * t2 + 2.0 / 3.0 * t3;
  } else if (m == 1) {
    b[0] = 1.0 - 3.0 * t + 2.0 * t2;
    b[1] = 2.0 * t - 2.0 * t2;
    b[2] = b[1];
    b[3] = -t + 2.0 * t2;
  } else if (m == 2) {
    b[0] = -3.0 + 4.0 * t;
    b[1] = 2.0 - 4.0 * t;
    b[2] = b[1];
    b[3] = -1.0 + 4.0 * t;
  } else {
    b[0] = 4.0;
    b[1] = -4.0;
    b[2] = -4.0;
    b[3] = 4.0;
  }
}

/* At the interior points of nfields fields: with k_j = dt L_j (L_j the
 * right-hand side at stage j of the step), m = 0 gives U(t^n + theta dt) and
 * m >= 1 the m-th time derivative, (1/dt^m) sum_j k_j b_j^(m)(theta). */
void orc_dense_output(const orc_grid* g, int nfields, double theta, double dt, int m, const double* Un,
                      const double* L0, const double* L1, const double* L2, const double* L3, double* out) {
  const int ng = g->ng;
  const int64_t Nx = g->n[0] + 2 * ng, Ny = g->n[1] + 2 * ng, Nz = g->n[2] + 2 * ng;
  const int64_t N = npts_of(g);
  const double* L[4] = {L0, L1, L2, L3};
  double b[4];
  int f, j;
  orc_dense_weights(theta, m, b);
  for (f = 0; f < nfields; ++f)
    for (int64_t k = ng; k < Nz - ng; ++k)
      for (int64_t jj = ng; jj < Ny - ng; ++jj)
        for (int64_t i = ng; i < Nx - ng; ++i) {
          const int64_t p = f * N + i + Nx * (jj + Ny * k);
          double s = 0.0;
          for (j = 0; j < 4; ++j) s += b[j] * (dt * L[j][p]);
          out[p] = m == 0 ? Un[p] + s : s / pow(dt, (double)m);
        }
}
