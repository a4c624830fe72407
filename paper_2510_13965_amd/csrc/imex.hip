// IMEX(4,4,2) of Table I for the radiation's stiff collision terms.
//
//   k_imex_combine  stage s = 0..3: Ustage = Un + dt sum_{j<s} AE[s][j] F_j on
//                   every field, + dt sum_{j<s} AI[s][j] R_j on the radiation
//                   fields (= V*); s = 4: Un + dt sum_i (BE[i] F_i + BI[i] R_i)
//   k_m1_implicit   per interior point and species, V = (E, F_i) solving
//                   V = V* + adt alpha (S_n, S_i)(V) (undensitized), fluid from
//                   the stage's primitives, the closure's Eddington factor
//                   frozen at its value for V*; Newton's method with the exact
//                   Jacobian (dual numbers), 4x4 elimination with partial
//                   pivoting, at most 60 iterations; converged at
//                   |dV| <= 1e-15 (E + |F|), or once an update no larger than
//                   1e-9 (E + |F|) is not below half of the previous one
//                   (Newton has stopped contracting: rounding floor); a solve
//                   that does not converge keeps the first Newton iterate
//                   (App. C's linearised implicit update about V*); with the
//                   number densities, each species' N then takes App. C's
//                   closed-form update N = (N* + adt alpha eta0) /
//                   (1 + adt alpha kappa0_a/Gamma), Gamma from the updated
//                   E, F_i and their closure
#include "c2p_dev.hpp"
#include "m1_dev.hpp"
#include "prof.hpp"

namespace mhd {

#pragma clang fp contract(off)

// Tableaux, [scheme][stage][j]: scheme 0 is Table I's IMEX(4,4,2) (explicit
// RK4 with I42L); scheme 1 is IMEX(3,3,2): Table II's explicit SSP-RK(3,3)
// with an L-stable I32L re-derived from Sec. 3.1's conditions (the printed one
// is first order: its rows sum to (0, 1, 1) against its c = (0, 1, 1/2)).
// The re-derived I32L keeps the printed explicit first stage, c and b and has
// equal diagonal entries gamma = 1 - 1/sqrt(2): rows (0, 0, 0),
// (1 - gamma, gamma, 0), (1/2 - gamma - a32, a32, gamma) with
// a32 = 3 gamma (1 - 2 gamma)/4 (the values below are those expressions
// evaluated in double).  In both schemes b is the same for the two halves.
__constant__ double kImAE[2][4][4] = {
    {{0, 0, 0, 0}, {0.5, 0, 0, 0}, {0, 0.5, 0, 0}, {0, 0, 1.0, 0}},
    {{0, 0, 0, 0}, {1.0, 0, 0, 0}, {0.25, 0.25, 0, 0}, {0, 0, 0, 0}}};
__constant__ double kImAI[2][4][4] = {
    {{0, 0, 0, 0}, {0.25, 0.25, 0, 0}, {0, 1.0 / 6.0, 1.0 / 3.0, 0}, {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0}},
    {{0, 0, 0, 0},
     {0.7071067811865476, 0.2928932188134524, 0, 0},
     {0.11611652351681563, 0.09099025766973194, 0.2928932188134524, 0},
     {0, 0, 0, 0}}};
__constant__ double kImB[2][4] = {{1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0, 0}};
__constant__ int kImStages[2] = {4, 3};

struct ImexArgs {
  Geom g;
  int scheme;  // 0: IMEX(4,4,2), 1: IMEX(3,3,2)
  int stage;
  double dt;
  const double* Un;
  const double* F[4];  // explicit parts of the earlier stages (44 or 47 fields)
  const double* R[4];  // stiff parts (12 or 15 fields; 16 or 20 with the coupled exchange)
  double* Uout;
  int nfields;
  int coupled;  // the fluid's share of the exchange is in R too
};

// block 64x4, grid z = nz * nfields (field-major)
// stiff slot of evolved field f (nfields 44 or 47), or -1: the radiation's
// fields (32 and up) in order, then with the coupled exchange the fluid's
// tau and S_i, and DYe with the number densities
__device__ __forceinline__ int stiff_slot(int f, int nfields, int coupled) {
  const int nrad = nfields - 32;
  if (f >= 32) return f - 32;
  if (!coupled) return -1;
  if (f >= 24 && f <= 27) return nrad + f - 24;
  if (f == 23 && nfields == MHD_NU_M1N) return nrad + 4;
  return -1;
}

// one element of stage `s` of the IMEX combination: field f (0..46) at point
// pt, with stiff slot rs (-1: the field has no stiff part)
__device__ __forceinline__ void imex_element(int sc, int s, double dt, const double* Un, const double* const* F,
                                             const double* const* R, double* Uout, int f, int64_t pt, int64_t sf,
                                             int rs) {
  const int64_t p = (int64_t)f * sf + pt;
  const int ns = kImStages[sc];
  double v = Un[p];
  if (s < ns) {
    for (int jj = 0; jj < s; ++jj) v += dt * kImAE[sc][s][jj] * F[jj][p];
    if (rs >= 0)
      for (int jj = 0; jj < s; ++jj) v += dt * kImAI[sc][s][jj] * R[jj][(int64_t)rs * sf + pt];
  } else {
    for (int st = 0; st < ns; ++st) v += dt * kImB[sc][st] * F[st][p];
    if (rs >= 0)
      for (int st = 0; st < ns; ++st) v += dt * kImB[sc][st] * R[st][(int64_t)rs * sf + pt];
  }
  Uout[p] = v;
}

__global__ void __launch_bounds__(256) k_imex_combine(ImexArgs a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int kz = blockIdx.z % g.nz;
  const int f = blockIdx.z / g.nz;
  if (i >= g.nx || j >= g.ny) return;
  imex_element(a.scheme, a.stage, a.dt, a.Un, a.F, a.R, a.Uout, f, g.at(i + g.ng, j + g.ng, kz + g.ng), g.sf,
               stiff_slot(f, a.nfields, a.coupled));
}

// every field of every interior point of a level's boxes; stage 4 writes U
__global__ void __launch_bounds__(256) k_imex_combine_lv(LevelArgs L) {
  for_each_level_point(L, kRegionInterior, [&](const BoxDev& B, int i, int j, int k, bool live) {
    if (!live) return;
    const int64_t pt = B.g.at(i + B.g.ng, j + B.g.ng, k + B.g.ng);
    double* out = L.stage < 4 ? B.Us : B.U;
    const double* const* F = B.F;
    const double* const* R = B.R;
#pragma unroll 4
    for (int f = 0; f < L.nfields; ++f)
      imex_element(0, L.stage, L.dt, B.U, F, R, out, f, pt, B.g.sf, stiff_slot(f, L.nfields, 0));
  });
}

template <class T>
__device__ __forceinline__ void implicit_G(const M1State& s0, const double gd[6], const double gu[6], double chi,
                                           const T V[4], const double Vs[4], double adt, double alp, double ka,
                                           double ks, double eta, T G[4]) {
  const double W = s0.W, W2 = W * W;
  const double dthick = 1.5 * (1.0 - chi), dthin = 1.0 - dthick;
  const T E = V[0];
  const T F[3] = {V[1], V[2], V[3]};
  T Fu[3], F2 = F[0] * 0.0, vF = F[0] * 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    Fu[r] = F[0] * 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) Fu[r] = Fu[r] + gu[sym(r, c)] * F[c];
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    F2 = F2 + Fu[r] * F[r];
    vF = vF + F[r] * s0.v[r];
  }
  const T Jth = 3.0 / (2.0 * W2 + 1.0) * ((2.0 * W2 - 1.0) * E - 2.0 * W2 * vF);
  T Hth[3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    Hth[r] = F[r] / W + W * s0.vd[r] / (2.0 * W2 + 1.0) * ((4.0 * W2 + 1.0) * vF - 4.0 * W2 * E);
  T P[6];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = r; c < 3; ++c) {
      const T thin = val(F2) > 0.0 ? E * F[r] * F[c] / F2 : F[0] * 0.0;
      const T thick = 4.0 / 3.0 * Jth * W2 * s0.vd[r] * s0.vd[c] + W * (Hth[r] * s0.vd[c] + Hth[c] * s0.vd[r]) +
                      1.0 / 3.0 * Jth * gd[sym(r, c)];
      P[sym(r, c)] = dthin * thin + dthick * thick;
    }
  T Pv[3], vPv = F[0] * 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    Pv[r] = F[0] * 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) Pv[r] = Pv[r] + P[sym(r, c)] * s0.v[c];
    vPv = vPv + s0.v[r] * Pv[r];
  }
  const T J = W2 * (E - 2.0 * vF + vPv);
  const T Sn = W * ((eta + ks * J) - (ka + ks) * (E - vF));
  G[0] = V[0] - Vs[0] - adt * alp * Sn;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const T H = W * (F[r] - Pv[r] - J * s0.vd[r]);
    const T Si = W * (eta - ka * J) * s0.vd[r] - (ka + ks) * H;
    G[1 + r] = V[1 + r] - Vs[1 + r] - adt * alp * Si;
  }
}

__device__ __forceinline__ bool solve4(double A[4][4], double b[4], double x[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int piv = k;
#pragma unroll
    for (int r = k + 1; r < 4; ++r)
      if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
    if (A[piv][k] == 0.0) return false;
    if (piv != k) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double t = A[k][c];
        A[k][c] = A[piv][c];
        A[piv][c] = t;
      }
      const double t = b[k];
      b[k] = b[piv];
      b[piv] = t;
    }
#pragma unroll
    for (int r = k + 1; r < 4; ++r) {
      const double f = A[r][k] / A[k][k];
#pragma unroll
      for (int c = k; c < 4; ++c) A[r][c] -= f * A[k][c];
      b[r] -= f * b[k];
    }
  }
#pragma unroll
  for (int r = 3; r >= 0; --r) {
    double t = b[r];
#pragma unroll
    for (int c = r + 1; c < 4; ++c) t -= A[r][c] * x[c];
    x[r] = t / A[r][r];
  }
  return true;
}

struct ImplArgs {
  Geom g;
  double* U;
  const double* __restrict__ P;
  const double* __restrict__ aux;
  double adt;
  unsigned long long* nfail;
  int nd;       // nonzero: the number densities (U fields 44..46, aux 9..14) follow
  int coupled;  // nonzero: the fluid's taubar, Sbar_i (and DYe) give up what the radiation gains
  double m_b;   // baryon mass of the electron fraction's exchange
};

// the implicit collision solve of the three species at interior point q (padded
// index); returns the number of species solves that did not converge.  With
// coupled, the fluid's taubar and Sbar_i lose what each species' Ebar and
// Fbar_i gain, and DYe loses m_b times the gain of (Nbar_nue - Nbar_nuebar).
__device__ __forceinline__ unsigned long long m1_implicit_at(double* U, const double* __restrict__ P,
                                                           const double* __restrict__ aux, int64_t sf, int64_t q,
                                                           double adt, int nd = 0, int coupled = 0,
                                                           double m_b = 0.0) {
  MetricR m;
  m1_metric(U, sf, q, m);
  const double alp = U[18 * sf + q];
  unsigned long long bad = 0;
  double dN[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
  for (int sp = 0; sp < 3; ++sp) {
    const double ka = aux[(int64_t)(3 * sp) * sf + q], ks = aux[(int64_t)(3 * sp + 1) * sf + q];
    const double eta = aux[(int64_t)(3 * sp + 2) * sf + q];
    M1State s0;
    m1_load_state(U, P, sf, q, sp, m, s0);
    const double chi = m1_closure_chi(s0, m.gd, m.gu);
    const double Vs[4] = {s0.E, s0.F[0], s0.F[1], s0.F[2]};
    double V[4] = {Vs[0], Vs[1], Vs[2], Vs[3]};
    bool ok = false;
    double prev = HUGE_VAL;
    double V1[4] = {Vs[0], Vs[1], Vs[2], Vs[3]};
#pragma unroll 1
    for (int it = 0; it < 60; ++it) {
      const double scale = fabs(V[0]) + fabs(V[1]) + fabs(V[2]) + fabs(V[3]);
      double Jm[4][4], rhs[4], dV[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        Dual Vd[4], Gd[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) Vd[r] = Dual{V[r], r == c ? 1.0 : 0.0};
        implicit_G<Dual>(s0, m.gd, m.gu, chi, Vd, Vs, adt, alp, ka, ks, eta, Gd);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          Jm[r][c] = Gd[r].d;
          if (c == 0) rhs[r] = -Gd[r].v;
        }
      }
      if (!solve4(Jm, rhs, dV)) break;
      double nrm = 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        V[r] += dV[r];
        nrm += fabs(dV[r]);
      }
      if (it == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) V1[r] = V[r];
      }
      // converged, or stopped contracting at the rounding floor
      if (nrm <= 1e-15 * scale || (nrm <= 1e-9 * scale && nrm >= 0.5 * prev)) {
        ok = true;
        break;
      }
      prev = nrm;
    }
    if (!ok) {
      ++bad;
#pragma unroll
      for (int r = 0; r < 4; ++r) V[r] = V1[r];
    }
    {
      const double E0 = U[(int64_t)(32 + 4 * sp) * sf + q];
      U[(int64_t)(32 + 4 * sp) * sf + q] = m.sqrtg * V[0];
      if (coupled) U[24 * sf + q] -= U[(int64_t)(32 + 4 * sp) * sf + q] - E0;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double F0 = U[(int64_t)(33 + 4 * sp + r) * sf + q];
      U[(int64_t)(33 + 4 * sp + r) * sf + q] = m.sqrtg * V[1 + r];
      if (coupled) U[(25 + r) * sf + q] -= U[(int64_t)(33 + 4 * sp + r) * sf + q] - F0;
    }
    if (nd) {
      // the number density, from the moments just stored (read back as the
      // densitized fields they now are) and their closure
      M1State s1;
      m1_load_state(U, P, sf, q, sp, m, s1);
      const double chi1 = m1_closure_chi(s1, m.gd, m.gu);
      double Pij[6], J, H[3], HH;
      m1_closure_eval(s1, m.gd, m.gu, chi1, Pij, J, H, HH);
      const double gam = s1.W * (s1.E - s1.vF) / J;
      const double k0 = aux[(int64_t)(9 + 2 * sp) * sf + q], e0 = aux[(int64_t)(10 + 2 * sp) * sf + q];
      const double Ns = U[(int64_t)(44 + sp) * sf + q] / m.sqrtg;
      double d = -U[(int64_t)(44 + sp) * sf + q];
      U[(int64_t)(44 + sp) * sf + q] = m.sqrtg * (Ns + adt * alp * e0) / (1.0 + adt * alp * k0 / gam);
      d += U[(int64_t)(44 + sp) * sf + q];
      if (sp == 0) dN[0] = d;
      else if (sp == 1) dN[1] = d;
    }
  }
  if (nd && coupled) U[23 * sf + q] -= m_b * (dN[0] - dN[1]);
  return bad;
}

__global__ void __launch_bounds__(256) k_m1_implicit(ImplArgs a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const unsigned long long bad =
      m1_implicit_at(a.U, a.P, a.aux, g.sf, g.at(i + g.ng, j + g.ng, k + g.ng), a.adt, a.nd, a.coupled, a.m_b);
  if (bad && a.nfail) atomicAdd(a.nfail, bad);
}

// the stage state Us of every box (non-converged solves are rare: one atomic
// per thread that has any)
__global__ void __launch_bounds__(256) k_m1_implicit_lv(LevelArgs L) {
  unsigned long long bad = 0;
  for_each_level_point(L, kRegionInterior, [&](const BoxDev& B, int i, int j, int k, bool live) {
    if (!live) return;
    bad += m1_implicit_at(B.Us, B.P, B.aux, B.g.sf, B.g.at(i + B.g.ng, j + B.g.ng, k + B.g.ng), L.adt, L.nd);
  });
  if (bad && L.nfail) atomicAdd(L.nfail, bad);
}

int launch_imex_combine(const Geom& g, int scheme, int nfields, int coupled, int stage, double dt, const double* Un,
                        const double* const* F, const double* const* R, double* Uout, hipStream_t s) {
  ImexArgs a;
  a.g = g;
  a.nfields = nfields;
  a.coupled = coupled;
  a.scheme = scheme;
  a.stage = stage;
  a.dt = dt;
  a.Un = Un;
  for (int st = 0; st < 4; ++st) {
    a.F[st] = F[st];
    a.R[st] = R[st];
  }
  a.Uout = Uout;
  dim3 grd((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz * nfields);
  MHD_LAUNCH(KID_IMEX_COMBINE, k_imex_combine, grd, dim3(64, 4, 1), 0, s, a);
  return (int)hipGetLastError();
}

int launch_imex_combine_level(const LevelArgs& L, int grid, int block, hipStream_t s) {
  MHD_LAUNCH(KID_IMEX_COMBINE, k_imex_combine_lv, dim3(grid), dim3(block), 0, s, L);
  return (int)hipGetLastError();
}

int launch_m1_implicit_level(const LevelArgs& L, int grid, int block, hipStream_t s) {
  MHD_LAUNCH(KID_M1_IMPLICIT, k_m1_implicit_lv, dim3(grid), dim3(block), 0, s, L);
  return (int)hipGetLastError();
}

int launch_m1_implicit(const Geom& g, double* U, const double* P, const double* aux, double adt, int nd, int coupled,
                       double m_b,
                       unsigned long long* nfail, hipStream_t s) {
  ImplArgs a{g, U, P, aux, adt, nfail, nd, coupled, m_b};
  MHD_LAUNCH(KID_M1_IMPLICIT, k_m1_implicit, dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz), dim3(64, 4, 1), 0, s, a);
  return (int)hipGetLastError();
}

}  // namespace mhd
