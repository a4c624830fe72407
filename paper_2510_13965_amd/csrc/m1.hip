// Grey M1 neutrino moments, three species (Sec. 2.3, Sec. 3.4, App. B).
//
// Per species s the evolved fields are Ebar, Fbar_x,y,z (densitized by
// sqrt(gamma)) at U fields 32 + 4 s; per point and species the inputs
// kappa_a, kappa_s, eta sit in aux fields 3 s + (0, 1, 2).
//
//   k_m1_point   every padded point: the Minerbo closure (root xi in [0, 1] of
//                R(xi) = (xi^2 J^2 - H_a H^a)/E^2 by Brent's method), the
//                closure P_ij, the point fluxes of the four fields along each
//                axis and the Minerbo-interpolated point speeds -> workspace
//   k_m1_update  interior points: HO/LO interface fluxes (limiter Phi,
//                opacity switch A = tanh(1/(kappa dx)), odd-even fix), the
//                conservative difference, the geometric sources, the
//                collision sources alpha sqrt(gamma) (S_n, S_i) and their
//                opposite on the fluid's taubar, Sbar_i
// With the number densities Nbar (U fields 44 + s), k_m1_point also stores
// each species' number flux along each axis, (-W beta^k + alpha W v^k +
// alpha H^k/J) Nbar/Gamma, with H^k the spatial part of the four-vector H^a
// (gamma^kj H_j + W (J - E + F_i v^i) beta^k/alpha) and Gamma = W (E - F_i
// v^i)/J, the number current N^a = n (u^a + H^a/J) of Sec. 2.3; k_m1_update
// takes their HO/LO interfaces with the energy moments' speed and opacity
// switch, the source alpha sqrt(gamma) (eta0 - kappa0_a N/Gamma), and adds
// -alpha sqrt(gamma) m_b (C_0 - C_1) to the electron fraction's DYebar.
// The CCZ4 kernels read the closure P_ij from the same workspace for the
// radiation part of the matter terms.
//
// Readings where the text is silent or garbled: the low-order flux is
// 1/2 (F_i + F_i+1) - lambda/2 (u_i+1 - u_i); lambda at an interface is the
// larger point speed; Phi = 0 when u_i+1 = u_i; Phi and the odd-even test act
// per field; P^thin and the thin speed are dropped when F_k F^k = 0; xi = 1 when
// R(1) <= 0 and xi = 0 when R(0) >= 0; a negative argument of the thick-speed
// root counts as 0; kappa = 0 gives A = 1.  Everything runs in one fixed
// evaluation order without FMA contraction.
#include "m1_dev.hpp"
#include "prof.hpp"

namespace mhd {

#pragma clang fp contract(off)

struct M1Args {
  Geom g;
  const double* __restrict__ U;
  const double* __restrict__ P;
  const double* __restrict__ aux;
  double* __restrict__ W;  // M1 workspace (kM1Fields fields)
  double* __restrict__ rhs;
  unsigned long long* max_speed;
  double* __restrict__ stiff;  // IMEX split: the radiation's collision terms (12 or 15 fields), or null
  int nd;                      // nonzero: the number densities are evolved (47 fields, 15 aux, 75 workspace fields)
  double m_b;                  // reference baryon mass of the electron-fraction source
  int coupled;                 // with stiff: the fluid's share of the exchange goes to stiff too (after the radiation's)
};

// padded indices
template <bool ND>
__device__ __forceinline__ void m1_point_at(const M1Args& a, int i, int j, int k) {
  const Geom& g = a.g;
  const int64_t sf = g.sf, p = g.at(i, j, k);
  MetricR m;
  m1_metric(a.U, sf, p, m);
  const double alp = a.U[18 * sf + p];
#pragma unroll 1
  for (int sp = 0; sp < 3; ++sp) {
    M1State s;
    m1_load_state(a.U, a.P, sf, p, sp, m, s);
    const double chi = m1_closure_chi(s, m.gd, m.gu);
    double Pij[6], J, H[3], HH;
    m1_closure_eval(s, m.gd, m.gu, chi, Pij, J, H, HH);
#pragma unroll
    for (int c = 0; c < 6; ++c) a.W[(kM1Closure + 6 * sp + c) * sf + p] = Pij[c];
    const double Eb = a.U[(32 + 4 * sp) * sf + p];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double bd = a.U[(19 + d) * sf + p];
      double* f = a.W + (int64_t)(kM1Flux + 5 * (3 * sp + d)) * sf + p;
      f[0] = -bd * Eb + alp * m.sqrtg * s.Fu[d];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double Pdc = 0.0;
#pragma unroll
        for (int e = 0; e < 3; ++e) Pdc += m.gu[sym(d, e)] * Pij[sym(e, c)];
        f[(1 + c) * sf] = -bd * a.U[(33 + 4 * sp + c) * sf + p] + alp * m.sqrtg * Pdc;
      }
      f[4 * sf] = m1_speed(s, m.gu, chi, alp, bd, d);
    }
    if (ND) {
      const double gam = s.W * (s.E - s.vF) / J;
      a.W[(int64_t)(kM1Gamma + sp) * sf + p] = gam;
      const double Hn = s.W * (J - s.E + s.vF);
      const double Nb = a.U[(int64_t)(44 + sp) * sf + p];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double bd = a.U[(19 + d) * sf + p];
        double Hu = Hn * bd / alp;
#pragma unroll
        for (int e = 0; e < 3; ++e) Hu += m.gu[sym(d, e)] * H[e];
        a.W[(int64_t)(kM1NFlux + 3 * sp + d) * sf + p] = (-s.W * bd + alp * s.W * s.v[d] + alp * Hu / J) * Nb / gam;
      }
    }
  }
}

// ND: the number densities too (a compile-time switch, so the kernels without
// them carry none of their registers)
// The update reads the point fluxes and speeds at the interior points and
// their first neighbours, and the closure at the interior points, so the pass
// covers the interior and one ghost layer (grid over nx + 2, ny + 2, nz + 2).
template <bool ND>
__global__ void __launch_bounds__(256) k_m1_point(M1Args a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nx + 2 || j >= g.ny + 2) return;
  m1_point_at<ND>(a, i + g.ng - 1, j + g.ng - 1, k + g.ng - 1);
}

// Lax-Friedrichs speed and the thick-limit weight A = tanh(1/(kappa h)) at the
// interface between points 0 and 1 of the three-point columns (lam, kappa_a,
// kappa_s at p - st, p, p + st: o = 0 for the interface below p, 1 above);
// both are shared by the four fields of a species, so they are evaluated once
// per interface
struct M1Iface {
  double lh, A;
};
__device__ __forceinline__ M1Iface m1_iface(const double (&lam)[3], const double (&ka)[3], const double (&ks)[3],
                                            int o, double h) {
  M1Iface r;
  r.lh = fmax(lam[o], lam[o + 1]);
  const double kap = 0.5 * (ka[o] + ka[o + 1] + ks[o] + ks[o + 1]);
  r.A = kap > 0.0 ? tanh(1.0 / (kap * h)) : 1.0;
  return r;
}

// interface value of one field between u0 and u1 (um, u2 the next points out;
// f0, f1 the point fluxes at u0 and u1)
__device__ __forceinline__ double m1_holo(double um, double u0, double u1, double u2, double f0, double f1,
                                          const M1Iface& w) {
  const double fho = 0.5 * (f0 + f1);
  const double flo = fho - 0.5 * w.lh * (u1 - u0);
  const double du = u1 - u0;
  double phi = 0.0;
  // min(2 (u0 - um) / du, 2 (u2 - u1) / du) with one division: rounding is
  // monotone, so the smaller quotient is the quotient of the smaller numerator
  // for du > 0 and of the larger one for du < 0 (same bits, NaNs included)
  if (du != 0.0) {
    const double a = u0 - um, b = u2 - u1;
    phi = fmax(0.0, fmin(1.0, 2.0 * (du > 0.0 ? fmin(a, b) : fmax(a, b)) / du));
  }
  double A = w.A;
  if ((u0 - um) * du < 0.0 && du * (u2 - u1) < 0.0) A = 1.0;
  return fho - A * (1.0 - phi) * (fho - flo);
}

// flux difference -(F_{p+1/2} - F_{p-1/2}) / h of one field along st
__device__ __forceinline__ double m1_fdiff(const double* u, const double* f, const M1Iface& wl, const M1Iface& wr,
                                           int64_t st, uint32_t voff, int s8, double h, double ih) {
  double v[5], fv[3];
  ld_col(u, st, 2, voff, s8, v);
  ld_col(f, st, 1, voff, s8, fv);
  const double fr = m1_holo(v[1], v[2], v[3], v[4], fv[1], fv[2], wr);
  const double fl = m1_holo(v[0], v[1], v[2], v[3], fv[0], fv[1], wl);
  return div_rn(fr - fl, h, ih);
}

// interior indices; returns the largest M1 point speed at the point (0 if not live)
template <bool ND>
__device__ __forceinline__ double m1_update_at(const M1Args& a, int i, int j, int k, bool live) {
  const Geom& g = a.g;
  const int64_t sf = g.sf;
  const int64_t q = live ? g.at(i + g.ng, j + g.ng, k + g.ng) : g.at(g.ng, g.ng, k + g.ng);
  const double* __restrict__ U = a.U;
  double vmax = 0.0;
  if (live) {
    const uint32_t voff = (uint32_t)(q * 8);
    MetricR m;
    m1_metric(U, sf, q, m);
    const double chi = U[12 * sf + q];
    const double alp = U[18 * sf + q], Kh = U[13 * sf + q], Th = U[14 * sf + q];
    // flux differences of the three species first (the metric derivatives of
    // the sources are not live meanwhile); each output then gets its
    // geometric and collision terms in the same order as before
    double outs[3][4], outN[3] = {0.0, 0.0, 0.0};
    const double hx = g.h[0], hy = g.h[1], hz = g.h[2];
    const double ihx = g.idx[0], ihy = g.idx[1], ihz = g.idx[2];
#pragma unroll 1
    for (int sp = 0; sp < 3; ++sp) {
      double out[4] = {0.0, 0.0, 0.0, 0.0};
      const double* ka = a.aux + (int64_t)(3 * sp) * sf;
      const double* ks = a.aux + (int64_t)(3 * sp + 1) * sf;
#pragma unroll 1
      for (int d = 0; d < 3; ++d) {
        const int64_t st = g.stride(d);
        const double* lam = a.W + (int64_t)(kM1Flux + 5 * (3 * sp + d) + 4) * sf;
        vmax = fmax(vmax, lam[q]);
        const double h = d == 0 ? hx : (d == 1 ? hy : hz), ih = d == 0 ? ihx : (d == 1 ? ihy : ihz);
        const int s8 = (int)(st * 8);
        double lv[3], kav[3], ksv[3];
        ld_col(lam, st, 1, voff, s8, lv);
        ld_col(ka, st, 1, voff, s8, kav);
        ld_col(ks, st, 1, voff, s8, ksv);
        const M1Iface wr = m1_iface(lv, kav, ksv, 1, h), wl = m1_iface(lv, kav, ksv, 0, h);
#pragma unroll
        for (int c = 0; c < 4; ++c)
          out[c] -= m1_fdiff(U + (int64_t)(32 + 4 * sp + c) * sf, a.W + (int64_t)(kM1Flux + 5 * (3 * sp + d) + c) * sf,
                             wl, wr, st, voff, s8, h, ih);
        if (ND) {
          const double dN = m1_fdiff(U + (int64_t)(44 + sp) * sf, a.W + (int64_t)(kM1NFlux + 3 * sp + d) * sf, wl, wr,
                                     st, voff, s8, h, ih);
          if (sp == 0) outN[0] -= dN;
          else if (sp == 1) outN[1] -= dN;
          else outN[2] -= dN;
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (sp == 0) outs[0][c] = out[c];
        else if (sp == 1) outs[1][c] = out[c];
        else outs[2][c] = out[c];
      }
    }
    double dalp[3], dchi[3], dbeta[3][3], dgt[3][6];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t st = g.stride(d);
      dalp[d] = fd1(U + 18 * sf, st, voff, g.i12[d]);
      dchi[d] = fd1(U + 12 * sf, st, voff, g.i12[d]);
#pragma unroll
      for (int b = 0; b < 3; ++b) dbeta[d][b] = fd1(U + (19 + b) * sf, st, voff, g.i12[d]);
#pragma unroll
      for (int c = 0; c < 6; ++c) dgt[d][c] = fd1(U + c * sf, st, voff, g.i12[d]);
    }
#pragma unroll 1
    for (int sp = 0; sp < 3; ++sp) {
      double out[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) out[c] = sp == 0 ? outs[0][c] : (sp == 1 ? outs[1][c] : outs[2][c]);
      const double* ka = a.aux + (int64_t)(3 * sp) * sf;
      const double* ks = a.aux + (int64_t)(3 * sp + 1) * sf;
      // closure quantities at the point
      M1State s;
      m1_load_state(U, a.P, sf, q, sp, m, s);
      double Pij[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) Pij[c] = a.W[(kM1Closure + 6 * sp + c) * sf + q];
      double Pv[3], vPv = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        Pv[r] = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) Pv[r] += Pij[sym(r, c)] * s.v[c];
        vPv += s.v[r] * Pv[r];
      }
      const double J = s.W * s.W * (s.E - 2.0 * s.vF + vPv);
      double H[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) H[r] = s.W * (s.F[r] - Pv[r] - J * s.vd[r]);
      // geometric sources
      double Pbu[3][3], trP = 0.0, Fbu[3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          double t = 0.0;
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int e = 0; e < 3; ++e) t += m.gu[sym(r, c)] * m.gu[sym(b, e)] * Pij[sym(c, e)];
          Pbu[r][b] = m.sqrtg * t;
        }
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int b = 0; b < 3; ++b) trP += m.gd[sym(r, b)] * Pbu[r][b];
      const double Fb[3] = {U[(33 + 4 * sp) * sf + q], U[(34 + 4 * sp) * sf + q], U[(35 + 4 * sp) * sf + q]};
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        Fbu[r] = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b) Fbu[r] += m.gu[sym(r, b)] * Fb[b];
      }
      const double Eb = U[(32 + 4 * sp) * sf + q];
      {
        double r = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2)
#pragma unroll
          for (int b = 0; b < 3; ++b) r += alp / chi * Pbu[a2][b] * U[(6 + sym(a2, b)) * sf + q];
        r += alp / 3.0 * trP * (Kh + 2.0 * Th);
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2) r -= Fbu[a2] * dalp[a2];
        out[0] += r;
      }
#pragma unroll
      for (int a2 = 0; a2 < 3; ++a2) {
        double r = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
          for (int c = 0; c < 3; ++c) r += Pbu[b][c] * dgt[a2][sym(b, c)];
        r = alp / (2.0 * chi) * (r - trP * dchi[a2]);
#pragma unroll
        for (int b = 0; b < 3; ++b) r += Fb[b] * dbeta[a2][b];
        r -= Eb * dalp[a2];
        out[1 + a2] += r;
      }
      // collisions, and the opposite exchange with the fluid
      const double kA = ka[q], kS = ks[q], eta = a.aux[(int64_t)(3 * sp + 2) * sf + q];
      const double Sn = s.W * ((eta + kS * J) - (kA + kS) * (s.E - s.vF));
      double Si[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) Si[r] = s.W * (eta - kA * J) * s.vd[r] - (kA + kS) * H[r];
      if (a.stiff) {
        a.stiff[(int64_t)(4 * sp) * sf + q] = alp * m.sqrtg * Sn;
#pragma unroll
        for (int r = 0; r < 3; ++r) a.stiff[(int64_t)(4 * sp + 1 + r) * sf + q] = alp * m.sqrtg * Si[r];
      } else {
        out[0] += alp * m.sqrtg * Sn;
#pragma unroll
        for (int r = 0; r < 3; ++r) out[1 + r] += alp * m.sqrtg * Si[r];
      }
      if (a.stiff && a.coupled) {
        // the fluid's share in the stiff part too: slots (12 or 15) + 0 (tau), + 1..3 (S_i)
        double* fs = a.stiff + (int64_t)(ND ? 15 : 12) * sf + q;
        fs[0] = (sp == 0 ? 0.0 : fs[0]) - alp * m.sqrtg * Sn;
#pragma unroll
        for (int r = 0; r < 3; ++r) fs[(1 + r) * sf] = (sp == 0 ? 0.0 : fs[(1 + r) * sf]) - alp * m.sqrtg * Si[r];
      } else {
        a.rhs[24 * sf + q] -= alp * m.sqrtg * Sn;
#pragma unroll
        for (int r = 0; r < 3; ++r) a.rhs[(25 + r) * sf + q] -= alp * m.sqrtg * Si[r];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) a.rhs[(int64_t)(32 + 4 * sp + c) * sf + q] = out[c];
    }
    if (ND) {
      // number densities: emission and absorption, and the electron fraction's source
      double C[3];
#pragma unroll 1
      for (int sp = 0; sp < 3; ++sp) {
        const double k0 = a.aux[(int64_t)(9 + 2 * sp) * sf + q], e0 = a.aux[(int64_t)(10 + 2 * sp) * sf + q];
        const double gam = a.W[(int64_t)(kM1Gamma + sp) * sf + q];
        const double Cs = e0 - k0 * (U[(int64_t)(44 + sp) * sf + q] / m.sqrtg) / gam;
        double o = sp == 0 ? outN[0] : (sp == 1 ? outN[1] : outN[2]);
        if (a.stiff)
          a.stiff[(int64_t)(12 + sp) * sf + q] = alp * m.sqrtg * Cs;
        else
          o += alp * m.sqrtg * Cs;
        a.rhs[(int64_t)(44 + sp) * sf + q] = o;
        if (sp == 0) C[0] = Cs;
        else if (sp == 1) C[1] = Cs;
        else C[2] = Cs;
      }
      if (a.stiff && a.coupled)
        a.stiff[(int64_t)(15 + 4) * sf + q] = -alp * m.sqrtg * a.m_b * (C[0] - C[1]);
      else
        a.rhs[23 * sf + q] -= alp * m.sqrtg * a.m_b * (C[0] - C[1]);
    }
  }
  return vmax;
}

template <bool ND>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_m1_update(M1Args a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  const double vmax = m1_update_at<ND>(a, i, j, k, i < g.nx && j < g.ny);
  if (a.max_speed) block_max_to(a.max_speed, vmax);
}

// levels: the same point functions over every box, one persistent launch each
template <bool ND>
__global__ void __launch_bounds__(256) k_m1_point_lv(LevelArgs L) {
  for_each_level_point(L, kRegionHalo1, [&](const BoxDev& B, int i, int j, int k, bool live) {
    if (!live) return;
    const M1Args a{B.g, L.src ? B.Us : B.U, B.P, B.aux, B.ws_m1, nullptr, nullptr, nullptr, ND, L.par.m_b, 0};
    m1_point_at<ND>(a, i, j, k);
  });
}

template <bool IMEX, bool ND>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_m1_update_lv(LevelArgs L) {
  double vmax = 0.0;
  for_each_level_point(L, kRegionInterior, [&](const BoxDev& B, int i, int j, int k, bool live) {
    const M1Args a{B.g,      L.src ? B.Us : B.U, B.P, B.aux, B.ws_m1, level_rhs<IMEX>(B, L), L.max_speed,
                   level_stiff<IMEX>(B, L), ND, L.par.m_b, 0};
    vmax = fmax(vmax, m1_update_at<ND>(a, i, j, k, live));
  });
  if (L.max_speed) block_max_to(L.max_speed, vmax);
}

int m1_workspace_fields(bool nd) { return nd ? kM1NFields : kM1Fields; }

int launch_m1_point_level(const LevelArgs& L, int grid, int block, hipStream_t s) {
  if (L.nd)
    MHD_LAUNCH(KID_M1_POINT, k_m1_point_lv<true>, dim3(grid), dim3(block), 0, s, L);
  else
    MHD_LAUNCH(KID_M1_POINT, k_m1_point_lv<false>, dim3(grid), dim3(block), 0, s, L);
  return (int)hipGetLastError();
}

int launch_m1_update_level(const LevelArgs& L, int grid, int block, hipStream_t s) {
  if (L.slot >= 0) {
    if (L.nd)
      MHD_LAUNCH(KID_M1_UPDATE, (k_m1_update_lv<true, true>), dim3(grid), dim3(block), 0, s, L);
    else
      MHD_LAUNCH(KID_M1_UPDATE, (k_m1_update_lv<true, false>), dim3(grid), dim3(block), 0, s, L);
  } else {
    if (L.nd)
      MHD_LAUNCH(KID_M1_UPDATE, (k_m1_update_lv<false, true>), dim3(grid), dim3(block), 0, s, L);
    else
      MHD_LAUNCH(KID_M1_UPDATE, (k_m1_update_lv<false, false>), dim3(grid), dim3(block), 0, s, L);
  }
  return (int)hipGetLastError();
}

int launch_m1_point(const Geom& g, const double* U, const double* P, const double* aux, double* ws, int nd,
                    hipStream_t s) {
  M1Args a{g, U, P, aux, ws, nullptr, nullptr, nullptr, nd, 0.0, 0};
  const int Nx = g.nx + 2, Ny = g.ny + 2, Nz = g.nz + 2;  // the interior and one ghost layer
  const dim3 grd((Nx + 63) / 64, (Ny + 3) / 4, Nz);
  if (nd)
    MHD_LAUNCH(KID_M1_POINT, k_m1_point<true>, grd, dim3(64, 4, 1), 0, s, a);
  else
    MHD_LAUNCH(KID_M1_POINT, k_m1_point<false>, grd, dim3(64, 4, 1), 0, s, a);
  return (int)hipGetLastError();
}

int launch_m1_update(const Geom& g, const double* U, const double* P, const double* aux, double* ws, double* rhs,
                     double* max_speed, double* stiff, int nd, double m_b, int coupled, hipStream_t s) {
  M1Args a{g, U, P, aux, ws, rhs, reinterpret_cast<unsigned long long*>(max_speed), stiff, nd, m_b, coupled};
  const dim3 grd((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz);
  if (nd)
    MHD_LAUNCH(KID_M1_UPDATE, k_m1_update<true>, grd, dim3(64, 4, 1), 0, s, a);
  else
    MHD_LAUNCH(KID_M1_UPDATE, k_m1_update<false>, grd, dim3(64, 4, 1), 0, s, a);
  return (int)hipGetLastError();
}

}  // namespace mhd
