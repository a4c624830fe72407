// GRMHD part of the right-hand side (Sec. 2.2 balance laws with divergence
// cleaning; Sec. 3.3 conservative Lax-Friedrichs / MP5 scheme; App. B speeds).
//
// Two passes over the patch:
//   k_mhd_point   every padded point: the physical fluxes F^d of the 10
//                 densitized fields for d = x,y,z and the point speed lambda^d
//                 (fast-magnetosonic bound for normal propagation, and the
//                 cleaning mode -beta^d +- alpha c_b sqrt(gamma^dd)); the
//                 metric, S_ij and the EoS are evaluated once for all three
//                 directions.  Written to the workspace (33 fields).
//   k_mhd_update  every interior point: for each direction the interface
//                 fluxes at i-1/2 and i+1/2 (lambda = max over the six
//                 reconstruction points, F^pm = (F +- lambda U)/2, MP5 on F^+
//                 and mirrored on F^-), -(Fhat_{i+1/2} - Fhat_{i-1/2})/dx,
//                 plus the geometric sources with centred metric derivatives,
//                 plus the wavefront max of the point speeds (CFL reduction).
#include "dev_common.hpp"
#include "prof.hpp"

namespace mhd {

// Reproducible evaluation order.  For smooth flows the interface fluxes cancel
// to a flux difference 5-6 orders of magnitude below the fluxes themselves, so
// one rounding of a point flux (1e-16 relative) is 1e-11..1e-10 of the
// right-hand side.  The point fluxes, speeds, the Lax-Friedrichs split and
// the MP5 reconstruction are therefore evaluated in a fixed order of plain
// IEEE operations, FMA contraction off, with the divisions the formulas
// contain (metric inverse by the determinant, undensitizing by sqrt(gamma),
// the 1/60 of the interpolant, computed as a correctly rounded quotient with
// div_rn, 1/dx of the difference); any FP64 implementation following the same
// order gets identical results.
#pragma clang fp contract(off)

// ------------------------------------------------------------------ MP5 (Sec. 3.3)

// minmod of 2 and 4 arguments: the argument of least magnitude when all share a
// strict sign, else 0; taken from the extremes (the smallest is the answer when it
// is positive, the largest when it is negative), which gives the same bits as the
// case-by-case definition with fewer compares and selects
__device__ __forceinline__ double minmod2(double a, double b) {
  const double lo = fmin(a, b), hi = fmax(a, b);
  return lo > 0.0 ? lo : (hi < 0.0 ? hi : 0.0);
}

__device__ __forceinline__ double minmod4(double a, double b, double c, double d) {
  const double lo = fmin(fmin(a, b), fmin(c, d)), hi = fmax(fmax(a, b), fmax(c, d));
  return lo > 0.0 ? lo : (hi < 0.0 ? hi : 0.0);
}

// value at i+1/2 from F_{i-2} .. F_{i+2} (= a b c d e)
__device__ __forceinline__ double mp5(double a, double b, double c, double d, double e, double alpha) {
  // identical inputs: the limiter below returns c exactly (every difference is 0,
  // so lo = hi = c and the final correction is minmod2(., 0) = 0); zero
  // magnetic and cleaning fields outside matter take this exit
  if (a == c && b == c && d == c && e == c) return c;
  const double unl = div_rn(2.0 * a - 13.0 * b + 47.0 * c + 27.0 * d - 3.0 * e, 60.0, 1.0 / 60.0);
  const double dm = c - b;
  const double fmp = c + minmod2(d - c, alpha * dm);
  if ((unl - c) * (unl - fmp) < 0.0) return unl;
  const double ddm = a - 2.0 * b + c;
  const double dd0 = b - 2.0 * c + d;
  const double ddp = c - 2.0 * d + e;
  const double m4p = minmod4(4.0 * dd0 - ddp, 4.0 * ddp - dd0, dd0, ddp);
  const double m4m = minmod4(4.0 * ddm - dd0, 4.0 * dd0 - ddm, ddm, dd0);
  const double ful = c + alpha * dm;
  const double fmd = 0.5 * (c + d) - 0.5 * m4p;
  const double flc = c + 0.5 * dm + (4.0 / 3.0) * m4m;
  const double lo = fmax(fmin(fmin(c, d), fmd), fmin(fmin(c, ful), flc));
  const double hi = fmin(fmax(fmax(c, d), fmd), fmax(fmax(c, ful), flc));
  return lo + minmod2(unl - lo, hi - lo);
}

// ------------------------------------------------------------------ point fluxes

struct MhdPointArgs {
  Geom g;
  mhd_params_t par;
  mhd_eos_t eos;
  const double* __restrict__ U;
  const double* __restrict__ P;
  double* __restrict__ W;  // workspace: (d*11 + f) * sf, f = 0..9 fluxes, 10 = speed
};

// lowering in index order: o_i = ((g_i0 v0 + g_i1 v1) + g_i2 v2)
__device__ __forceinline__ void lower3(const double g[6], const double v[3], double o[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) o[i] = g[sym(i, 0)] * v[0] + g[sym(i, 1)] * v[1] + g[sym(i, 2)] * v[2];
}

__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// S_ij of the magnetised fluid (Sec. 2.2), lower indices, undensitized:
// 1/2 (v_i S_j + v_j S_i) + gamma_ij p - 1/(2W^2) [2 B_i B_j - gamma_ij B^2]
//   - 1/2 (B.v) [B_i v_j + B_j v_i - gamma_ij (B.v)]
__device__ __forceinline__ void stress(const double gd[6], const double vd[3], const double S[3],
                                       const double Bd[3], double pr, double B2, double Bv, double W,
                                       double Sij[6]) {
  const double hw = 0.5 / (W * W);
  const double hb = 0.5 * Bv;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const int a = sym(i, j);
      Sij[a] = 0.5 * (vd[i] * S[j] + vd[j] * S[i]) + gd[a] * pr - hw * (2.0 * Bd[i] * Bd[j] - gd[a] * B2) -
               hb * (Bd[i] * vd[j] + Bd[j] * vd[i] - gd[a] * Bv);
    }
}

// c_s^2 = (dp/drho + p/rho^2 dp/deps) / (1 + eps + p/rho) for the hybrid EoS
__device__ __forceinline__ double cs2_repro(const mhd_eos_t& e, double rho, double eps) {
  int i = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b)
    if (b < e.npieces - 1 && rho >= e.rho_b[b]) i = b + 1;
  const double K = e.K[i], G = e.Gamma[i], gth = e.Gamma_th;
  const double pc = (K == 0.0) ? 0.0 : K * pow(rho, G);
  const double ec = (K == 0.0) ? e.a[i] : e.a[i] + K / (G - 1.0) * pow(rho, G - 1.0);
  const double p = pc + (gth - 1.0) * rho * (eps - ec);
  const double dpdrho = G * pc / rho + (gth - 1.0) * (eps - ec) - (gth - 1.0) * pc / rho;
  const double dpdeps = (gth - 1.0) * rho;
  return (dpdrho + p / (rho * rho) * dpdeps) / (1.0 + eps + p / rho);
}

// padded indices (i, j, k) of a point inside the padded patch
__device__ __forceinline__ void mhd_point_at(const MhdPointArgs& a, const mhd_params_t& par, const mhd_eos_t& eos, int i,
                                             int j, int k) {
  const Geom& g = a.g;
  const int64_t sf = g.sf;
  const int64_t p = g.at(i, j, k);
  const double* __restrict__ U = a.U;
  const double* __restrict__ P = a.P;

  double gt[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) gt[c] = U[c * sf + p];
  const double chi = U[12 * sf + p];
  MetricR m;
  metric_repro(gt, chi, m);
  const double alp = U[18 * sf + p];
  const double beta[3] = {U[19 * sf + p], U[20 * sf + p], U[21 * sf + p]};
  const double Dbar = U[22 * sf + p], DYbar = U[23 * sf + p], taubar = U[24 * sf + p];
  const double Sbar[3] = {U[25 * sf + p], U[26 * sf + p], U[27 * sf + p]};
  const double Bbar[3] = {U[28 * sf + p], U[29 * sf + p], U[30 * sf + p]};
  const double phibar = U[31 * sf + p];
  const double rho = P[p], eps = P[sf + p], pr = P[2 * sf + p];
  const double v[3] = {P[3 * sf + p], P[4 * sf + p], P[5 * sf + p]};
  const double W = P[6 * sf + p];

  const double B[3] = {Bbar[0] / m.sqrtg, Bbar[1] / m.sqrtg, Bbar[2] / m.sqrtg};
  const double S[3] = {Sbar[0] / m.sqrtg, Sbar[1] / m.sqrtg, Sbar[2] / m.sqrtg};
  double vd[3], Bd[3];
  lower3(m.gd, v, vd);
  lower3(m.gd, B, Bd);
  const double B2 = dot3(B, Bd);
  const double Bv = dot3(B, vd);
  const double v2 = dot3(v, vd);
  double Sij[6];
  stress(m.gd, vd, S, Bd, pr, B2, Bv, W, Sij);

  // characteristic speed ingredients (App. B)
  const double h = rho * (1.0 + eps) + pr;
  const double b2 = B2 / (W * W) + Bv * Bv;
  const double cs2 = cs2_repro(eos, rho, eps);
  const double ca2 = b2 / (h + b2);
  const double a2 = cs2 + ca2 - cs2 * ca2;
  const double cb = par.c_b;

  double* __restrict__ Wk = a.W + p;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double vk = v[d];
    double* __restrict__ o = Wk + (int64_t)(d * 11) * sf;
    const double adv = -beta[d] + alp * vk;
    o[0] = adv * Dbar;
    o[sf] = adv * DYbar;
    const double Supd = m.gu[sym(d, 0)] * Sbar[0] + m.gu[sym(d, 1)] * Sbar[1] + m.gu[sym(d, 2)] * Sbar[2];
    o[2 * sf] = -beta[d] * taubar + alp * (Supd - Dbar * vk);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double Smix = m.gu[sym(d, 0)] * Sij[sym(0, c)] + m.gu[sym(d, 1)] * Sij[sym(1, c)] +
                          m.gu[sym(d, 2)] * Sij[sym(2, c)];
      o[(3 + c) * sf] = -beta[d] * Sbar[c] + alp * m.sqrtg * Smix;
      o[(6 + c) * sf] = Bbar[c] * (alp * vk - beta[d]) - Bbar[d] * (alp * v[c] - beta[c]) +
                        alp * chi * m.gtu[sym(d, c)] * phibar;
    }
    o[9 * sf] = -beta[d] * phibar + alp * cb * cb * Bbar[d];
    const double gdd = m.gu[sym(d, d)];
    const double rad = a2 * (1.0 - v2) * ((1.0 - v2 * a2) * gdd - (1.0 - a2) * vk * vk);
    const double sq = sqrt(fmax(rad, 0.0));
    const double lp = -beta[d] + alp / (1.0 - v2 * a2) * ((1.0 - a2) * vk + sq);
    const double lm = -beta[d] + alp / (1.0 - v2 * a2) * ((1.0 - a2) * vk - sq);
    const double cp = -beta[d] + alp * cb * sqrt(gdd);
    const double cm = -beta[d] - alp * cb * sqrt(gdd);
    o[10 * sf] = fmax(fmax(fabs(lp), fabs(lm)), fmax(fabs(cp), fabs(cm)));
  }
}

// ------------------------------------------------------------------ update

struct MhdUpdArgs {
  Geom g;
  int nbx, nby, nbz, strip;  // tile grid (64x4 tiles) and strip height of the tile order
  mhd_params_t par;
  const double* __restrict__ U;
  const double* __restrict__ P;
  const double* __restrict__ W;
  double* __restrict__ rhs;
  unsigned long long* max_speed;  // bit pattern of a non-negative double
};

// interior indices (i, j, k); lanes without a point come with live = false
// and a valid k.  Returns the largest point speed at the point (0 if not live).
__device__ __forceinline__ double mhd_update_at(const MhdUpdArgs& a, int i, int j, int k, bool live) {
  const Geom& g = a.g;
  const int64_t sf = g.sf;
  const int64_t p = live ? g.at(i + g.ng, j + g.ng, k + g.ng) : g.at(g.ng, g.ng, k + g.ng);
  const double* __restrict__ U = a.U;
  const double* __restrict__ P = a.P;
  const uint32_t voff = (uint32_t)(p * 8);
  const double alpha_mp5 = a.par.alpha_mp5;

  double out[10];
#pragma unroll
  for (int f = 0; f < 10; ++f) out[f] = 0.0;
  double vmax = 0.0;

  // spacings as values: selecting among fields of a local copy of the geometry
  // (level kernels build one per box) would keep that copy in private memory
  const double hx = g.h[0], hy = g.h[1], hz = g.h[2];
  const double ihx = g.idx[0], ihy = g.idx[1], ihz = g.idx[2];
#pragma unroll 1
  for (int d = 0; d < 3; ++d) {
    const int64_t s = g.stride(d);
    const int s8 = (int)(s * 8);
    double l[7];
    ld_col(a.W + (int64_t)(d * 11 + 10) * sf, s, 3, voff, s8, l);
    vmax = fmax(vmax, l[3]);
    double lL = 0.0, lR = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      lL = fmax(lL, l[m]);
      lR = fmax(lR, l[m + 1]);
    }
    const double hd = d == 0 ? hx : (d == 1 ? hy : hz);
    const double ihd = d == 0 ? ihx : (d == 1 ? ihy : ihz);
#pragma unroll
    for (int f = 0; f < 10; ++f) {
      double F[7], u[7];
      ld_col(a.W + (int64_t)(d * 11 + f) * sf, s, 3, voff, s8, F);
      ld_col(U + (int64_t)(22 + f) * sf, s, 3, voff, s8, u);
      // 2 F^+ and 2 F^- (MP5 is homogeneous, so the factor 1/2 is applied once at the end)
      double pR[7], mR[7], pL[7], mL[7];
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        pR[m] = F[m] + lR * u[m];
        mR[m] = F[m] - lR * u[m];
        pL[m] = F[m] + lL * u[m];
        mL[m] = F[m] - lL * u[m];
      }
      // interface i+1/2: F^+ on i-2..i+2 (m = 1..5), F^- mirrored on i+3..i-1 (m = 6..2)
      const double fr = 0.5 * (mp5(pR[1], pR[2], pR[3], pR[4], pR[5], alpha_mp5) +
                               mp5(mR[6], mR[5], mR[4], mR[3], mR[2], alpha_mp5));
      // interface i-1/2: F^+ on i-3..i+1 (m = 0..4), F^- mirrored on i+2..i-2 (m = 5..1)
      const double fl = 0.5 * (mp5(pL[0], pL[1], pL[2], pL[3], pL[4], alpha_mp5) +
                               mp5(mL[5], mL[4], mL[3], mL[2], mL[1], alpha_mp5));
      out[f] -= div_rn(fr - fl, hd, ihd);
    }
  }

  // geometric sources (Sec. 2.2) with centred metric derivatives
  {
    const int64_t st[3] = {1, g.sy, g.sz};
    double gt[6], At[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      gt[c] = U[c * sf + p];
      At[c] = U[(6 + c) * sf + p];
    }
    const double chi = U[12 * sf + p], Kh = U[13 * sf + p], Th = U[14 * sf + p];
    const double Gh[3] = {U[15 * sf + p], U[16 * sf + p], U[17 * sf + p]};
    const double alp = U[18 * sf + p];
    double gtu[6];
    const double det = sym_inv(gt, gtu);
    const double ichi = 1.0 / chi;
    double gd[6], gu[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      gd[c] = gt[c] * ichi;
      gu[c] = gtu[c] * chi;
    }
    const double sqrtg = sqrt(det * ichi * ichi * ichi);
    const double isg = 1.0 / sqrtg;
    double dalp[3], dchi[3], db[3][3], dg[3][6];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      dalp[d] = fd1(U + 18 * sf, st[d], voff, g.i12[d]);
      dchi[d] = fd1(U + 12 * sf, st[d], voff, g.i12[d]);
#pragma unroll
      for (int c = 0; c < 3; ++c) db[d][c] = fd1(U + (19 + c) * sf, st[d], voff, g.i12[d]);
#pragma unroll
      for (int c = 0; c < 6; ++c) dg[d][c] = fd1(U + c * sf, st[d], voff, g.i12[d]);
    }
    // Z^i = chi/2 (Ghat^i - Gt^i), Gt^i = gt^{ij} gt^{kl} d_l gt_jk
    double w[3], Gt[3];
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      double s = 0.0;
#pragma unroll
      for (int kk = 0; kk < 3; ++kk)
#pragma unroll
        for (int ll = 0; ll < 3; ++ll) s += gtu[sym(kk, ll)] * dg[ll][sym(jj, kk)];
      w[jj] = s;
    }
    sym_mv(gtu, w, Gt);

    const double Dbar = U[22 * sf + p], taubar = U[24 * sf + p], phibar = U[31 * sf + p];
    const double Sbar[3] = {U[25 * sf + p], U[26 * sf + p], U[27 * sf + p]};
    const double Bbar[3] = {U[28 * sf + p], U[29 * sf + p], U[30 * sf + p]};
    const double v[3] = {P[3 * sf + p], P[4 * sf + p], P[5 * sf + p]};
    const double W = P[6 * sf + p], pr = P[2 * sf + p];
    const double B[3] = {Bbar[0] * isg, Bbar[1] * isg, Bbar[2] * isg};
    const double S[3] = {Sbar[0] * isg, Sbar[1] * isg, Sbar[2] * isg};
    double vd[3], Bd[3];
    sym_mv(gd, v, vd);
    sym_mv(gd, B, Bd);
    const double B2 = B[0] * Bd[0] + B[1] * Bd[1] + B[2] * Bd[2];
    const double Bv = B[0] * vd[0] + B[1] * vd[1] + B[2] * vd[2];
    double Sij[6];
    stress(gd, vd, S, Bd, pr, B2, Bv, W, Sij);
    // Sbar^{ij} = sqrt(gamma) gamma^{ik} gamma^{jl} S_kl
    double T[3][3], Su[6];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
      for (int ll = 0; ll < 3; ++ll)
        T[ii][ll] = gu[sym(ii, 0)] * Sij[sym(0, ll)] + gu[sym(ii, 1)] * Sij[sym(1, ll)] + gu[sym(ii, 2)] * Sij[sym(2, ll)];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
      for (int jj = ii; jj < 3; ++jj)
        Su[sym(ii, jj)] = sqrtg * (T[ii][0] * gu[sym(0, jj)] + T[ii][1] * gu[sym(1, jj)] + T[ii][2] * gu[sym(2, jj)]);
    const double trS = sqrtg * (T[0][0] + T[1][1] + T[2][2]);
    double Sup[3];
    sym_mv(gu, Sbar, Sup);
    const double Kf = Kh + 2.0 * Th;

    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) s += (c == 1 || c == 2 || c == 4 ? 2.0 : 1.0) * Su[c] * At[c];
    out[2] += alp * ichi * s + alp / 3.0 * trS * Kf - (Sup[0] * dalp[0] + Sup[1] * dalp[1] + Sup[2] * dalp[2]);
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) {
      double q = 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) q += (c == 1 || c == 2 || c == 4 ? 2.0 : 1.0) * Su[c] * dg[ii][c];
      out[3 + ii] += 0.5 * alp * ichi * (q - trS * dchi[ii]) +
                     (Sbar[0] * db[ii][0] + Sbar[1] * db[ii][1] + Sbar[2] * db[ii][2]) - (taubar + Dbar) * dalp[ii];
    }
    const double cb2 = a.par.c_b * a.par.c_b;
    double tmp[3], gtu_t[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) tmp[c] = -0.5 * alp * dchi[c] + chi / cb2 * dalp[c];
    sym_mv(gtu, tmp, gtu_t);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double Zc = 0.5 * chi * (Gh[c] - Gt[c]);
      out[6 + c] += phibar * (-alp * (chi * Gh[c] - 2.0 * Zc) + gtu_t[c]);
    }
    out[9] += -alp * cb2 * phibar * Kf + cb2 * (Bbar[0] * dalp[0] + Bbar[1] * dalp[1] + Bbar[2] * dalp[2]) -
              alp * a.par.kappa_b * phibar;
  }

  if (live) {
#pragma unroll
    for (int f = 0; f < 10; ++f) a.rhs[(int64_t)(22 + f) * sf + p] = out[f];
  }
  return live ? vmax : 0.0;
}

__global__ void __launch_bounds__(256) k_mhd_point(MhdPointArgs a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nx + 2 * g.ng || j >= g.ny + 2 * g.ng) return;
  mhd_point_at(a, a.par, a.eos, i, j, k);
}

// persistent: each XCD takes a contiguous range of the 64x4 tiles in the
// strip order and its blocks stride through it; the speed maximum is kept per
// thread and reduced once per block
__global__ void __launch_bounds__(256) k_mhd_update(MhdUpdArgs a) {
  const Geom& g = a.g;
  const TileXYZ t = tile_of_block(a.nbx, a.nby, a.nbz, a.strip);
  const int i = t.bx * 64 + threadIdx.x;
  const int j = t.by * 4 + threadIdx.y;
  const int k = t.bz < 0 ? 0 : t.bz;
  const bool live = (t.bx >= 0 && i < g.nx && j < g.ny);
  const double vmax = mhd_update_at(a, i, j, k, live);
  if (a.max_speed) block_max_to(a.max_speed, vmax);
}

__global__ void __launch_bounds__(256) k_mhd_point_lv(LevelArgs L) {
  for_each_level_point(L, kRegionPadded, [&](const BoxDev& B, int i, int j, int k, bool live) {
    if (!live) return;
    MhdPointArgs a;  // par and eos stay in the kernel arguments
    a.g = B.g;
    a.U = L.src ? B.Us : B.U;
    a.P = B.P;
    a.W = B.ws;
    mhd_point_at(a, L.par, L.eos, i, j, k);
  });
}

template <bool IMEX>
__global__ void __launch_bounds__(256) k_mhd_update_lv(LevelArgs L) {
  double vmax = 0.0;
  for_each_level_point(L, kRegionInterior, [&](const BoxDev& B, int i, int j, int k, bool live) {
    const MhdUpdArgs a{B.g, 0, 0, 0, 0, L.par, L.src ? B.Us : B.U, B.P, B.ws, level_rhs<IMEX>(B, L), L.max_speed};
    vmax = fmax(vmax, mhd_update_at(a, i, j, k, live));
  });
  if (L.max_speed) block_max_to(L.max_speed, vmax);
}

int launch_mhd_level(const LevelArgs& L, int grid_pad, int grid_int, int block, hipStream_t s) {
  MHD_LAUNCH(KID_MHD_POINT, k_mhd_point_lv, dim3(grid_pad), dim3(block), 0, s, L);
  if (L.slot >= 0)
    MHD_LAUNCH(KID_MHD_UPDATE, k_mhd_update_lv<true>, dim3(grid_int), dim3(block), 0, s, L);
  else
    MHD_LAUNCH(KID_MHD_UPDATE, k_mhd_update_lv<false>, dim3(grid_int), dim3(block), 0, s, L);
  return (int)hipGetLastError();
}

int launch_mhd(const Geom& g, const mhd_params_t& par, const mhd_eos_t& eos, const double* U, const double* P,
               double* ws, double* rhs, double* max_speed, int strip, hipStream_t s) {
  MhdPointArgs pa{g, par, eos, U, P, ws};
  dim3 blk(64, 4, 1);
  const int Nx = g.nx + 2 * g.ng, Ny = g.ny + 2 * g.ng, Nz = g.nz + 2 * g.ng;
  MHD_LAUNCH(KID_MHD_POINT, k_mhd_point, dim3((Nx + 63) / 64, (Ny + 3) / 4, Nz), blk, 0, s, pa);
  const int nbx = (g.nx + 63) / 64, nby = (g.ny + 3) / 4, nbz = g.nz;
  MhdUpdArgs ua{g, nbx, nby, nbz, strip, par, U, P, ws, rhs, reinterpret_cast<unsigned long long*>(max_speed)};
  const int nblk = nbx * nby * nbz;
  MHD_LAUNCH(KID_MHD_UPDATE, k_mhd_update, dim3(8 * ((nblk + 7) / 8), 1, 1), blk, 0, s, ua);
  return (int)hipGetLastError();
}

}  // namespace mhd
