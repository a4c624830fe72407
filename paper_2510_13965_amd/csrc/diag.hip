// Constraint monitors of the evolution (Sec. 2.1: the Z4 constraints
// Theta = 0, Z_i = 0 and the energy and momentum constraints they integrate;
// Sec. 5: the accuracy checks of the star tests, i.e. L2 norms of the energy
// and momentum residuals, the baryonic mass as the volume integral of the
// conserved density, Theta, Z, and the cleaning field against |B|).
//
// The residuals are the 3+1 constraints of the physical metric
// gamma_ij = gt_ij / chi with K_ij = (At_ij + gt_ij K / 3) / chi and the
// physical trace K = Khat + 2 Theta:
//   H   = R + K^2 - K_ij K^ij - 16 pi E,        E   = (taubar + Dbar) / sqrt(gamma)
//   M_i = D_j K^j_i - d_i K - 8 pi S_i,          S_i = Sbar_i / sqrt(gamma)
// and Z^i = chi (Ghat^i - Gt^i) / 2 with Gt^i = gt^ij gt^kl d_l gt_jk.  All
// derivatives come from the 4th-order centred operators applied to the
// evolved fields, products by the product rule.
//
// The Ricci scalar is evaluated as
//   R = gamma^ac gamma^bd (d_a d_b gamma_cd) - gamma^ab gamma^cd (d_a d_b gamma_cd)
//     + gamma^ij (d_k gamma^kl G_lij - d_j gamma^kl G_lik)
//     + gamma^ij (G^k_kl G^l_ij - G^k_jl G^l_ik),
// which is gamma^ij R_ij of the Christoffel form of the Ricci tensor with the
// second derivatives of the Christoffel symbols collected: one pass over the six
// derivative pairs (a, b) consumes each second derivative as it is formed, so
// no 81-entry Hessian is held in registers.
//
// One thread per interior point, loads straight from HBM through the buffer
// path of the stencil helpers (the monitors run once per output interval, not
// per stage).  The volume integrals are reduced per z plane by one block in a
// fixed order and the planes summed in order by one more block: the result is
// the same on every run.
#include "dev_common.hpp"
#include "prof.hpp"

namespace mhd {

#pragma clang fp contract(off)

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kNumSums = 7;

// index of the symmetric pair (i, j) in xx, xy, xz, yy, yz, zz
__device__ __forceinline__ constexpr int sy6(int i, int j) {
  return i == j ? (i == 0 ? 0 : (i == 1 ? 3 : 5)) : (i + j == 1 ? 1 : (i + j == 2 ? 2 : 4));
}

// inverse and determinant of a symmetric 3x3 matrix in sy6 storage
__device__ __forceinline__ double inv_sym3(const double a[6], double u[6]) {
  const double c00 = a[3] * a[5] - a[4] * a[4];
  const double c01 = a[2] * a[4] - a[1] * a[5];
  const double c02 = a[1] * a[4] - a[2] * a[3];
  const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  const double id = 1.0 / det;
  u[0] = c00 * id;
  u[1] = c01 * id;
  u[2] = c02 * id;
  u[3] = (a[0] * a[5] - a[2] * a[2]) * id;
  u[4] = (a[2] * a[1] - a[0] * a[4]) * id;
  u[5] = (a[0] * a[3] - a[1] * a[1]) * id;
  return det;
}

struct DiagArgs {
  Geom g;
  const double* __restrict__ U;
  double* __restrict__ C;
  double* __restrict__ sums;
};

}  // namespace

// block 64 x 4 over (x, y) of the interior, grid.z over z
__global__ void __launch_bounds__(256) k_constraints(DiagArgs a) {
  const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y * 4 + threadIdx.y, kz = blockIdx.z;
  const int nx = a.g.nx, ny = a.g.ny, ng = a.g.ng;
  if (i >= nx || j >= ny) return;
  const int64_t sf = a.g.sf;
  const int64_t st[3] = {1, a.g.sy, a.g.sz};
  const double i12[3] = {a.g.i12[0], a.g.i12[1], a.g.i12[2]};
  const int64_t p = a.g.at(i + ng, j + ng, kz + ng);
  const uint32_t voff = (uint32_t)(p * 8);
  const double* U = a.U;

  double gt[6], dgt[3][6], dchi[3];
#pragma unroll
  for (int c = 0; c < 6; ++c) gt[c] = U[c * sf + p];
  const double chi = U[12 * sf + p];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int c = 0; c < 6; ++c) dgt[d][c] = fd1(U + c * sf, st[d], voff, i12[d]);
    dchi[d] = fd1(U + 12 * sf, st[d], voff, i12[d]);
  }
  const double chi2 = chi * chi, chi3 = chi2 * chi;

  // physical metric, its inverse and first derivatives (quotient rule)
  double gd[6], gu[6], dg[3][6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    gd[c] = gt[c] / chi;
#pragma unroll
    for (int d = 0; d < 3; ++d) dg[d][c] = dgt[d][c] / chi - gt[c] * dchi[d] / chi2;
  }
  const double sqrtg = sqrt(inv_sym3(gd, gu));

  // Christoffels: c1[k][ij] = G_kij, c2[k][ij] = G^k_ij
  double c1[3][6], c2[3][6];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
      for (int jj = ii; jj < 3; ++jj)
        c1[k][sy6(ii, jj)] = 0.5 * (dg[ii][sy6(k, jj)] + dg[jj][sy6(k, ii)] - dg[k][sy6(ii, jj)]);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int c = 0; c < 6; ++c) c2[k][c] = gu[sy6(k, 0)] * c1[0][c] + gu[sy6(k, 1)] * c1[1][c] + gu[sy6(k, 2)] * c1[2][c];

  // first-derivative part of R
  double R = 0.0;
  {
    double cl[3], Gam[3], tr2[3];  // gamma^ij G_lij, gamma^ij G^l_ij, G^k_kl
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      double s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
          s1 += gu[sy6(ii, jj)] * c1[l][sy6(ii, jj)];
          s2 += gu[sy6(ii, jj)] * c2[l][sy6(ii, jj)];
        }
      cl[l] = s1;
      Gam[l] = s2;
      tr2[l] = c2[0][sy6(0, l)] + c2[1][sy6(1, l)] + c2[2][sy6(2, l)];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      // d_m gamma^{kl} = -gamma^{ka} gamma^{lb} d_m gamma_ab
      double dgu[6];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = k; l < 3; ++l) {
          double s = 0.0;
#pragma unroll
          for (int aa = 0; aa < 3; ++aa)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) s -= gu[sy6(k, aa)] * gu[sy6(l, bb)] * dg[m][sy6(aa, bb)];
          dgu[sy6(k, l)] = s;
        }
      // gamma^ij d_k gamma^kl G_lij with k = m
#pragma unroll
      for (int l = 0; l < 3; ++l) R += dgu[sy6(m, l)] * cl[l];
      // - gamma^ij d_j gamma^kl G_lik with j = m
#pragma unroll
      for (int ii = 0; ii < 3; ++ii)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int l = 0; l < 3; ++l) R -= gu[sy6(ii, m)] * dgu[sy6(k, l)] * c1[l][sy6(ii, k)];
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) R += tr2[l] * Gam[l];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int l = 0; l < 3; ++l) R -= gu[sy6(ii, jj)] * c2[k][sy6(jj, l)] * c2[l][sy6(ii, k)];
  }

  // second-derivative part: for each pair (a, b), the six d_a d_b gamma_cd
  // (quotient rule) weighted by gamma^ac gamma^bd - gamma^ab gamma^cd, summed
  // over both orders of (a, b) and of (c, d)
#pragma unroll
  for (int pa = 0; pa < 3; ++pa)
#pragma unroll
    for (int pb = pa; pb < 3; ++pb) {
      const double ddchi = pa == pb ? fd2(U + 12 * sf, st[pa], voff, a.g.i12s[pa])
                                    : fd11(U + 12 * sf, st[pa], st[pb], voff, i12[pa], i12[pb]);
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int dd = cc; dd < 3; ++dd) {
          const int c = sy6(cc, dd);
          const double ddgt = pa == pb ? fd2(U + c * sf, st[pa], voff, a.g.i12s[pa])
                                       : fd11(U + c * sf, st[pa], st[pb], voff, i12[pa], i12[pb]);
          const double ddg = ddgt / chi - (dgt[pa][c] * dchi[pb] + dgt[pb][c] * dchi[pa]) / chi2 -
                             gt[c] * ddchi / chi2 + 2.0 * gt[c] * dchi[pa] * dchi[pb] / chi3;
          double w;
          if (pa == pb)
            w = gu[sy6(pa, cc)] * gu[sy6(pa, dd)] - gu[sy6(pa, pa)] * gu[c];
          else
            w = gu[sy6(pa, cc)] * gu[sy6(pb, dd)] + gu[sy6(pb, cc)] * gu[sy6(pa, dd)] - 2.0 * gu[sy6(pa, pb)] * gu[c];
          R += (cc == dd ? w : 2.0 * w) * ddg;
        }
    }

  // extrinsic curvature
  const double Kt = U[13 * sf + p] + 2.0 * U[14 * sf + p];
  double num[6], Kdn[6], Kmix[3][3];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    num[c] = U[(6 + c) * sf + p] + gt[c] * Kt / 3.0;
    Kdn[c] = num[c] / chi;
  }
#pragma unroll
  for (int ii = 0; ii < 3; ++ii)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj)
      Kmix[ii][jj] = gu[sy6(ii, 0)] * Kdn[sy6(0, jj)] + gu[sy6(ii, 1)] * Kdn[sy6(1, jj)] +
                     gu[sy6(ii, 2)] * Kdn[sy6(2, jj)];
  double KK = 0.0;
#pragma unroll
  for (int ii = 0; ii < 3; ++ii)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) KK += Kmix[ii][jj] * Kmix[jj][ii];

  const double E = (U[24 * sf + p] + U[22 * sf + p]) / sqrtg;
  double* C = a.C;
  C[p] = R + Kt * Kt - KK - 16.0 * kPi * E;

  // momentum: gamma^jk d_k K_ji - gamma^jk G^l_kj K_li - gamma^jk G^l_ki K_jl - d_i K - 8 pi S_i
  double M[3] = {0.0, 0.0, 0.0}, dK[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dK[k] = fd1(U + 13 * sf, st[k], voff, i12[k]) + 2.0 * fd1(U + 14 * sf, st[k], voff, i12[k]);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double dAt = fd1(U + (6 + c) * sf, st[k], voff, i12[k]);
      const double dnum = dAt + dgt[k][c] * Kt / 3.0 + gt[c] * dK[k] / 3.0;
      const double dKc = dnum / chi - num[c] * dchi[k] / chi2;
      // component c = (cc, dd) serves M_dd (j = cc) and, off the diagonal, M_cc (j = dd)
      const int cc = c == 0 || c == 1 || c == 2 ? 0 : (c == 5 ? 2 : 1);
      const int dd = c == 0 ? 0 : (c == 1 || c == 3 ? 1 : 2);
      M[dd] += gu[sy6(cc, k)] * dKc;
      if (cc != dd) M[cc] += gu[sy6(dd, k)] * dKc;
    }
  }
  // contracted Christoffels gamma^jk G^l_jk (recomputed: a few FLOPs, fewer live registers)
#pragma unroll
  for (int ii = 0; ii < 3; ++ii) {
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      double gl = 0.0;
#pragma unroll
      for (int jj = 0; jj < 3; ++jj)
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) gl += gu[sy6(jj, kk)] * c2[l][sy6(jj, kk)];
      s += gl * Kdn[sy6(l, ii)];
#pragma unroll
      for (int k = 0; k < 3; ++k) s += c2[l][sy6(k, ii)] * Kmix[k][l];
    }
    C[(1 + ii) * sf + p] = M[ii] - s - dK[ii] - 8.0 * kPi * (U[(25 + ii) * sf + p] / sqrtg);
  }

  // Z^i = chi (Ghat^i - Gt^i) / 2, Z_i Z^i with the physical metric
  double gtu[6];
  inv_sym3(gt, gtu);
  double Zu[3];
#pragma unroll
  for (int ii = 0; ii < 3; ++ii) {
    double s = 0.0;
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) t += gtu[sy6(k, l)] * dgt[l][sy6(jj, k)];
      s += gtu[sy6(ii, jj)] * t;
    }
    Zu[ii] = 0.5 * chi * (U[(15 + ii) * sf + p] - s);
  }
  double Z2 = 0.0;
#pragma unroll
  for (int ii = 0; ii < 3; ++ii)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) Z2 += gd[sy6(ii, jj)] * Zu[ii] * Zu[jj];
  C[4 * sf + p] = Z2;
}

// one block per interior z plane: the plane's seven volume sums
__global__ void __launch_bounds__(256) k_constraint_planes(DiagArgs a) {
  __shared__ double red[kNumSums][256];
  const int nx = a.g.nx, ny = a.g.ny, ng = a.g.ng, kz = blockIdx.x;
  const int64_t sf = a.g.sf;
  const double* U = a.U;
  const double* C = a.C;
  double s[kNumSums] = {0, 0, 0, 0, 0, 0, 0};
  for (int e = threadIdx.x; e < nx * ny; e += 256) {
    const int i = e % nx, j = e / nx;
    const int64_t p = a.g.at(i + ng, j + ng, kz + ng);
    double gd[6], gu[6];
    const double chi = U[12 * sf + p];
#pragma unroll
    for (int c = 0; c < 6; ++c) gd[c] = U[c * sf + p] / chi;
    const double sg = sqrt(inv_sym3(gd, gu));
    const double H = C[p], M1 = C[sf + p], M2 = C[2 * sf + p], M3 = C[3 * sf + p];
    const double th = U[14 * sf + p], phi = U[31 * sf + p] / sg;
    double B[3], B2 = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) B[q] = U[(28 + q) * sf + p] / sg;
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int r = 0; r < 3; ++r) B2 += gd[sy6(q, r)] * B[q] * B[r];
    s[0] += H * H;
    s[1] += M1 * M1 + M2 * M2 + M3 * M3;
    s[2] += U[22 * sf + p];
    s[3] += th * th;
    s[4] += C[4 * sf + p];
    s[5] += phi * phi;
    s[6] += B2;
  }
#pragma unroll
  for (int q = 0; q < kNumSums; ++q) red[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int q = 0; q < kNumSums; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < kNumSums) {
    const double dV = a.g.h[0] * a.g.h[1] * a.g.h[2];
    a.sums[kNumSums + kNumSums * kz + threadIdx.x] = red[threadIdx.x][0] * dV;
  }
}

// totals: the planes in order
__global__ void __launch_bounds__(64) k_constraint_total(DiagArgs a) {
  const int q = threadIdx.x;
  if (q >= kNumSums) return;
  double s = 0.0;
  for (int k = 0; k < a.g.nz; ++k) s += a.sums[kNumSums + kNumSums * k + q];
  a.sums[q] = s;
}

int launch_constraints(const Geom& g, const double* U, double* C, double* sums, hipStream_t s) {
  DiagArgs a;
  a.g = g;
  a.U = U;
  a.C = C;
  a.sums = sums;
  MHD_LAUNCH(KID_CONSTRAINTS, k_constraints, dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz), dim3(64, 4, 1), 0, s, a);
  MHD_LAUNCH(KID_CONSTRAINT_PLANES, k_constraint_planes, dim3(g.nz), dim3(256), 0, s, a);
  MHD_LAUNCH(KID_CONSTRAINT_TOTAL, k_constraint_total, dim3(1), dim3(64), 0, s, a);
  return (int)hipGetLastError();
}

}  // namespace mhd
