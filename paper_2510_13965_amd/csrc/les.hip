// Gradient sub-grid-scale (LES) term of the induction equation (App. A).
//
// The flux of Bbar^i along k gains -alpha G_B^{ki}, G_B^{ki} = -C_M xi sqrt(gamma)
// H_M^{ki}, xi = gamma^{1/3} Delta^2/24, Delta^2 = (dx dy dz)^{2/3}, with
//   H_M^{ki} = B^i H_v^k - B^k H_v^i + 2 (grad B^i . grad v^k - grad B^k . grad v^i),
// grad a . grad b = gamma^{jl} d_j a d_l b.  H_v is the velocity part of the
// primitives' second-order response to filtering the conserved fields, the
// quantity the gradient model expands: C_P H_P = -C_PP(grad P, grad P) for the
// conserved fields C = (D, S_i, tau) of Sec. 2.2 as functions of
// P = (rho, eps, v^i) at the point's metric (B^i enters C_PP through its
// gradients).  C_PP(grad P, grad P) is the sum of second directional
// derivatives along the columns of the Cholesky factor of gamma^{jl}, each by
// second-order Taylor arithmetic (the EoS differentiated with it); C_P by
// first-order directions; the 5x5 system by Gaussian elimination with partial
// pivoting.
//
//   k_les_b     B^i = Bbar^i / sqrt(gamma) at every padded point -> workspace
//   k_les_flux  alpha G_B^{ki} (xy, xz, yz) at the interior points and one
//               beyond: 4th-order centred first derivatives of rho, eps, v^i
//               (from P) and B^i (two points on each side)
//   k_les_div   rhs[28 + i] += d_k (alpha G_B^{ki}) at the interior points,
//               2nd-order centred differences (so three ghost points suffice)
#include "dev_common.hpp"
#include "prof.hpp"

namespace mhd {

namespace {

struct T2 {  // a0 + a1 t + a2 t^2
  double a0, a1, a2;
};
__device__ __forceinline__ T2 t2c(double c) { return {c, 0.0, 0.0}; }
__device__ __forceinline__ T2 operator+(T2 a, T2 b) { return {a.a0 + b.a0, a.a1 + b.a1, a.a2 + b.a2}; }
__device__ __forceinline__ T2 operator-(T2 a, T2 b) { return {a.a0 - b.a0, a.a1 - b.a1, a.a2 - b.a2}; }
__device__ __forceinline__ T2 operator*(T2 a, T2 b) {
  return {a.a0 * b.a0, a.a0 * b.a1 + a.a1 * b.a0, a.a0 * b.a2 + a.a1 * b.a1 + a.a2 * b.a0};
}
__device__ __forceinline__ T2 operator*(double s, T2 a) { return {s * a.a0, s * a.a1, s * a.a2}; }
__device__ __forceinline__ T2 operator/(T2 a, T2 b) {
  const double q0 = a.a0 / b.a0;
  const double q1 = (a.a1 - q0 * b.a1) / b.a0;
  return {q0, q1, (a.a2 - q0 * b.a2 - q1 * b.a1) / b.a0};
}
__device__ __forceinline__ T2 t2sqrt(T2 a) {
  const double s = sqrt(a.a0);
  const double s1 = a.a1 / (2.0 * s);
  return {s, s1, (a.a2 - s1 * s1) / (2.0 * s)};
}
__device__ __forceinline__ T2 t2pow(T2 a, double e) {  // a0 > 0
  const double p = pow(a.a0, e);
  return {p, e * p / a.a0 * a.a1, e * p / a.a0 * a.a2 + 0.5 * e * (e - 1.0) * p / (a.a0 * a.a0) * a.a1 * a.a1};
}

// pressure of the hybrid EoS with the piece chosen by rho's value
__device__ __forceinline__ T2 t2_press(const mhd_eos_t& e, T2 rho, T2 eps) {
  int i = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b)
    if (b < e.npieces - 1 && rho.a0 >= e.rho_b[b]) i = b + 1;
  T2 pc = t2c(0.0), ec = t2c(e.a[i]);
  if (e.K[i] != 0.0) {
    pc = e.K[i] * t2pow(rho, e.Gamma[i]);
    ec = t2c(e.a[i]) + (e.K[i] / (e.Gamma[i] - 1.0)) * t2pow(rho, e.Gamma[i] - 1.0);
  }
  return pc + (e.Gamma_th - 1.0) * (rho * (eps - ec));
}

// D, S_i, tau (undensitized) at the metric gd
__device__ __forceinline__ void t2_cons(const mhd_eos_t& e, const double gd[6], T2 rho, T2 eps, const T2 v[3],
                                        const T2 B[3], T2 C[5]) {
  T2 vd[3], Bd[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    vd[i] = t2c(0.0);
    Bd[i] = t2c(0.0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      vd[i] = vd[i] + gd[sym(i, j)] * v[j];
      Bd[i] = Bd[i] + gd[sym(i, j)] * B[j];
    }
  }
  T2 v2 = t2c(0.0), B2 = t2c(0.0), vB = t2c(0.0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    v2 = v2 + v[i] * vd[i];
    B2 = B2 + B[i] * Bd[i];
    vB = vB + B[i] * vd[i];
  }
  const T2 W = t2c(1.0) / t2sqrt(t2c(1.0) - v2);
  const T2 W2 = W * W;
  const T2 p = t2_press(e, rho, eps);
  const T2 hW2 = (rho * (t2c(1.0) + eps) + p) * W2;
  C[0] = rho * W;
#pragma unroll
  for (int i = 0; i < 3; ++i) C[1 + i] = (hW2 + B2) * vd[i] - vB * Bd[i];
  C[4] = hW2 - p + B2 - 0.5 * (vB * vB + B2 / W2) - C[0];
}

__device__ __forceinline__ bool solve5(double A[5][5], double b[5], double x[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    int piv = k;
#pragma unroll
    for (int r = k + 1; r < 5; ++r)
      if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
    if (A[piv][k] == 0.0) return false;
    if (piv != k) {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const double t = A[k][c];
        A[k][c] = A[piv][c];
        A[piv][c] = t;
      }
      const double t = b[k];
      b[k] = b[piv];
      b[piv] = t;
    }
#pragma unroll
    for (int r = k + 1; r < 5; ++r) {
      const double f = A[r][k] / A[k][k];
#pragma unroll
      for (int c = k; c < 5; ++c) A[r][c] -= f * A[k][c];
      b[r] -= f * b[k];
    }
  }
#pragma unroll
  for (int r = 4; r >= 0; --r) {
    double t = b[r];
#pragma unroll
    for (int c = r + 1; c < 5; ++c) t -= A[r][c] * x[c];
    x[r] = t / A[r][r];
  }
  return true;
}

__device__ __forceinline__ double d1c4(const double* __restrict__ f, int64_t p, int64_t st, double h) {
  return (8.0 * (f[p + st] - f[p - st]) - (f[p + 2 * st] - f[p - 2 * st])) / (12.0 * h);
}

struct LesArgs {
  Geom g;
  mhd_eos_t eos;
  const double* __restrict__ U;
  const double* __restrict__ P;
  double* __restrict__ Bw;  // 3 fields: B^i
  double* __restrict__ AG;  // 3 fields: alpha G_B^{xy, xz, yz}
  double* __restrict__ rhs;
  double cm, D2;  // C_M, Delta^2
};

__global__ void __launch_bounds__(256) k_les_b(LesArgs a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nx + 2 * g.ng || j >= g.ny + 2 * g.ng) return;
  const int64_t p = g.at(i, j, k), sf = g.sf;
  double gt[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) gt[c] = a.U[c * sf + p];
  MetricR m;
  metric_repro(gt, a.U[12 * sf + p], m);
#pragma unroll
  for (int c = 0; c < 3; ++c) a.Bw[c * sf + p] = a.U[(28 + c) * sf + p] / m.sqrtg;
}

// padded indices (ng - 1 .. n + ng inclusive on every axis)
__device__ __forceinline__ void les_flux_at(const LesArgs& a, int i, int j, int k) {
  const Geom& g = a.g;
  const int64_t sf = g.sf, p = g.at(i, j, k);
  double gt[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) gt[c] = a.U[c * sf + p];
  MetricR m;
  metric_repro(gt, a.U[12 * sf + p], m);
  // primitives (rho, eps, v^x, v^y, v^z, B^x, B^y, B^z) and their coordinate derivatives
  const int src[8] = {0, 1, 3, 4, 5, -1, -2, -3};
  double Pv[8], dP[3][8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double* f = src[q] >= 0 ? a.P + (int64_t)src[q] * sf : a.Bw + (int64_t)(-src[q] - 1) * sf;
    Pv[q] = f[p];
#pragma unroll
    for (int d = 0; d < 3; ++d) dP[d][q] = d1c4(f, p, g.stride(d), g.h[d]);
  }
  // Cholesky factor of gamma^{jl}, and derivatives along its columns
  double L[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double s = m.gu[sym(c, c)];
#pragma unroll
    for (int b = 0; b < c; ++b) s -= L[c][b] * L[c][b];
    L[c][c] = sqrt(s);
#pragma unroll
    for (int r = c + 1; r < 3; ++r) {
      double t = m.gu[sym(r, c)];
#pragma unroll
      for (int b = 0; b < c; ++b) t -= L[r][b] * L[c][b];
      L[r][c] = t / L[c][c];
    }
  }
  double gd[3][8];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int q = 0; q < 8; ++q) gd[c][q] = L[0][c] * dP[0][q] + L[1][c] * dP[1][q] + L[2][c] * dP[2][q];
  double rhs[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  T2 C[5], v[3], B[3];
#pragma unroll 1
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      v[q] = {Pv[2 + q], gd[c][2 + q], 0.0};
      B[q] = {Pv[5 + q], gd[c][5 + q], 0.0};
    }
    t2_cons(a.eos, m.gd, {Pv[0], gd[c][0], 0.0}, {Pv[1], gd[c][1], 0.0}, v, B, C);
#pragma unroll
    for (int r = 0; r < 5; ++r) rhs[r] += 2.0 * C[r].a2;
  }
  double J[5][5];
#pragma unroll 1
  for (int u = 0; u < 5; ++u) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      v[q] = {Pv[2 + q], u == 2 + q ? 1.0 : 0.0, 0.0};
      B[q] = t2c(Pv[5 + q]);
    }
    t2_cons(a.eos, m.gd, {Pv[0], u == 0 ? 1.0 : 0.0, 0.0}, {Pv[1], u == 1 ? 1.0 : 0.0, 0.0}, v, B, C);
#pragma unroll
    for (int r = 0; r < 5; ++r) J[r][u] = C[r].a1;
  }
  double x[5];
  double Hv[3] = {0.0, 0.0, 0.0};
  if (solve5(J, rhs, x)) {
    Hv[0] = -x[2];
    Hv[1] = -x[3];
    Hv[2] = -x[4];
  }
  const double xi = cbrt(m.sqrtg * m.sqrtg) * a.D2 / 24.0;
  const double fac = a.U[18 * sf + p] * (-a.cm * xi * m.sqrtg);
  const int KI[3][2] = {{0, 1}, {0, 2}, {1, 2}};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int kk = KI[c][0], ii = KI[c][1];
    double bv = 0.0, vb = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      bv += gd[d][5 + ii] * gd[d][2 + kk];
      vb += gd[d][5 + kk] * gd[d][2 + ii];
    }
    const double HM = Pv[5 + ii] * Hv[kk] - Pv[5 + kk] * Hv[ii] + 2.0 * (bv - vb);
    a.AG[c * sf + p] = fac * HM;
  }
}

__global__ void __launch_bounds__(256) k_les_flux(LesArgs a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nx + 2 || j >= g.ny + 2) return;
  les_flux_at(a, i + g.ng - 1, j + g.ng - 1, k + g.ng - 1);
}

__global__ void __launch_bounds__(256) k_les_div(LesArgs a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.nx || j >= g.ny) return;
  const int64_t sf = g.sf, p = g.at(i + g.ng, j + g.ng, k + g.ng);
  const int64_t sx = 1, sy = g.sy, sz = g.sz;
  const double* gxy = a.AG;
  const double* gxz = a.AG + sf;
  const double* gyz = a.AG + 2 * sf;
  const double dx2 = 2.0 * g.h[0], dy2 = 2.0 * g.h[1], dz2 = 2.0 * g.h[2];
  // G^{ki} antisymmetric: rhs of Bbar^i gains sum_k d_k (alpha G^{ki})
  a.rhs[28 * sf + p] += -(gxy[p + sy] - gxy[p - sy]) / dy2 - (gxz[p + sz] - gxz[p - sz]) / dz2;
  a.rhs[29 * sf + p] += (gxy[p + sx] - gxy[p - sx]) / dx2 - (gyz[p + sz] - gyz[p - sz]) / dz2;
  a.rhs[30 * sf + p] += (gxz[p + sx] - gxz[p - sx]) / dx2 + (gyz[p + sy] - gyz[p - sy]) / dy2;
}

}  // namespace

int les_workspace_fields() { return 6; }

int launch_les(const Geom& g, const mhd_eos_t& eos, double cm, const double* U, const double* P, double* ws,
               double* rhs, hipStream_t s) {
  LesArgs a{g, eos, U, P, ws, ws + 3 * g.sf, rhs, cm, cbrt(g.h[0] * g.h[1] * g.h[2]) * cbrt(g.h[0] * g.h[1] * g.h[2])};
  const int Nx = g.nx + 2 * g.ng, Ny = g.ny + 2 * g.ng, Nz = g.nz + 2 * g.ng;
  MHD_LAUNCH(KID_LES, k_les_b, dim3((Nx + 63) / 64, (Ny + 3) / 4, Nz), dim3(64, 4, 1), 0, s, a);
  MHD_LAUNCH(KID_LES, k_les_flux, dim3((g.nx + 2 + 63) / 64, (g.ny + 2 + 3) / 4, g.nz + 2), dim3(64, 4, 1), 0, s, a);
  MHD_LAUNCH(KID_LES, k_les_div, dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz), dim3(64, 4, 1), 0, s, a);
  return (int)hipGetLastError();
}

}  // namespace mhd
