// Device routines of the conserved-to-primitive recovery (App. D) shared by
// the bracketed kernel (c2p.hip) and the learned-guess kernel (learned.hip).
//
// The root functions are templated on the scalar type so that the same code
// gives f(mu) in double for Brent's method and (f, f') through forward-mode
// dual numbers for the Newton polish of the learned path.
//
// Reading of the error policy: the checks of App. D are applied to the
// unclamped rho = D/W and eps at the root (the clamps inside f only keep the
// EoS evaluation in range during the iteration); corrected points get their
// conserved variables rebuilt from the corrected primitives.
//
// The bracketed path is evaluated in a fixed order of plain IEEE operations
// (no FMA contraction, the divisions of the formulas kept as divisions), so
// Brent's iterates -- and with them mu, the primitives and the flags -- are
// reproducible bit for bit by any FP64 implementation of the same steps.  The
// right-hand side downstream cancels its fluxes by 5-6 digits, which would
// otherwise turn a last-ulp difference of the root into a visible one.
#pragma once

#include "dev_common.hpp"

namespace mhd {

#define C2P_CORRECTED (MHD_FLAG_ATMO | MHD_FLAG_EPS_LO | MHD_FLAG_EPS_HI | MHD_FLAG_VEL_LIMIT | MHD_FLAG_YE_RESET)
#define C2P_MAXIT 200

// ------------------------------------------------------------------ dual numbers

struct Dual {
  double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
__device__ __forceinline__ Dual operator/(double a, Dual b) {
  const double q = a / b.v;
  return {q, -q * b.d / b.v};
}
__device__ __forceinline__ Dual dsqrt(Dual a) {
  const double s = sqrt(a.v);
  return {s, 0.5 * a.d / s};
}
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }
__device__ __forceinline__ double val(double a) { return a; }
__device__ __forceinline__ double val(Dual a) { return a.v; }
__device__ __forceinline__ Dual dmin(Dual a, Dual b) { return a.v <= b.v ? a : b; }
__device__ __forceinline__ Dual dmax(Dual a, Dual b) { return a.v >= b.v ? a : b; }
__device__ __forceinline__ Dual dmin(Dual a, double b) { return a.v <= b ? a : Dual{b, 0.0}; }
__device__ __forceinline__ Dual dmax(Dual a, double b) { return a.v >= b ? a : Dual{b, 0.0}; }
__device__ __forceinline__ double dmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ double dmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ double dpow(double a, double e) { return pow(a, e); }
__device__ __forceinline__ Dual dpow(Dual a, double e) {
  const double r = pow(a.v, e);
  return {r, e * r / a.v * a.d};
}

// cold part of the EoS for either scalar type: returns eps_cold, sets p_cold
template <class T>
__device__ __forceinline__ T eos_cold_t(const mhd_eos_t& e, T rho, T& pc) {
#pragma clang fp contract(off)
  const double r = val(rho);
  int i = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b)
    if (b < e.npieces - 1 && r >= e.rho_b[b]) i = b + 1;
  const double K = e.K[i], G = e.Gamma[i];
  if (K == 0.0) {
    pc = rho * 0.0;
    return rho * 0.0 + e.a[i];
  }
  pc = K * dpow(rho, G);
  return e.a[i] + K / (G - 1.0) * dpow(rho, G - 1.0);
}

// ------------------------------------------------------------------ per-point data

struct C2pPoint {
  double gd[6], gu[6], sqrtg, alpha;
  double cons[6];  // undensitized D, DYe, tau, S_x, S_y, S_z
  double B[3];     // undensitized B^i
};

struct C2pInv {  // quantities fixed during the iterations (App. D, step 1)
  double D, q, r2, B2, rB, B2rp2, v02, h0;
  double rup[3], cB[3];
};

struct C2pOut {
  double prim[8];
  double mup, mu;
  unsigned flags;
  int iters;
  double cons[6];  // rebuilt conserved variables of corrected points (undensitized)
};

__device__ __forceinline__ void load_point(const double* __restrict__ U, int64_t sf, int64_t p, C2pPoint& pt) {
#pragma clang fp contract(off)
  double gt[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) gt[c] = U[c * sf + p];
  MetricR m;
  metric_repro(gt, U[12 * sf + p], m);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    pt.gd[c] = m.gd[c];
    pt.gu[c] = m.gu[c];
  }
  pt.sqrtg = m.sqrtg;
  pt.alpha = U[18 * sf + p];
#pragma unroll
  for (int c = 0; c < 6; ++c) pt.cons[c] = U[(22 + c) * sf + p] / m.sqrtg;
#pragma unroll
  for (int c = 0; c < 3; ++c) pt.B[c] = U[(28 + c) * sf + p] / m.sqrtg;
}

// returns false when D is below the density threshold (atmosphere, no solve)
__device__ __forceinline__ bool c2p_setup(const mhd_eos_t& e, const C2pPoint& pt, C2pInv& c) {
#pragma clang fp contract(off)
  const double D = pt.cons[0];
  if (!(D >= e.rho_min)) return false;
  c.D = D;
  c.h0 = e.h0;
  c.q = pt.cons[2] / D;
  const double r[3] = {pt.cons[3] / D, pt.cons[4] / D, pt.cons[5] / D};
  const double sD = sqrt(D);
#pragma unroll
  for (int a = 0; a < 3; ++a) c.cB[a] = pt.B[a] / sD;
  sym_mv(pt.gu, r, c.rup);
  double cBd[3];
  sym_mv(pt.gd, c.cB, cBd);
  c.r2 = c.rup[0] * r[0] + c.rup[1] * r[1] + c.rup[2] * r[2];
  c.B2 = c.cB[0] * cBd[0] + c.cB[1] * cBd[1] + c.cB[2] * cBd[2];
  c.rB = r[0] * c.cB[0] + r[1] * c.cB[1] + r[2] * c.cB[2];
  c.B2rp2 = fmax(0.0, c.B2 * c.r2 - c.rB * c.rB);
  c.v02 = c.r2 / (c.h0 * c.h0 + c.r2);
  return true;
}

template <class T>
__device__ __forceinline__ T fa_t(const C2pInv& c, T mu) {
#pragma clang fp contract(off)
  const T x = 1.0 / (1.0 + mu * c.B2);
  const T rb2 = c.r2 * x * x + mu * x * (1.0 + x) * c.rB * c.rB;
  return mu * dsqrt(c.h0 * c.h0 + rb2) - 1.0;
}

template <class T>
__device__ __forceinline__ T f_t(const mhd_eos_t& e, const C2pInv& c, T mu) {
#pragma clang fp contract(off)
  const T x = 1.0 / (1.0 + mu * c.B2);
  const T rb2 = c.r2 * x * x + mu * x * (1.0 + x) * c.rB * c.rB;
  const T qb = c.q - 0.5 * c.B2 - 0.5 * mu * mu * x * x * c.B2rp2;
  const T v2 = dmin(mu * mu * rb2, c.v02);
  const T W = 1.0 / dsqrt(1.0 - v2);
  const T rho = dmax(dmin(c.D / W, e.rho_max), e.rho_min);
  T pc;
  const T ec = eos_cold_t(e, rho, pc);
  T eps = W * (qb - mu * rb2) + v2 * W * W / (1.0 + W);
  eps = dmax(dmin(eps, e.eps_max), ec);
  const T pr = pc + (e.Gamma_th - 1.0) * rho * (eps - ec);
  const T ah = pr / (rho * (1.0 + eps));
  const T nuA = (1.0 + ah) * (1.0 + eps) / W;
  const T nuB = (1.0 + ah) * (1.0 + qb - mu * rb2);
  return mu - 1.0 / (dmax(nuA, nuB) + mu * rb2);
}

struct FaFn {
  const C2pInv& c;
  __device__ double operator()(double mu) const { return fa_t<double>(c, mu); }
};
struct FFn {
  const mhd_eos_t& e;
  const C2pInv& c;
  __device__ double operator()(double mu) const { return f_t<double>(e, c, mu); }
};

// Brent's method on [lo, hi] with f(lo) < 0 <= f(hi).  b is the current
// estimate, c the contrapoint (f(b) f(c) <= 0), a the previous estimate.
template <class Fn>
__device__ double brent_root(const Fn& f, double lo, double hi, double flo, double fhi, int& nit, bool& ok) {
#pragma clang fp contract(off)
  double a = lo, fa = flo, b = hi, fb = fhi;
  double c = a, fc = fa, step = b - a, prev = step;
  ok = true;
  for (int it = 0; it < C2P_MAXIT; ++it) {
    if ((fb > 0.0 && fc > 0.0) || (fb < 0.0 && fc < 0.0)) {
      c = a;
      fc = fa;
      step = prev = b - a;
    }
    if (fabs(fc) < fabs(fb)) {
      a = b;
      b = c;
      c = a;
      fa = fb;
      fb = fc;
      fc = fa;
    }
    const double tol = 2.0 * 2.220446049250313e-16 * fabs(b);
    const double half = 0.5 * (c - b);
    if (fabs(half) <= tol || fb == 0.0) {
      nit = it;
      return b;
    }
    bool bisect = true;
    if (fabs(prev) >= tol && fabs(fa) > fabs(fb)) {
      double pn, qd;
      const double s = fb / fa;
      if (a == c) {
        pn = 2.0 * half * s;
        qd = 1.0 - s;
      } else {
        const double qa = fa / fc, rb = fb / fc;
        pn = s * (2.0 * half * qa * (qa - rb) - (b - a) * (rb - 1.0));
        qd = (qa - 1.0) * (rb - 1.0) * (s - 1.0);
      }
      if (pn > 0.0) qd = -qd;
      else pn = -pn;
      if (2.0 * pn < 3.0 * half * qd - fabs(tol * qd) && pn < fabs(0.5 * prev * qd)) {
        prev = step;
        step = pn / qd;
        bisect = false;
      }
    }
    if (bisect) {
      step = half;
      prev = half;
    }
    a = b;
    fa = fb;
    b += (fabs(step) > tol) ? step : (half > 0.0 ? tol : -tol);
    fb = f(b);
  }
  nit = C2P_MAXIT;
  ok = false;
  return b;
}

__device__ __forceinline__ void prim_to_cons(const double gd[6], double rho, double eps, double pr, const double v[3],
                                             double ye, const double B[3], double cons[6], double& W) {
#pragma clang fp contract(off)
  double vd[3], Bd[3];
  sym_mv(gd, v, vd);
  sym_mv(gd, B, Bd);
  const double v2 = v[0] * vd[0] + v[1] * vd[1] + v[2] * vd[2];
  W = 1.0 / sqrt(1.0 - v2);
  const double B2 = B[0] * Bd[0] + B[1] * Bd[1] + B[2] * Bd[2];
  const double Bv = B[0] * vd[0] + B[1] * vd[1] + B[2] * vd[2];
  const double hW2 = (rho * (1.0 + eps) + pr) * W * W;
  cons[0] = rho * W;
  cons[1] = rho * W * ye;
  cons[2] = hW2 - pr + B2 - 0.5 * (Bv * Bv + B2 / (W * W)) - cons[0];
#pragma unroll
  for (int a = 0; a < 3; ++a) cons[3 + a] = (hW2 + B2) * vd[a] - Bv * Bd[a];
}

__device__ __forceinline__ void atmosphere_prims(const mhd_eos_t& e, double prim[8]) {
  const Cold c = eos_cold(e, e.rho_atm);
  prim[0] = e.rho_atm;
  prim[1] = c.e;
  prim[2] = c.p;
  prim[3] = prim[4] = prim[5] = 0.0;
  prim[6] = 1.0;
  prim[7] = e.ye_atm;
}

// primitives at the root mu, error policy, rebuilt conserved variables
__device__ __forceinline__ void c2p_finish(const mhd_eos_t& e, const C2pPoint& pt, const C2pInv& c, double mu,
                                           C2pOut& o) {
#pragma clang fp contract(off)
  const double x = 1.0 / (1.0 + mu * c.B2);
  const double rb2 = c.r2 * x * x + mu * x * (1.0 + x) * c.rB * c.rB;
  const double qb = c.q - 0.5 * c.B2 - 0.5 * mu * mu * x * x * c.B2rp2;
  const double v2 = fmin(mu * mu * rb2, c.v02);
  double W = 1.0 / sqrt(1.0 - v2);
  double rho = c.D / W;
  double eps = W * (qb - mu * rb2) + v2 * W * W / (1.0 + W);
  double v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) v[a] = mu * x * (c.rup[a] + mu * c.rB * c.cB[a]);
  double ye = pt.cons[1] / pt.cons[0];
  unsigned fl = o.flags;
  const bool low = (rho < e.rho_low) || (pt.alpha < e.alpha_bh);
  if (rho < e.rho_min) {
    atmosphere_prims(e, o.prim);
    fl |= MHD_FLAG_ATMO;
  } else {
    if (rho > e.rho_max) {
      fl |= MHD_FLAG_FATAL;
      rho = e.rho_max;
    }
    if (W > e.W_max) {
      if (low) {
        double vd[3];
        sym_mv(pt.gd, v, vd);
        const double vv = v[0] * vd[0] + v[1] * vd[1] + v[2] * vd[2];
        const double sc = sqrt((1.0 - 1.0 / (e.W_max * e.W_max)) / vv);
#pragma unroll
        for (int a = 0; a < 3; ++a) v[a] *= sc;
        W = e.W_max;
        rho = c.D / W;
        fl |= MHD_FLAG_VEL_LIMIT;
      } else {
        fl |= MHD_FLAG_FATAL;
      }
    }
    const Cold cold = eos_cold(e, rho);
    if (eps < cold.e) {
      eps = cold.e;
      fl |= MHD_FLAG_EPS_LO;
    } else if (eps > e.eps_max) {
      eps = e.eps_max;
      fl |= low ? MHD_FLAG_EPS_HI : MHD_FLAG_FATAL;
    }
    if (ye < e.ye_min || ye > e.ye_max) {
      if (low) {
        ye = e.ye_atm;
        fl |= MHD_FLAG_YE_RESET;
      } else {
        fl |= MHD_FLAG_FATAL;
      }
    }
    o.prim[0] = rho;
    o.prim[1] = eps;
    o.prim[2] = cold.p + (e.Gamma_th - 1.0) * rho * (eps - cold.e);
    o.prim[3] = v[0];
    o.prim[4] = v[1];
    o.prim[5] = v[2];
    o.prim[6] = W;
    o.prim[7] = ye;
  }
  o.flags = fl;
  if (fl & C2P_CORRECTED) {
    double Wn;
    const double vv[3] = {o.prim[3], o.prim[4], o.prim[5]};
    prim_to_cons(pt.gd, o.prim[0], o.prim[1], o.prim[2], vv, o.prim[7], pt.B, o.cons, Wn);
  }
}

__device__ __forceinline__ void c2p_plain(const mhd_eos_t& e, const C2pPoint& pt, C2pOut& o) {
  o.flags = 0;
  o.iters = 0;
  o.mup = o.mu = 0.0;
  C2pInv c;
  if (!c2p_setup(e, pt, c)) {
    atmosphere_prims(e, o.prim);
    o.flags = MHD_FLAG_ATMO;
    double Wn;
    const double z[3] = {0.0, 0.0, 0.0};
    prim_to_cons(pt.gd, o.prim[0], o.prim[1], o.prim[2], z, o.prim[7], pt.B, o.cons, Wn);
    return;
  }
  int it1 = 0, it2 = 0;
  bool ok1 = true, ok2 = true;
  const double hi = 1.0 / c.h0;
  const double fhi = fa_t<double>(c, hi);
  const double mup = (fhi <= 0.0) ? hi : brent_root(FaFn{c}, 0.0, hi, -1.0, fhi, it1, ok1);
  const FFn f{e, c};
  const double f0 = f(0.0), f1 = f(mup);
  const double mu = (f1 <= 0.0) ? mup : brent_root(f, 0.0, mup, f0, f1, it2, ok2);
  o.mup = mup;
  o.mu = mu;
  o.iters = it1 + it2 + 3;  // root-function evaluations, the three bracket ends included
  if (!(ok1 && ok2)) o.flags |= MHD_FLAG_NOT_CONVERGED;
  c2p_finish(e, pt, c, mu, o);
}

__device__ __forceinline__ void store_point(double* __restrict__ U, double* __restrict__ P, uint8_t* __restrict__ flags,
                                            double* __restrict__ mu, int64_t sf, int64_t p, const C2pPoint& pt,
                                            const C2pOut& o) {
#pragma unroll
  for (int c = 0; c < 8; ++c) P[c * sf + p] = o.prim[c];
  if (flags) flags[p] = (uint8_t)o.flags;
  if (mu) {
    mu[p] = o.mup;
    mu[sf + p] = o.mu;
  }
  if (o.flags & C2P_CORRECTED) {
#pragma unroll
    for (int c = 0; c < 6; ++c) U[(22 + c) * sf + p] = pt.sqrtg * o.cons[c];
  }
}

// The EoS copied to LDS by the block (every thread calls this): its piece
// tables are read with lane-dependent indices, which kernel arguments would
// serve through a private copy per lane.
__device__ __forceinline__ const mhd_eos_t& stage_eos(const mhd_eos_t& e, mhd_eos_t& lds) {
  if (threadIdx.x + threadIdx.y * blockDim.x == 0) lds = e;
  __syncthreads();
  return lds;
}

// Block-wide sums of the statistics, then at most one atomic per counter per
// block: atomics on one address are serialised in L2, so one per wavefront
// would dominate the cost of a cheap launch.  Every thread of the block (at
// most 256 threads) must call this, once, after its last point.
__device__ __forceinline__ void block_add_stats(int64_t* stats, int64_t nfatal, int64_t ncorr, int64_t nfb,
                                                int64_t nit) {
  __shared__ int64_t red[4][4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    nfatal += __shfl_xor(nfatal, off, 64);
    ncorr += __shfl_xor(ncorr, off, 64);
    nfb += __shfl_xor(nfb, off, 64);
    nit += __shfl_xor(nit, off, 64);
  }
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int w = tid / 64;
  if (tid % 64 == 0) {
    red[w][0] = nfatal;
    red[w][1] = ncorr;
    red[w][2] = nfb;
    red[w][3] = nit;
  }
  __syncthreads();
  if (tid == 0) {
    const int nw = (int)((blockDim.x * blockDim.y + 63) / 64);
    int64_t sum[4] = {0, 0, 0, 0};
    for (int v = 0; v < nw; ++v)
#pragma unroll
      for (int c = 0; c < 4; ++c) sum[c] += red[v][c];
    if (sum[0]) atomicAdd((unsigned long long*)&stats[MHD_STAT_FATAL], (unsigned long long)sum[0]);
    if (sum[1]) atomicAdd((unsigned long long*)&stats[MHD_STAT_CORRECTED], (unsigned long long)sum[1]);
    if (sum[2]) atomicAdd((unsigned long long*)&stats[MHD_STAT_FALLBACK], (unsigned long long)sum[2]);
    if (sum[3]) atomicAdd((unsigned long long*)&stats[MHD_STAT_ITERATIONS], (unsigned long long)sum[3]);
  }
}

}  // namespace mhd
