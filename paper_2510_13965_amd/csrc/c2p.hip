// Conserved <-> primitive conversion on the device.
//
// prim -> cons: the definitions of Sec. 2.2 (restated in App. D).
// cons -> prim: App. D.  With q = tau/D, r_i = S_i/D, calB^i = B^i/sqrt(D) and
// chi(mu) = 1/(1 + mu calB^2), rbar^2(mu) = r^2 chi^2 + mu chi (1+chi) (r.calB)^2:
//   mu_+ = root of f_a(mu) = mu sqrt(h0^2 + rbar^2) - 1 on (0, 1/h0],
//   mu   = root of f(mu)   = mu - 1/(nuhat + mu rbar^2) on (0, mu_+],
// each bracketed and found with Brent's method (inverse quadratic
// interpolation / secant steps safeguarded by bisection) until the bracket is
// a few ulp wide; primitives from mu; then the error policy.
//
// Threads stride over the padded points.  Iteration counts differ from lane
// to lane, so the kernel is divergence bound; the learned-guess path in learned.hip
// replaces most of the Brent iterations with three Newton steps.
#include "c2p_dev.hpp"
#include "prof.hpp"

namespace mhd {

struct C2pArgs {
  Geom g;
  mhd_eos_t eos;
  double* __restrict__ U;
  double* __restrict__ P;
  uint8_t* __restrict__ flags;
  double* __restrict__ mu;
  int64_t* __restrict__ stats;
};

// padded indices; adds the point's statistics to the counters
__device__ __forceinline__ void con2prim_at(const C2pArgs& a, const mhd_eos_t& eos, int i, int j, int k,
                                            int64_t& nfatal, int64_t& ncorr, int64_t& nit) {
  const Geom& g = a.g;
  const int64_t p = g.at(i, j, k);
  C2pPoint pt;
  load_point(a.U, g.sf, p, pt);
  C2pOut o;
  c2p_plain(eos, pt, o);
  store_point(a.U, a.P, a.flags, a.mu, g.sf, p, pt, o);
  nfatal += (o.flags & MHD_FLAG_FATAL) ? 1 : 0;
  ncorr += (o.flags & C2P_CORRECTED) ? 1 : 0;
  nit += o.iters;
}

// grid-stride over the padded points in memory order
__global__ void __launch_bounds__(256) k_con2prim(C2pArgs a, int64_t npts) {
  __shared__ mhd_eos_t seos;
  const mhd_eos_t& eos = stage_eos(a.eos, seos);
  const Geom& g = a.g;
  const int Nx = g.nx + 2 * g.ng, Ny = g.ny + 2 * g.ng;
  int64_t nfatal = 0, ncorr = 0, nit = 0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npts; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % Nx), j = (int)((t / Nx) % Ny), k = (int)(t / ((int64_t)Nx * Ny));
    con2prim_at(a, eos, i, j, k, nfatal, ncorr, nit);
  }
  if (a.stats) block_add_stats(a.stats, nfatal, ncorr, 0, nit);
}

__global__ void __launch_bounds__(256) k_con2prim_lv(LevelArgs L) {
  __shared__ mhd_eos_t seos;
  const mhd_eos_t& eos = stage_eos(L.eos, seos);
  int64_t nfatal = 0, ncorr = 0, nit = 0;
  for_each_level_point(L, kRegionPadded, [&](const BoxDev& B, int i, int j, int k, bool live) {
    C2pArgs a;  // the EoS is read from LDS
    a.g = B.g;
    a.U = L.src ? B.Us : B.U;
    a.P = B.P;
    a.flags = B.flags;
    a.mu = nullptr;
    a.stats = L.stats;
    if (live) con2prim_at(a, eos, i, j, k, nfatal, ncorr, nit);
  });
  if (L.stats) block_add_stats(L.stats, nfatal, ncorr, 0, nit);
}

int launch_con2prim_level(const LevelArgs& L, int grid, int block, hipStream_t s) {
  MHD_LAUNCH(KID_CON2PRIM, k_con2prim_lv, dim3(grid), dim3(block), 0, s, L);
  return (int)hipGetLastError();
}

struct P2cArgs {
  Geom g;
  mhd_eos_t eos;
  double* __restrict__ U;
  double* __restrict__ P;
  const double* __restrict__ EM;
  int eps_mode;
};

__global__ void __launch_bounds__(256) k_prim2con(P2cArgs a) {
  const Geom& g = a.g;
  const int Nx = g.nx + 2 * g.ng, Ny = g.ny + 2 * g.ng;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= Nx || j >= Ny) return;
  const int64_t sf = g.sf;
  const int64_t p = g.at(i, j, k);
  double gt[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) gt[c] = a.U[c * sf + p];
  MetricR m;
  metric_repro(gt, a.U[12 * sf + p], m);
  double rho = a.P[p], eps = a.P[sf + p];
  if (a.eps_mode == 1) eps += eos_cold(a.eos, rho).e;
  const double v[3] = {a.P[3 * sf + p], a.P[4 * sf + p], a.P[5 * sf + p]};
  const double B[3] = {a.EM[p], a.EM[sf + p], a.EM[2 * sf + p]};
  const double ye = a.P[7 * sf + p];
  const double pr = eos_press(a.eos, rho, eps);
  double cons[6], W;
  prim_to_cons(m.gd, rho, eps, pr, v, ye, B, cons, W);
#pragma unroll
  for (int c = 0; c < 6; ++c) a.U[(22 + c) * sf + p] = m.sqrtg * cons[c];
#pragma unroll
  for (int c = 0; c < 3; ++c) a.U[(28 + c) * sf + p] = m.sqrtg * B[c];
  a.U[31 * sf + p] = m.sqrtg * a.EM[3 * sf + p];
  a.P[sf + p] = eps;
  a.P[2 * sf + p] = pr;
  a.P[6 * sf + p] = W;
}

int launch_con2prim(const Geom& g, const mhd_eos_t& eos, double* U, double* P, uint8_t* flags, double* mu,
                    int64_t* stats, hipStream_t s) {
  C2pArgs a{g, eos, U, P, flags, mu, stats};
  const int64_t npts = (int64_t)(g.nx + 2 * g.ng) * (g.ny + 2 * g.ng) * (g.nz + 2 * g.ng);
  const int64_t nblk = (npts + 255) / 256;
  MHD_LAUNCH(KID_CON2PRIM, k_con2prim, dim3((unsigned)(nblk < 2048 ? nblk : 2048)), dim3(256), 0, s, a, npts);
  return (int)hipGetLastError();
}

int launch_prim2con(const Geom& g, const mhd_eos_t& eos, double* U, double* P, const double* EM, int eps_mode,
                    hipStream_t s) {
  P2cArgs a{g, eos, U, P, EM, eps_mode};
  const int Nx = g.nx + 2 * g.ng, Ny = g.ny + 2 * g.ng, Nz = g.nz + 2 * g.ng;
  MHD_LAUNCH(KID_PRIM2CON, k_prim2con, dim3((Nx + 63) / 64, (Ny + 3) / 4, Nz), dim3(64, 4, 1), 0, s, a);
  return (int)hipGetLastError();
}

}  // namespace mhd
