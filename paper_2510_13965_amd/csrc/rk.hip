// Explicit RK4 stage update (Table I, explicit part) and periodic ghost fill.
//
// The stage kernel is a pure streaming kernel (HBM bound): each thread owns one
// interior element of one field; a wavefront covers 64 consecutive x of a row,
// so every access is a coalesced 512-byte transaction.  Per element it moves
// 3 reads + 2 writes (stages 0-2) or 3 reads + 1 write (stage 3) of 8 bytes.
#include "dev_common.hpp"
#include "prof.hpp"

namespace mhd {

// plain IEEE adds and multiplies (no contraction): the stage update is then
// reproducible bit for bit by any FP64 implementation of the same formula
#pragma clang fp contract(off)

__constant__ double kRk4A[3] = {0.5, 0.5, 1.0};
__constant__ double kRk4B[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};

struct RkArgs {
  Geom g;
  int stage;
  double dt;
  const double* Un;
  const double* __restrict__ k;
  double* acc;
  double* Unext;
};

// one element: acc and Unext of Table I's stage `a.stage`
__device__ __forceinline__ void rk4_element(const RkArgs& a, int64_t p) {
  const double kv = a.k[p];
  const int s = a.stage;
  const double b = kRk4B[s] * kv;
  if (s < 3) {
    a.acc[p] = (s == 0) ? b : a.acc[p] + b;
    a.Unext[p] = a.Un[p] + a.dt * kRk4A[s] * kv;
  } else {
    a.Unext[p] = a.Un[p] + a.dt * (a.acc[p] + b);
  }
}

// SSP-RK(3,3) of Shu and Osher (Sec. 3.1; the explicit half of IMEX(3,3,2)):
// c = (0, 1, 1/2), A = ((0), (1), (1/4, 1/4)), b = (1/6, 1/6, 2/3).  Stored as
// acc = sum of b_j k_j so far, which after stage 1 is (k0 + k1)/6, so the third
// stage state Un + dt (k0 + k1)/4 is Un + dt (3/2) acc:
//   s = 0: acc = k/6;        Unext = Un + dt k
//   s = 1: acc = acc + k/6;  Unext = Un + dt (3/2 acc)
//   s = 2: Unext = Un + dt (acc + 2/3 k)
__device__ __forceinline__ void ssprk3_element(const RkArgs& a, int64_t p) {
  const double kv = a.k[p];
  const int s = a.stage;
  if (s == 0) {
    a.acc[p] = kv / 6.0;
    a.Unext[p] = a.Un[p] + a.dt * kv;
  } else if (s == 1) {
    const double acc = a.acc[p] + kv / 6.0;
    a.acc[p] = acc;
    a.Unext[p] = a.Un[p] + a.dt * (1.5 * acc);
  } else {
    a.Unext[p] = a.Un[p] + a.dt * (a.acc[p] + 2.0 / 3.0 * kv);
  }
}

__global__ void __launch_bounds__(256) k_ssprk3_stage(RkArgs a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int kz = blockIdx.z % g.nz;
  const int f = blockIdx.z / g.nz;
  if (i >= g.nx || j >= g.ny) return;
  ssprk3_element(a, (int64_t)f * g.sf + g.at(i + g.ng, j + g.ng, kz + g.ng));
}

// block 64x4: x = 64 consecutive points of a row, y = 4 rows; grid z = k * nfields + f
__global__ void __launch_bounds__(256) k_rk4_stage(RkArgs a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int kz = blockIdx.z % g.nz;
  const int f = blockIdx.z / g.nz;
  if (i >= g.nx || j >= g.ny) return;
  rk4_element(a, (int64_t)f * g.sf + g.at(i + g.ng, j + g.ng, kz + g.ng));
}

// all evolved fields (32, or 44 with M1) of every interior point of a level's boxes
template <int NF>
__device__ __forceinline__ void rk4_level_point(const LevelArgs& L) {
  for_each_level_point(L, kRegionInterior, [&](const BoxDev& B, int i, int j, int k, bool live) {
    if (!live) return;
    const RkArgs a{B.g, L.stage, L.dt, B.U, B.k, B.acc, L.stage < 3 ? B.Us : B.U};
    const int64_t p = B.g.at(i + B.g.ng, j + B.g.ng, k + B.g.ng);
#pragma unroll 4
    for (int f = 0; f < NF; ++f) rk4_element(a, (int64_t)f * B.g.sf + p);
  });
}

__global__ void __launch_bounds__(256) k_rk4_stage_lv(LevelArgs L) {
  if (L.nfields == MHD_NU_M1N) rk4_level_point<MHD_NU_M1N>(L);
  else if (L.nfields == MHD_NU_M1) rk4_level_point<MHD_NU_M1>(L);
  else rk4_level_point<MHD_NU>(L);
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

int launch_ssprk3_stage(const Geom& g, int nfields, int stage, double dt, const double* Un, const double* k,
                        double* acc, double* Unext, hipStream_t s) {
  const RkArgs a{g, stage, dt, Un, k, acc, Unext};
  MHD_LAUNCH(KID_SSPRK3_STAGE, k_ssprk3_stage, dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz * nfields), dim3(64, 4, 1), 0,
             s, a);
  return (int)hipGetLastError();
}

int launch_rk4_level(const LevelArgs& L, int grid, int block, hipStream_t s) {
  MHD_LAUNCH(KID_RK4_STAGE, k_rk4_stage_lv, dim3(grid), dim3(block), 0, s, L);
  return (int)hipGetLastError();
}

int launch_zero_u64(unsigned long long* p, hipStream_t s) {
  MHD_LAUNCH(KID_ZERO, k_zero_u64, dim3(1), dim3(1), 0, s, p);
  return (int)hipGetLastError();
}

struct GhostArgs {
  Geom g;
  double* U;
};

// periodic: every ghost point copies the interior point a whole number of
// periods away (faces, edges and corners in one pass; interior threads exit)
__global__ void __launch_bounds__(256) k_ghosts_periodic(GhostArgs a) {
  const Geom& g = a.g;
  const int Nx = g.nx + 2 * g.ng, Ny = g.ny + 2 * g.ng, Nz = g.nz + 2 * g.ng;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int kz = blockIdx.z % Nz;
  const int f = blockIdx.z / Nz;
  if (i >= Nx || j >= Ny) return;
  auto wrap = [](int q, int n, int ng) { return ((q - ng) % n + n) % n + ng; };
  const int si = wrap(i, g.nx, g.ng), sj = wrap(j, g.ny, g.ng), sk = wrap(kz, g.nz, g.ng);
  if (si == i && sj == j && sk == kz) return;
  double* u = a.U + (int64_t)f * g.sf;
  u[g.at(i, j, kz)] = u[g.at(si, sj, sk)];
}

struct ZeroArgs {
  Geom g;
  int f0;
  double* A;
};

__global__ void __launch_bounds__(256) k_zero_interior(ZeroArgs a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int kz = blockIdx.z % g.nz;
  const int f = a.f0 + blockIdx.z / g.nz;
  if (i >= g.nx || j >= g.ny) return;
  a.A[(int64_t)f * g.sf + g.at(i + g.ng, j + g.ng, kz + g.ng)] = 0.0;
}

int launch_zero_interior(const Geom& g, int f0, int nfields, double* A, hipStream_t s) {
  ZeroArgs a{g, f0, A};
  dim3 grd((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz * nfields);
  MHD_LAUNCH(KID_ZERO, k_zero_interior, grd, dim3(64, 4, 1), 0, s, a);
  return (int)hipGetLastError();
}

int launch_rk4_stage(const Geom& g, int nfields, int stage, double dt, const double* Un, const double* k, double* acc,
                     double* Unext, hipStream_t s) {
  RkArgs a{g, stage, dt, Un, k, acc, Unext};
  dim3 grd((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz * nfields);
  MHD_LAUNCH(KID_RK4_STAGE, k_rk4_stage, grd, dim3(64, 4, 1), 0, s, a);
  return (int)hipGetLastError();
}

int launch_ghosts_periodic(const Geom& g, double* U, int nfields, hipStream_t s) {
  GhostArgs a{g, U};
  const int Nx = g.nx + 2 * g.ng, Ny = g.ny + 2 * g.ng, Nz = g.nz + 2 * g.ng;
  dim3 grd((Nx + 63) / 64, (Ny + 3) / 4, Nz * nfields);
  MHD_LAUNCH(KID_GHOSTS, k_ghosts_periodic, grd, dim3(64, 4, 1), 0, s, a);
  return (int)hipGetLastError();
}

}  // namespace mhd
