// Mesh-refinement glue: 2:1 vertex-centred prolongation by the symmetric
// six-point Lagrange interpolation and restriction by copy (Sec. 4.2), and the
// dense output of RK4 with its time derivatives (Sec. 3.1), for boundary data
// of sub-cycled fine levels.
//
// Index convention: fine padded index I and coarse padded index i coincide
// when I = 2 i + off (per axis).  A fine point with I - off odd lies half-way
// between coarse i = (I - off - 1)/2 and i + 1 and takes
//   (3 U_{i-2} - 25 U_{i-1} + 150 U_i + 150 U_{i+1} - 25 U_{i+2} + 3 U_{i+3}) / 256,
// the Lagrange polynomial through the six nearest coarse points evaluated at
// the midpoint.  In 3D the one-dimensional interpolation is applied along x,
// then y, then z (a tensor product: polynomials of degree <= 5 in each variable
// are reproduced).  The six weights are exact binary fractions and the sums
// are taken in node order without contraction.
#include "dev_common.hpp"
#include "prof.hpp"

namespace mhd {

#pragma clang fp contract(off)

__constant__ double kLag6[6] = {3.0 / 256.0, -25.0 / 256.0, 150.0 / 256.0, 150.0 / 256.0, -25.0 / 256.0, 3.0 / 256.0};

struct ProlongArgs {
  Geom gc, gf;  // coarse and fine patches
  const double* __restrict__ Uc;
  double* __restrict__ Uf;
  int nfields;
  int off[3];
  int lo[3];   // fine padded index box [lo, lo + n)
  int n[3];
};

// first coarse node and node count along one axis for half-index t = I - off
__device__ __forceinline__ void prolong_nodes(int t, int& first, int& count) {
  if ((t & 1) == 0) {
    first = t >> 1;  // arithmetic shift: floor(t / 2)
    count = 1;
  } else {
    first = ((t - 1) >> 1) - 2;
    count = 6;
  }
}

// block 64x4 over (x, y) of the fine box, grid.z over its z extent
__global__ void __launch_bounds__(256) k_prolong(ProlongArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.n[0] || y >= a.n[1]) return;
  const int I = a.lo[0] + x, J = a.lo[1] + y, K = a.lo[2] + z;
  int fx, nx, fy, ny, fz, nz;
  prolong_nodes(I - a.off[0], fx, nx);
  prolong_nodes(J - a.off[1], fy, ny);
  prolong_nodes(K - a.off[2], fz, nz);
  const Geom& gc = a.gc;
  const int64_t pf = a.gf.at(I, J, K);
#pragma unroll 1
  for (int f = 0; f < a.nfields; ++f) {
    const double* __restrict__ A = a.Uc + (int64_t)f * gc.sf;
    // loops unrolled to six with a guard, so vy and vz stay in registers
    double vz[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if (c >= nz) break;
      double vy[6];
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        if (b >= ny) break;
        const double* row = A + gc.at(fx, fy + b, fz + c);
        double s;
        if (nx == 1) {
          s = row[0];
        } else {
          s = 0.0;
#pragma unroll
          for (int q = 0; q < 6; ++q) s += kLag6[q] * row[q];
        }
        vy[b] = s;
      }
      double s;
      if (ny == 1) {
        s = vy[0];
      } else {
        s = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) s += kLag6[q] * vy[q];
      }
      vz[c] = s;
    }
    double s;
    if (nz == 1) {
      s = vz[0];
    } else {
      s = 0.0;
#pragma unroll
      for (int q = 0; q < 6; ++q) s += kLag6[q] * vz[q];
    }
    a.Uf[(int64_t)f * a.gf.sf + pf] = s;
  }
}

struct RestrictArgs {
  Geom gf, gc;
  const double* __restrict__ Uf;
  double* __restrict__ Uc;
  int nfields;
  int off[3];
  int lo[3];  // coarse padded index box [lo, lo + n)
  int n[3];
};

__global__ void __launch_bounds__(256) k_restrict(RestrictArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.n[0] || y >= a.n[1]) return;
  const int i = a.lo[0] + x, j = a.lo[1] + y, k = a.lo[2] + z;
  const int64_t pc = a.gc.at(i, j, k), pf = a.gf.at(2 * i + a.off[0], 2 * j + a.off[1], 2 * k + a.off[2]);
#pragma unroll 4
  for (int f = 0; f < a.nfields; ++f) a.Uc[(int64_t)f * a.gc.sf + pc] = a.Uf[(int64_t)f * a.gf.sf + pf];
}

struct DenseArgs {
  Geom g;
  int nfields;
  int add_un;      // 1: U^n + sum (value), 0: the derivative sum alone
  double dt;
  double b[4];     // b_j^(m)(theta)
  double dtm;      // dt^m for m >= 1 (unused for m = 0)
  const double* __restrict__ Un;
  const double* __restrict__ L[4];  // stage right-hand sides
  double* __restrict__ out;
};

// block 64x4 over (x, y) of the interior, grid.z over z * nfields
__global__ void __launch_bounds__(256) k_dense_output(DenseArgs a) {
  const Geom& g = a.g;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y * blockDim.y + threadIdx.y;
  const int kz = blockIdx.z % g.nz, f = blockIdx.z / g.nz;
  if (i >= g.nx || j >= g.ny) return;
  const int64_t p = (int64_t)f * g.sf + g.at(i + g.ng, j + g.ng, kz + g.ng);
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) s += a.b[q] * (a.dt * a.L[q][p]);
  a.out[p] = a.add_un ? a.Un[p] + s : s / a.dtm;
}

int launch_prolong(const Geom& gc, const double* Uc, const Geom& gf, double* Uf, int nfields, const int off[3],
                   const int lo[3], const int n[3], hipStream_t s) {
  ProlongArgs a;
  a.gc = gc;
  a.gf = gf;
  a.Uc = Uc;
  a.Uf = Uf;
  a.nfields = nfields;
  for (int d = 0; d < 3; ++d) {
    a.off[d] = off[d];
    a.lo[d] = lo[d];
    a.n[d] = n[d];
  }
  MHD_LAUNCH(KID_PROLONG, k_prolong, dim3((n[0] + 63) / 64, (n[1] + 3) / 4, n[2]), dim3(64, 4, 1), 0, s, a);
  return (int)hipGetLastError();
}

int launch_restrict(const Geom& gf, const double* Uf, const Geom& gc, double* Uc, int nfields, const int off[3],
                    const int lo[3], const int n[3], hipStream_t s) {
  RestrictArgs a;
  a.gf = gf;
  a.gc = gc;
  a.Uf = Uf;
  a.Uc = Uc;
  a.nfields = nfields;
  for (int d = 0; d < 3; ++d) {
    a.off[d] = off[d];
    a.lo[d] = lo[d];
    a.n[d] = n[d];
  }
  MHD_LAUNCH(KID_RESTRICT, k_restrict, dim3((n[0] + 63) / 64, (n[1] + 3) / 4, n[2]), dim3(64, 4, 1), 0, s, a);
  return (int)hipGetLastError();
}

int launch_dense_output(const Geom& g, int nfields, double dt, const double b[4], int add_un, double dtm,
                        const double* Un, const double* const* L, double* out, hipStream_t s) {
  DenseArgs a;
  a.g = g;
  a.nfields = nfields;
  a.add_un = add_un;
  a.dt = dt;
  for (int q = 0; q < 4; ++q) {
    a.b[q] = b[q];
    a.L[q] = L[q];
  }
  a.dtm = dtm;
  a.Un = Un;
  a.out = out;
  MHD_LAUNCH(KID_DENSE, k_dense_output, dim3((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz * nfields), dim3(64, 4, 1), 0,
             s, a);
  return (int)hipGetLastError();
}

}  // namespace mhd
