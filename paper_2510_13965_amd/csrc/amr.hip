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

// Separable form: a block owns a fine tile of kPx x kPy x kPz points and, per
// field, stages the coarse nodes under it in LDS, interpolates along x (fine x,
// coarse y and z), then along y, then along z.  Every intermediate value is the
// sum the per-point definition forms for it (same nodes, same order), so the
// result is the tensor product above, bit for bit, with ~6 LDS reads per fine
// point instead of up to 216 global ones.
constexpr int kPx = 32, kPy = 8, kPz = 8;
constexpr int kCx = kPx / 2 + 7, kCy = kPy / 2 + 7, kCz = kPz / 2 + 7;  // coarse nodes under a tile (bound)

// one-dimensional interpolation at half-index t from nodes src[(node - c0) * stride]
__device__ __forceinline__ double interp1(const double* src, int t, int c0, int stride) {
  if ((t & 1) == 0) return src[((t >> 1) - c0) * stride];
  const int first = ((t - 1) >> 1) - 2 - c0;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 6; ++q) s += kLag6[q] * src[(first + q) * stride];
  return s;
}

__global__ void __launch_bounds__(256) k_prolong(ProlongArgs a) {
  __shared__ double X[kCz * kCy * kPx];  // x-interpolated: [cz][cy][fx]
  __shared__ double CY[kCz * kPy * kPx];  // coarse block [cz][cy][cx], then y-interpolated [cz][fy][fx]
  static_assert(kCz * kCy * kCx <= kCz * kPy * kPx, "the coarse block fits the second buffer");
  const int tid = threadIdx.x;
  const int fx0 = blockIdx.x * kPx, fy0 = blockIdx.y * kPy, fz0 = blockIdx.z * kPz;  // tile origin in the box
  // half-indices of the tile's first fine point and the first coarse node staged
  const int tx0 = a.lo[0] + fx0 - a.off[0], ty0 = a.lo[1] + fy0 - a.off[1], tz0 = a.lo[2] + fz0 - a.off[2];
  const int cx0 = ((tx0 - 1) >> 1) - 2, cy0 = ((ty0 - 1) >> 1) - 2, cz0 = ((tz0 - 1) >> 1) - 2;
  const Geom& gc = a.gc;
  const int Ncx = gc.nx + 2 * gc.ng, Ncy = gc.ny + 2 * gc.ng, Ncz = gc.nz + 2 * gc.ng;
#pragma unroll 1
  for (int f = 0; f < a.nfields; ++f) {
    const double* __restrict__ A = a.Uc + (int64_t)f * gc.sf;
    __syncthreads();  // the previous field's last pass has read CY
    for (int e = tid; e < kCz * kCy * kCx; e += blockDim.x) {
      const int cx = e % kCx, cy = (e / kCx) % kCy, cz = e / (kCx * kCy);
      const int i = cx0 + cx, j = cy0 + cy, k = cz0 + cz;
      // nodes outside the coarse array serve only points outside the box
      CY[e] = (i >= 0 && j >= 0 && k >= 0 && i < Ncx && j < Ncy && k < Ncz) ? A[gc.at(i, j, k)] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < kCz * kCy * kPx; e += blockDim.x) {
      const int fx = e % kPx, row = e / kPx;  // row = cz * kCy + cy
      X[e] = interp1(CY + row * kCx, tx0 + fx, cx0, 1);
    }
    __syncthreads();
    for (int e = tid; e < kCz * kPy * kPx; e += blockDim.x) {
      const int fx = e % kPx, fy = (e / kPx) % kPy, cz = e / (kPx * kPy);
      CY[e] = interp1(X + cz * kCy * kPx + fx, ty0 + fy, cy0, kPx);
    }
    __syncthreads();
    for (int e = tid; e < kPz * kPy * kPx; e += blockDim.x) {
      const int fx = e % kPx, fy = (e / kPx) % kPy, fz = e / (kPx * kPy);
      if (fx0 + fx < a.n[0] && fy0 + fy < a.n[1] && fz0 + fz < a.n[2]) {
        const double v = interp1(CY + fy * kPx + fx, tz0 + fz, cz0, kPy * kPx);
        a.Uf[(int64_t)f * a.gf.sf + a.gf.at(a.lo[0] + fx0 + fx, a.lo[1] + fy0 + fy, a.lo[2] + fz0 + fz)] = v;
      }
    }
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
  MHD_LAUNCH(KID_PROLONG, k_prolong, dim3((n[0] + kPx - 1) / kPx, (n[1] + kPy - 1) / kPy, (n[2] + kPz - 1) / kPz),
             dim3(256), 0, s, a);
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
