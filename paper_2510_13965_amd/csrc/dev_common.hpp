// Device-side building blocks shared by the HIP kernels of the library:
// patch geometry, the hybrid EoS of Sec. 2.2, 3x3 symmetric algebra and the
// finite-difference operators of Sec. 3.2.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mhd.h"

namespace mhd {

// symmetric 3x3 storage order: xx xy xz yy yz zz
__host__ __device__ constexpr int sym(int i, int j) {
  return (i <= j) ? (i == 0 ? j : (i == 1 ? 2 + j : 5)) : (j == 0 ? i : (j == 1 ? 2 + i : 5));
}

struct Geom {
  int nx, ny, nz, ng;
  int64_t sy, sz, sf;
  double h[3];     // dx per axis
  double idx[3];   // 1/dx per axis
  double i12[3];   // 1/(12 dx)
  double i12s[3];  // 1/(12 dx^2)
  __device__ __forceinline__ int64_t at(int i, int j, int k) const {
    return (int64_t)i + (int64_t)j * sy + (int64_t)k * sz;
  }
  __device__ __forceinline__ int64_t stride(int a) const { return a == 0 ? 1 : (a == 1 ? sy : sz); }
};

// x / b rounded to nearest for b > 0, given rb = 1/b rounded to nearest (by a
// correctly rounded division): q = RN(x rb) is within an ulp of x/b, the
// remainder x - b q is exact with an FMA, and one correction step
// RN(q + (x - b q) rb) is the correctly rounded quotient (Markstein's theorem
// for division with a correctly rounded reciprocal; finite x, no underflow).
// Three FP64 operations in place of the ~10 of the general division, with the
// same result.
__device__ __forceinline__ double div_rn(double x, double b, double rb) {
  const double q = x * rb;
  const double r = __builtin_fma(-q, b, x);
  return __builtin_fma(r, rb, q);
}

// ------------------------------------------------------------------ tile order
//
// Stencil kernels run on a 1D grid of 64x4 (x,y) tiles.  The hardware hands
// consecutive workgroups to the 8 XCDs round-robin, and each XCD has its own
// L2, so with the natural order y-neighbour tiles (which share halo rows) land
// on different L2s.  The mapping below gives every XCD a contiguous range of
// tiles, and walks that range in strips of `strip` tile rows, z fastest, so
// the tiles an XCD has in flight are stacked in z and share their +-3-plane
// halos in its L2.
struct TileXYZ {
  int bx, by, bz;
};

// tile of linear id `id` (0 <= id < nbx*nby*nbz) in the strip order
__device__ __forceinline__ TileXYZ tile_of_index(int id, int nbx, int nby, int nbz, int strip) {
  const int sh = strip < nby ? strip : nby;
  const int per_strip = sh * nbx * nbz;
  const int st = id / per_strip;
  int r = id - st * per_strip;
  const int rows = (st * sh + sh <= nby) ? sh : (nby - st * sh);  // last strip may be short
  const int per_plane = rows * nbx;
  TileXYZ t;
  t.bz = r / per_plane;
  r -= t.bz * per_plane;
  t.by = st * sh + r / nbx;
  t.bx = r - (r / nbx) * nbx;
  return t;
}

__device__ __forceinline__ TileXYZ tile_of_block(int nbx, int nby, int nbz, int strip) {
  const int nblk = nbx * nby * nbz;
  const int b = blockIdx.x;
  const int per_xcd = (nblk + 7) / 8;
  const int xcd = b & 7, slot = b >> 3;
  const int id = xcd * per_xcd + slot;  // contiguous range per XCD
  if (id >= nblk) {
    TileXYZ t{-1, -1, -1};
    return t;
  }
  return tile_of_index(id, nbx, nby, nbz, strip);
}

// Maximum of a non-negative value over the block, then one atomic max (on the
// bit pattern) per block: atomics on one address are serialised in L2.  Every
// thread of the block (at most 256 threads) calls this once.
__device__ __forceinline__ void block_max_to(unsigned long long* dst, double v) {
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  if (tid % 64 == 0) red[tid / 64] = v;
  __syncthreads();
  if (tid == 0) {
    const int nw = (int)((blockDim.x * blockDim.y + 63) / 64);
    double m = red[0];
    for (int w = 1; w < nw; ++w) m = fmax(m, red[w]);
    atomicMax(dst, (unsigned long long)__double_as_longlong(m));
  }
}

// ------------------------------------------------------------------ batched levels
//
// A level is a list of boxes (patches of any shape) processed by persistent
// kernels, one per phase of the right-hand side.  Each phase walks a global
// tile space: box-major, and inside a box the chunks of `blockDim.x`
// consecutive points of a z plane (row-major, so narrow boxes still fill the
// wavefront), in the strip order (z fastest inside strips of `strip` chunks).
// Every XCD takes a contiguous range of the global space.  The per-point work
// is the same device code as the single-patch kernels, so results are bitwise
// those of per-box launches.
// LDS-staged level kernels: kLevelLdsTile x kLevelLdsTile (x,y) tiles streamed
// through chunks of kLevelLdsZ z planes
constexpr int kLevelLdsTile = 16, kLevelLdsZ = 8;

struct BoxDev {
  Geom g;
  double* U;    // state at t^n
  double* Us;   // stage state
  double* P;    // primitives
  double* k;    // right-hand side
  double* acc;  // RK accumulator
  double* ws;   // RHS workspace
  uint8_t* flags;
  const double* aux;  // M1 opacities and emissivities (levels evolving radiation), else null
  double* ws_m1;      // M1 part of the RHS workspace, else null
  double* F[4];       // IMEX: explicit parts of the four stages (44 or 47 fields), else null
  double* R[4];       // IMEX: stiff parts of the four stages (12 or 15 fields), else null
  int cpp_int, cpp_pad, cpp_h1;    // chunks per z plane of the interior / padded box / interior plus one layer
  int64_t t0_int, t0_pad, t0_h1;  // first global tile id of the box in each space
  int ntx_lds, nty_lds, nzc_lds;  // LDS-staged kernels: (x, y) tiles and z chunks of the box
  int64_t t0_lds;                 // first global id of the box in the LDS tile space
};

struct LevelArgs {
  const BoxDev* __restrict__ boxes;
  int nboxes;
  int strip;
  int src;  // 0: evaluate at U, 1: at Us
  int stage;
  int nfields;  // evolved fields: 32, 44 with three M1 species, 47 with their number densities
  int m1;       // nonzero: the boxes evolve the M1 radiation
  int nd;       // nonzero: and the three number densities (15 aux fields, 75 M1 workspace fields)
  int slot;     // right-hand side into k (-1) or, in an IMEX stage, into F[slot] with the stiff part in R[slot]
  double adt;   // IMEX: implicit step a_ii dt of the collision solve
  unsigned long long* nfail;  // IMEX: count of collision solves that did not converge (may be null)
  int64_t ntile_int, ntile_pad, ntile_h1, ntile_lds;
  double dt;
  mhd_params_t par;
  mhd_eos_t eos;
  unsigned long long* max_speed;
  int64_t* stats;
  // con2prim with the learned guess (mlp == nullptr: the bracketed solver)
  const float* mlp;
  uint32_t* qcount;  // [0]: points to solve, [1]: points for the bracketed solver
  uint64_t* queue;   // (box << 32) | padded point of the points to solve
  uint64_t* fqueue;  // the same for the rejected points
  float* feat;       // per solve-queue slot: 8 network inputs, then its 2 outputs in place
};

// where the right-hand-side kernels of a level write: k (RK), or an IMEX
// stage's explicit part and, for the radiation, its stiff part.  The kernels
// are instantiated per case, so the RK ones carry no trace of the IMEX outputs
// (a runtime choice cost registers and up to 10 % of the level step).
template <bool IMEX>
__device__ __forceinline__ double* level_rhs(const BoxDev& B, const LevelArgs& L) {
  return IMEX ? B.F[L.slot] : B.k;
}
template <bool IMEX>
__device__ __forceinline__ double* level_stiff(const BoxDev& B, const LevelArgs& L) {
  return IMEX ? B.R[L.slot] : nullptr;
}

// the regions a level kernel can walk: the interior, the padded box, or the
// interior with one ghost layer (the points whose M1 point fluxes and closure
// the update reads)
enum LevelRegion { kRegionInterior = 0, kRegionPadded = 1, kRegionHalo1 = 2 };

__device__ __forceinline__ int find_box(const LevelArgs& L, int64_t id, int region) {
  int lo = 0, hi = L.nboxes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const BoxDev& M = L.boxes[mid];
    const int64_t t0 = region == kRegionPadded ? M.t0_pad : (region == kRegionHalo1 ? M.t0_h1 : M.t0_int);
    if (t0 <= id) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Calls body(box, i, j, k, live) for every point of the region's tile space,
// once per thread and tile: i, j, k are interior indices for the interior and
// padded indices otherwise (kRegionHalo1 starts at padded index ng - 1).
template <class F>
__device__ __forceinline__ void for_each_level_point(const LevelArgs& L, int region, F&& body) {
  const bool padded = region == kRegionPadded, h1 = region == kRegionHalo1;
  const int64_t total = padded ? L.ntile_pad : (h1 ? L.ntile_h1 : L.ntile_int);
  const int per_g = gridDim.x >> 3;  // gridDim.x is a multiple of 8
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int64_t per = (total + 7) / 8;
  const int64_t lo = xcd * per;
  const int64_t hi = lo + per < total ? lo + per : total;
  for (int64_t id = lo + slot; id < hi; id += per_g) {
    const int b = find_box(L, id, region);
    const BoxDev& B = L.boxes[b];
    const int ext = padded ? 2 * B.g.ng : (h1 ? 2 : 0);  // points added to each extent
    const int nx = B.g.nx + ext, ny = B.g.ny + ext, nz = B.g.nz + ext;
    const int cpp = padded ? B.cpp_pad : (h1 ? B.cpp_h1 : B.cpp_int);
    const int local = (int)(id - (padded ? B.t0_pad : (h1 ? B.t0_h1 : B.t0_int)));
    const TileXYZ t = tile_of_index(local, 1, cpp, nz, L.strip);
    const int q = t.by * (int)blockDim.x + (int)threadIdx.x;
    const bool live = q < nx * ny;
    const int j = live ? q / nx : 0;
    const int i = live ? q - j * nx : 0;
    const int o = h1 ? B.g.ng - 1 : 0;  // to padded indices
    body(B, i + o, j + o, t.bz + o, live);
  }
}

// ------------------------------------------------------------------ EoS

struct Cold {
  double p, e;  // p_cold, eps_cold
  double K, G;  // piece constants
};

__device__ __forceinline__ Cold eos_cold(const mhd_eos_t& e, double rho) {
#pragma clang fp contract(off)
  int i = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b)
    if (b < e.npieces - 1 && rho >= e.rho_b[b]) i = b + 1;
  Cold c;
  c.K = e.K[i];
  c.G = e.Gamma[i];
  if (c.K == 0.0) {
    c.p = 0.0;
    c.e = e.a[i];
  } else {
    c.p = c.K * pow(rho, c.G);
    c.e = e.a[i] + c.K / (c.G - 1.0) * pow(rho, c.G - 1.0);
  }
  return c;
}

__device__ __forceinline__ double eos_press(const mhd_eos_t& e, double rho, double eps) {
#pragma clang fp contract(off)
  const Cold c = eos_cold(e, rho);
  return c.p + (e.Gamma_th - 1.0) * rho * (eps - c.e);
}

// c_s^2 = (dp/drho|_eps + p/rho^2 dp/deps|_rho) / (1 + eps + p/rho)
__device__ __forceinline__ double eos_cs2(const mhd_eos_t& e, double rho, double eps, double p) {
  const Cold c = eos_cold(e, rho);
  const double gt1 = e.Gamma_th - 1.0;
  const double dpdrho = (c.G - gt1) * c.p / rho + gt1 * (eps - c.e);
  const double dpdeps = gt1 * rho;
  return (dpdrho + p / (rho * rho) * dpdeps) / (1.0 + eps + p / rho);
}

// ------------------------------------------------------------------ 3x3 symmetric

// inverse of a symmetric 3x3 matrix; returns the determinant
__device__ __forceinline__ double sym_inv(const double g[6], double gi[6]) {
#pragma clang fp contract(off)
  const double c00 = g[3] * g[5] - g[4] * g[4];
  const double c01 = g[2] * g[4] - g[1] * g[5];
  const double c02 = g[1] * g[4] - g[2] * g[3];
  const double det = g[0] * c00 + g[1] * c01 + g[2] * c02;
  const double id = 1.0 / det;
  gi[0] = c00 * id;
  gi[1] = c01 * id;
  gi[2] = c02 * id;
  gi[3] = (g[0] * g[5] - g[2] * g[2]) * id;
  gi[4] = (g[1] * g[2] - g[0] * g[4]) * id;
  gi[5] = (g[0] * g[3] - g[1] * g[1]) * id;
  return det;
}

__device__ __forceinline__ void sym_mv(const double g[6], const double v[3], double o[3]) {
#pragma clang fp contract(off)
  o[0] = g[0] * v[0] + g[1] * v[1] + g[2] * v[2];
  o[1] = g[1] * v[0] + g[3] * v[1] + g[4] * v[2];
  o[2] = g[2] * v[0] + g[4] * v[1] + g[5] * v[2];
}

// Physical metric in a fixed order of plain IEEE operations (used wherever a
// result must be reproducible bit for bit): inverse by cofactors divided by
// the determinant, gamma_ij = gt_ij/chi, gamma^ij = chi gt^ij,
// sqrt(gamma) = sqrt(det/chi^3).
struct MetricR {
  double gtu[6], gd[6], gu[6], sqrtg;
};

__device__ __forceinline__ void metric_repro(const double g[6], double chi, MetricR& m) {
#pragma clang fp contract(off)
  const double c00 = g[3] * g[5] - g[4] * g[4];
  const double c01 = g[2] * g[4] - g[1] * g[5];
  const double c02 = g[1] * g[4] - g[2] * g[3];
  const double det = g[0] * c00 + g[1] * c01 + g[2] * c02;
  m.gtu[0] = c00 / det;
  m.gtu[1] = c01 / det;
  m.gtu[2] = c02 / det;
  m.gtu[3] = (g[0] * g[5] - g[2] * g[2]) / det;
  m.gtu[4] = (g[1] * g[2] - g[0] * g[4]) / det;
  m.gtu[5] = (g[0] * g[3] - g[1] * g[1]) / det;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    m.gd[a] = g[a] / chi;
    m.gu[a] = chi * m.gtu[a];
  }
  m.sqrtg = sqrt(det / (chi * chi * chi));
}

// physical metric from the conformal one: gamma_ij = gt_ij/chi, gamma^ij = chi gt^ij,
// sqrt(gamma) = sqrt(det gt / chi^3)
struct Metric {
  double gd[6], gu[6], sqrtg;
};

__device__ __forceinline__ void metric_from(const double gt[6], double chi, Metric& m) {
  double gtu[6];
  const double det = sym_inv(gt, gtu);
  const double ic = 1.0 / chi;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    m.gd[a] = gt[a] * ic;
    m.gu[a] = gtu[a] * chi;
  }
  m.sqrtg = sqrt(det * ic * ic * ic);
}

// ------------------------------------------------------------------ stencils (Sec. 3.2)
// u points at the centre value; s is the element stride along the axis; ih = 1/h.
//
// Conditioning: the fields carry O(1) values with small variations, so the
// weighted sums of the second-derivative, upwind and dissipation stencils
// cancel to a result many orders of magnitude below the summands.  Their
// numerators are therefore summed in a fixed paired order with FMA contraction
// disabled: every rounding is then a plain IEEE add or multiply, reproducible
// on any FP64 implementation, and only the final scaling by 1/h carries a
// (relative, harmless) rounding difference.

// Loads of stencil points go through a buffer resource built from a
// wavefront-uniform base (field start plus the stencil offset, kept in SGPRs)
// and one 32-bit per-lane byte offset shared by every load of the point, so
// the hundreds of stencil loads of a point need no per-load address VGPRs.
__device__ __forceinline__ double ldf(const double* fb, uint32_t voff) {
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)fb, 0, 0x7fffffff, 0x00020000);
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, 0, 0));
}

// One buffer resource per field and stencil: based at the stencil's lowest
// point (uniform), with the per-lane byte offset voff of the centre point and
// the position along the axis as the scalar offset (a multiple of s8 = 8 s),
// so a stencil's points share one resource and every field along an axis
// shares the scalar offsets.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_at(const double* base) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, 0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ double ld_at(__amdgpu_buffer_rsrc_t r, uint32_t voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, soff, 0));
}

// the N points fb[p + (m - lo) st], m = 0 .. N-1, into v (s8 = 8 st)
template <int N>
__device__ __forceinline__ void ld_col(const double* fb, int64_t st, int lo, uint32_t voff, int s8, double (&v)[N]) {
  const __amdgpu_buffer_rsrc_t r = rsrc_at(fb - lo * st);
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] = ld_at(r, voff, m * s8);
}

// fb: field base (uniform); s: element stride along the axis (uniform);
// voff: byte offset of the centre point; ih12 = 1/(12h), ih2_12 = 1/(12h^2)
__device__ __forceinline__ double fd1(const double* fb, int64_t s, uint32_t voff, double ih12) {
#pragma clang fp contract(off)
  const int s8 = (int)(s * 8);
  const __amdgpu_buffer_rsrc_t r = rsrc_at(fb - 2 * s);
  const double m2 = ld_at(r, voff, 0), m1 = ld_at(r, voff, s8), p1 = ld_at(r, voff, 3 * s8),
               p2 = ld_at(r, voff, 4 * s8);
  return (8.0 * (p1 - m1) - (p2 - m2)) * ih12;
}

__device__ __forceinline__ double fd2(const double* fb, int64_t s, uint32_t voff, double ih2_12) {
#pragma clang fp contract(off)
  double v[5];
  ld_col(fb, s, 2, voff, (int)(s * 8), v);
  return (16.0 * (v[3] + v[1]) - (v[4] + v[0]) - 30.0 * v[2]) * ih2_12;
}

// D_b(D_a u): the centred operator along a applied at the four b-neighbours,
// then along b
__device__ __forceinline__ double fd11(const double* fb, int64_t sa, int64_t sb, uint32_t voff, double iha12,
                                       double ihb12) {
#pragma clang fp contract(off)
  const double a1 = fd1(fb + sb, sa, voff, iha12);
  const double b1 = fd1(fb - sb, sa, voff, iha12);
  const double a2 = fd1(fb + 2 * sb, sa, voff, iha12);
  const double b2 = fd1(fb - 2 * sb, sa, voff, iha12);
  return (8.0 * (a1 - b1) - (a2 - b2)) * ihb12;
}

// beta * D^upwind u with the one-sided 4th-order stencils of Sec. 3.2:
//   beta >= 0: ( u_{+3} - 6u_{+2} + 18u_{+1} - 10u_0 - 3u_{-1})/(12h)
//   beta <  0: (-u_{-3} + 6u_{-2} - 18u_{-1} + 10u_0 + 3u_{+1})/(12h)
// (scalar offsets k s8 address u_{k-3})
__device__ __forceinline__ double fdadv(const double* fb, int64_t s, uint32_t voff, double ih12, double beta) {
#pragma clang fp contract(off)
  const int s8 = (int)(s * 8);
  const __amdgpu_buffer_rsrc_t r = rsrc_at(fb - 3 * s);
  double d;
  if (beta >= 0.0)
    d = ld_at(r, voff, 6 * s8) - 6.0 * ld_at(r, voff, 5 * s8) + 18.0 * ld_at(r, voff, 4 * s8) -
        10.0 * ld_at(r, voff, 3 * s8) - 3.0 * ld_at(r, voff, 2 * s8);
  else
    d = -ld_at(r, voff, 0) + 6.0 * ld_at(r, voff, s8) - 18.0 * ld_at(r, voff, 2 * s8) +
        10.0 * ld_at(r, voff, 3 * s8) + 3.0 * ld_at(r, voff, 4 * s8);
  return beta * (d * ih12);
}

// Kreiss-Oliger dissipation along one axis, sigma/(64h) * 6th difference
__device__ __forceinline__ double fdko(const double* fb, int64_t s, uint32_t voff, double sig_ih64) {
#pragma clang fp contract(off)
  double v[7];
  ld_col(fb, s, 3, voff, (int)(s * 8), v);
  const double q = (v[6] + v[0]) - 6.0 * (v[5] + v[1]) + 15.0 * (v[4] + v[2]) - 20.0 * v[3];
  return sig_ih64 * q;
}

}  // namespace mhd
