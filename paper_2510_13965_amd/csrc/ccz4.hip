// CCZ4 right-hand side (Sec. 2.1) at the interior points of a patch or of the
// boxes of a level.
//
// The point algebra needs well over 256 live FP64 values when evaluated in one
// piece, so it is split into kernels that each stay within the register file:
//   k_ccz4_stencil_lds  advection terms beta^k d_k u with the one-sided
//                   stencils and Kreiss-Oliger dissipation for all 22 fields
//                   (Sec. 3.2), staged through LDS; writes the 22 RHS fields;
//   k_ccz4_d2_lds   the second derivatives, contracted where possible:
//                   -1/2 gt^{mn} d_m d_n gt_ij, d_i d_j chi, d_i d_j alpha,
//                   gt^{jk} d_j d_k beta^i and d_i d_k beta^k, into 24 workspace
//                   fields, staged through LDS;
//   k_ccz4_curv     d_t At_ij, d_t Khat, d_t Theta: the Ricci split
//                   R_ij + 2 D_(i Z_j) = Rhat_ij + Rhat^chi_ij, D_i D_j alpha and
//                   the Laplacian of the lapse, matter S_ij, tau (= E), S;
//                   adds into the RHS;
//   k_ccz4_gauge    d_t gt_ij, d_t chi, d_t Ghat^i and the gauge (1+log or
//                   harmonic slicing, Gamma-freezing shift); adds into the RHS.
// The LDS-staged kernels stream (x,y) tiles along z: 64x4 on a patch, 16x16 on
// the boxes of a level.  The other two run one thread per interior point;
// 64x4 blocks put a wavefront on 64 consecutive x so every stencil row load is
// a coalesced 512-byte access and y/z neighbours come from L1/L2.
#include "dev_common.hpp"
#include "prof.hpp"

namespace mhd {

struct Ccz4Args {
  Geom g;
  mhd_params_t par;
  const double* __restrict__ U;
  const double* __restrict__ P;
  double* __restrict__ rhs;
  int nbx, nby, nbz, strip;  // tile grid (64x4 tiles) and the strip height of the tile order
  const double* __restrict__ m1P;  // closure P_ij of the three M1 species (6 s + c fields), or null
};

constexpr double kPi = 3.141592653589793;

__device__ __forceinline__ double wsym(int c) { return (c == 1 || c == 2 || c == 4) ? 2.0 : 1.0; }

struct PointIdx {
  int64_t p, sf;
  int64_t st[3];
  uint32_t voff;  // byte offset of the point within a field
  bool live;
};

// interior indices (i, j, k) -> addressing of the point
__device__ __forceinline__ PointIdx point_at(const Geom& g, int i, int j, int k) {
  PointIdx q;
  q.live = true;
  q.p = g.at(i + g.ng, j + g.ng, k + g.ng);
  q.voff = (uint32_t)(q.p * 8);
  q.sf = g.sf;
  q.st[0] = 1;
  q.st[1] = g.sy;
  q.st[2] = g.sz;
  return q;
}

__device__ __forceinline__ PointIdx point_index(const Ccz4Args& a) {
  const Geom& g = a.g;
  const TileXYZ t = tile_of_block(a.nbx, a.nby, a.nbz, a.strip);
  int i = t.bx * 64 + threadIdx.x;
  int j = t.by * 4 + threadIdx.y;
  int k = t.bz;
  const bool live = t.bx >= 0 && i < g.nx && j < g.ny;
  if (!live) i = j = k = 0;
  PointIdx q = point_at(g, i, j, k);
  q.live = live;
  return q;
}

// conformal metric, its inverse and first derivatives, Christoffels of the
// first kind c1[k][ij] = (d_i gt_kj + d_j gt_ki - d_k gt_ij)/2 and the
// contracted Christoffel computed as printed, Gt^i = gt^{ij} gt^{kl} d_l gt_jk
struct Conf {
  double gt[6], gtu[6], det, c1[3][6], Gt[3];
};

__device__ __forceinline__ void conf_point(const double* __restrict__ U, const PointIdx& q, const Geom& g, Conf& c) {
  const int64_t sf = q.sf;
#pragma unroll
  for (int a = 0; a < 6; ++a) c.gt[a] = ldf(U + (a) * sf, q.voff);
  c.det = sym_inv(c.gt, c.gtu);
  double dg[3][6];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int a = 0; a < 6; ++a) dg[d][a] = fd1(U + a * sf, q.st[d], q.voff, g.i12[d]);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) c.c1[k][sym(i, j)] = 0.5 * (dg[i][sym(k, j)] + dg[j][sym(k, i)] - dg[k][sym(i, j)]);
  double w[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) s += c.gtu[sym(k, l)] * dg[l][sym(j, k)];
    w[j] = s;
  }
  sym_mv(c.gtu, w, c.Gt);
}

// matter projections of the magnetised fluid (Sec. 2.2): E = tau + D, S_i, S_ij
struct Matter {
  double E, S[3], Sij[6], Str;
};

__device__ __forceinline__ void matter_point(const double* __restrict__ U, const double* __restrict__ P,
                                             const double* __restrict__ m1P, const PointIdx& q, const Conf& c,
                                             double chi, bool want_sij, Matter& m) {
  const int64_t sf = q.sf;
  const double ichi = 1.0 / chi;
  const double isg = 1.0 / sqrt(c.det * ichi * ichi * ichi);
  double Sf[3];  // fluid momentum (the fluid stress needs it alone)
#pragma unroll
  for (int a = 0; a < 3; ++a) Sf[a] = m.S[a] = ldf(U + ((25 + a)) * sf, q.voff) * isg;
  m.E = (ldf(U + (24) * sf, q.voff) + ldf(U + (22) * sf, q.voff)) * isg;
  if (m1P) {
    // radiation: E += sum E_nu, S_i += sum F_i (the stress is added below)
#pragma unroll 1
    for (int sp = 0; sp < 3; ++sp) {
      m.E += ldf(U + (32 + 4 * sp) * sf, q.voff) * isg;
#pragma unroll
      for (int a = 0; a < 3; ++a) m.S[a] += ldf(U + (33 + 4 * sp + a) * sf, q.voff) * isg;
    }
  }
  if (!want_sij) return;
  double gd[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) gd[a] = c.gt[a] * ichi;
  const double v[3] = {ldf(P + (3) * sf, q.voff), ldf(P + (4) * sf, q.voff), ldf(P + (5) * sf, q.voff)};
  const double B[3] = {ldf(U + (28) * sf, q.voff) * isg, ldf(U + (29) * sf, q.voff) * isg, ldf(U + (30) * sf, q.voff) * isg};
  double vd[3], Bd[3];
  sym_mv(gd, v, vd);
  sym_mv(gd, B, Bd);
  const double B2 = B[0] * Bd[0] + B[1] * Bd[1] + B[2] * Bd[2];
  const double Bv = B[0] * vd[0] + B[1] * vd[1] + B[2] * vd[2];
  const double W = ldf(P + (6) * sf, q.voff), pr = ldf(P + (2) * sf, q.voff);
  const double iW2 = 1.0 / (W * W);
  const double iso = pr + 0.5 * iW2 * B2 + 0.5 * Bv * Bv;
  m.Str = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const int a = sym(i, j);
      m.Sij[a] = 0.5 * (vd[i] * Sf[j] + vd[j] * Sf[i]) + gd[a] * iso - iW2 * Bd[i] * Bd[j] -
                 0.5 * Bv * (Bd[i] * vd[j] + Bd[j] * vd[i]);
      if (m1P) m.Sij[a] += ldf(m1P + a * sf, q.voff) + ldf(m1P + (6 + a) * sf, q.voff) + ldf(m1P + (12 + a) * sf, q.voff);
      m.Str += wsym(a) * c.gtu[a] * m.Sij[a];
    }
  m.Str *= chi;
}



// ------------------------------------------------------------------ advection + KO, LDS-staged
//
// The same stencils evaluated from staged values: a block owns a 64x4 (x,y)
// tile and streams it through a chunk of z planes.  Each thread keeps the
// seven z-values of its column in registers; the current plane, with its
// three-point x and y halos, sits in LDS (double-buffered, one barrier per
// plane), and the next plane's values are loaded while the current one is
// processed.  About three global loads per point and field (own column, halo)
// replace the ~19 stencil loads of the per-point kernel.  The arithmetic is the per-point kernel's, operation
// for operation, so both give identical bits.

constexpr int kStTX = 64, kStTY = 4, kStH = 3;  // patch tiles; halo of the 7-point stencils
constexpr int kLvT = kLevelLdsTile;             // level tiles are kLvT x kLvT

// beta * D^upwind u from the seven values v[m] = u_{m-3} (as fdadv)
__device__ __forceinline__ double adv7(const double v[7], double ih12, double beta) {
#pragma clang fp contract(off)
  double d;
  if (beta >= 0.0)
    d = v[6] - 6.0 * v[5] + 18.0 * v[4] - 10.0 * v[3] - 3.0 * v[2];
  else
    d = -v[0] + 6.0 * v[1] - 18.0 * v[2] + 10.0 * v[3] + 3.0 * v[4];
  return beta * (d * ih12);
}

// Kreiss-Oliger term from the seven values (as fdko)
__device__ __forceinline__ double ko7(const double v[7], double sig_ih64) {
#pragma clang fp contract(off)
  const double q = (v[6] + v[0]) - 6.0 * (v[5] + v[1]) + 15.0 * (v[4] + v[2]) - 20.0 * v[3];
  return sig_ih64 * q;
}

constexpr int kStZC = 8;  // z planes per block

struct StencilTile {
  int nbx, nby, nzc;  // tiles in x, y and z chunks of kStZC planes
};

// one TX x TY tile through one chunk of z planes (the whole block calls this)
template <int TX, int TY>
__device__ __forceinline__ void stencil_lds_tile(const Geom& g, const mhd_params_t& par, const double* __restrict__ U,
                                                 double* __restrict__ rhs, int tbx, int tby, int tbz,
                                                 double (&lds)[2][TY + 2 * kStH][TX + 2 * kStH]) {
#pragma clang fp contract(off)
  constexpr int NXH = 2 * kStH * TY, NH = NXH + 2 * kStH * TX;  // x-halo and all halo slots
  static_assert(NH <= 512, "two halo rounds per thread");
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
  const int i = tbx * TX + tx, j = tby * TY + ty;
  const int z0 = tbz * kStZC, nzb = min(kStZC, g.nz - z0);  // planes z0 .. z0+nzb-1 of the interior
  const bool col = i < g.nx + g.ng && j < g.ny + g.ng;      // the column exists in the padded patch
  const bool live = i < g.nx && j < g.ny;
  const int64_t sf = g.sf, sz = g.sz;
  const int64_t pc = col ? g.at(i + g.ng, j + g.ng, g.ng + z0) : 0;  // column at plane z0
  const double sko[3] = {par.sigma_ko * (1.0 / 64.0) * g.idx[0], par.sigma_ko * (1.0 / 64.0) * g.idx[1],
                         par.sigma_ko * (1.0 / 64.0) * g.idx[2]};
  // the shift of the chunk's planes
  double bta[3][kStZC];
#pragma unroll
  for (int zz = 0; zz < kStZC; ++zz)
#pragma unroll
    for (int d = 0; d < 3; ++d) bta[d][zz] = (live && zz < nzb) ? U[(int64_t)(19 + d) * sf + pc + zz * sz] : 0.0;
  // halo slots: x-halo (3 left, 3 right, TY rows), then y-halo (3 below, 3 above, TX columns)
  int hx[2], hy[2];
  bool hok[2];
  int64_t hp[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int h = tid + 256 * r;
    int lx = 0, ly = 0;
    if (h < NXH) {
      const int side = h / (kStH * TY), rr = h % (kStH * TY);
      ly = kStH + rr / kStH;
      lx = side == 0 ? rr % kStH : kStH + TX + rr % kStH;
    } else if (h < NH) {
      const int q = h - NXH, side = q / (kStH * TX), rr = q % (kStH * TX);
      lx = kStH + rr % TX;
      ly = side == 0 ? rr / TX : kStH + TY + rr / TX;
    }
    const int gi = tbx * TX + lx - kStH, gj = tby * TY + ly - kStH;  // interior indices
    hx[r] = lx;
    hy[r] = ly;
    hok[r] = h < NH && gi >= -g.ng && gj >= -g.ng && gi < g.nx + g.ng && gj < g.ny + g.ng;
    hp[r] = hok[r] ? g.at(gi + g.ng, gj + g.ng, g.ng + z0) : 0;
  }
  // software pipeline: the values of the next plane (the column's plane z+4
  // and the halo of plane z+1, or the first planes of the next field) are
  // loaded while the current plane is processed
  double qi[7], hn[2], qn = 0.0;
#pragma unroll
  for (int m = 0; m < 7; ++m) qi[m] = col ? U[pc + (m - 3) * sz] : 0.0;
#pragma unroll
  for (int r = 0; r < 2; ++r) hn[r] = hok[r] ? U[hp[r]] : 0.0;
  int buf = 0;
  for (int f = 0; f < 22; ++f) {
    const double* __restrict__ u = U + (int64_t)f * sf;
    double q[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) q[m] = qi[m];
#pragma unroll
    for (int zz = 0; zz < kStZC; ++zz) {
      if (zz < nzb) {  // uniform over the block
        if (zz > 0) {  // the column queue moves to planes z-3 .. z+3
#pragma unroll
          for (int m = 0; m < 6; ++m) q[m] = q[m + 1];
          q[6] = qn;
        }
        lds[buf][ty + kStH][tx + kStH] = q[3];
#pragma unroll
        for (int r = 0; r < 2; ++r)
          if (hok[r]) lds[buf][hy[r]][hx[r]] = hn[r];
        if (zz + 1 < nzb) {
          qn = col ? u[pc + (zz + 4) * sz] : 0.0;
#pragma unroll
          for (int r = 0; r < 2; ++r) hn[r] = hok[r] ? u[hp[r] + (zz + 1) * sz] : 0.0;
        } else if (f + 1 < 22) {
          const double* __restrict__ un = u + sf;
#pragma unroll
          for (int m = 0; m < 7; ++m) qi[m] = col ? un[pc + (m - 3) * sz] : 0.0;
#pragma unroll
          for (int r = 0; r < 2; ++r) hn[r] = hok[r] ? un[hp[r]] : 0.0;
        }
        __syncthreads();
        if (live) {
          double vx[7], vy[7];
#pragma unroll
          for (int m = 0; m < 7; ++m) {
            vx[m] = lds[buf][ty + kStH][tx + m];
            vy[m] = lds[buf][ty + m][tx + kStH];
          }
          double sacc = 0.0;
          sacc += adv7(vx, g.i12[0], bta[0][zz]) + ko7(vx, sko[0]);
          sacc += adv7(vy, g.i12[1], bta[1][zz]) + ko7(vy, sko[1]);
          sacc += adv7(q, g.i12[2], bta[2][zz]) + ko7(q, sko[2]);
          rhs[(int64_t)f * sf + pc + zz * sz] = sacc;
        }
        buf ^= 1;
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_ccz4_stencil_lds(Ccz4Args a, StencilTile T) {
  __shared__ double lds[2][kStTY + 2 * kStH][kStTX + 2 * kStH];
  const TileXYZ t = tile_of_block(T.nbx, T.nby, T.nzc, a.strip);
  if (t.bx < 0) return;  // whole block
  stencil_lds_tile<kStTX, kStTY>(a.g, a.par, a.U, a.rhs, t.bx, t.by, t.bz, lds);
}

// level: one block per tile of the boxes' LDS tile space (16x16 tiles, so
// boxes of edge 16..64 keep most lanes busy), in XCD-contiguous ranges
__device__ __forceinline__ bool level_lds_tile(const LevelArgs& L, int& box, TileXYZ& t) {
  const int64_t per = (L.ntile_lds + 7) / 8;
  const int64_t id = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (id >= L.ntile_lds) return false;
  int lo = 0, hi = L.nboxes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L.boxes[mid].t0_lds <= id) lo = mid;
    else hi = mid - 1;
  }
  const BoxDev& B = L.boxes[lo];
  box = lo;
  t = tile_of_index((int)(id - B.t0_lds), B.ntx_lds, B.nty_lds, B.nzc_lds, L.strip);
  return true;
}

template <bool IMEX>
__global__ void __launch_bounds__(256) k_ccz4_stencil_lds_lv(LevelArgs L) {
  __shared__ double lds[2][kLvT + 2 * kStH][kLvT + 2 * kStH];
  int b;
  TileXYZ t;
  if (!level_lds_tile(L, b, t)) return;  // whole block
  const BoxDev& B = L.boxes[b];
  stencil_lds_tile<kLvT, kLvT>(B.g, L.par, L.src ? B.Us : B.U, level_rhs<IMEX>(B, L), t.bx, t.by, t.bz, lds);
}

// ------------------------------------------------------------------ second derivatives

// workspace layout (field offsets, stride sf): 0-5 -1/2 gt^{mn} d_m d_n gt_ij,
// 6-11 d_i d_j chi, 12-17 d_i d_j alpha, 18-20 gt^{jk} d_j d_k beta^i,
// 21-23 d_i d_k beta^k
constexpr int kD2Fields = 24;

// -1/2 gt^{mn} d_m d_n gt_ij from the six second derivatives of one gt_ij
// (fixed evaluation order, no contraction: both d2 kernels give the same bits)
__device__ __forceinline__ double d2_gt_contract(const double gtu[6], double xx, double yy, double zz, double xy,
                                                 double xz, double yz) {
#pragma clang fp contract(off)
  double r = -0.5 * (gtu[0] * xx + gtu[3] * yy + gtu[5] * zz);
  r -= gtu[1] * xy;
  r -= gtu[2] * xz;
  r -= gtu[4] * yz;
  return r;
}

// gt^{jk} d_j d_k beta^i from the six second derivatives v (symmetric storage)
__device__ __forceinline__ double d2_beta_lap(const double gtu[6], const double v[6]) {
#pragma clang fp contract(off)
  double lap = 0.0;
#pragma unroll
  for (int b = 0; b < 6; ++b) lap += wsym(b) * gtu[b] * v[b];
  return lap;
}


// ------------------------------------------------------------------ second derivatives, LDS-staged
//
// The same derivatives and contractions from staged values: a block owns a
// 64x4 (x,y) tile and streams it along z, field by field, staging each plane
// with a two-point halo (corners included) in LDS, two planes ahead of the
// output plane.  When plane z' is staged the thread forms D_x u and D_y u at
// its point (queued over five planes, for the xz and yz mixed derivatives),
// and the in-plane d_xx, d_yy and d_xy (held two steps, until the z
// neighbours are staged); d_zz comes from a five-plane queue of u.  About
// four global loads per point and field replace the ~63 of the per-point
// kernel.  Every derivative is the per-point kernel's expression, operation
// for operation.

constexpr int kD2ZC = 8, kD2H = 2;  // z planes per block; halo of the 5-point stencils

struct D2Tile {
  int nbx, nby, nzc;  // tiles in x, y and z chunks of kD2ZC planes
};

// centred first derivative from five values v[m] = u_{m-2} (as fd1)
__device__ __forceinline__ double d1of5(double m2, double m1, double p1, double p2, double ih12) {
#pragma clang fp contract(off)
  return (8.0 * (p1 - m1) - (p2 - m2)) * ih12;
}
// centred second derivative from five values (as fd2)
__device__ __forceinline__ double d2of5(double m2, double m1, double c, double p1, double p2, double ih2_12) {
#pragma clang fp contract(off)
  return (16.0 * (p1 + m1) - (p2 + m2) - 30.0 * c) * ih2_12;
}

// one TX x TY tile through one chunk of z planes (the whole block calls this)
template <int TX, int TY>
__device__ __forceinline__ void d2_lds_tile(const Geom& g, const double* __restrict__ U, double* __restrict__ W,
                                            int tbx, int tby, int tbz,
                                            double (&lds)[2][TY + 2 * kD2H][TX + 2 * kD2H]) {
#pragma clang fp contract(off)
  constexpr int LX = TX + 2 * kD2H, NH = LX * (TY + 2 * kD2H) - TX * TY;  // halo slots per plane
  static_assert(NH <= 512, "two halo rounds per thread");
  const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
  const int i = tbx * TX + tx, j = tby * TY + ty;
  const int z0 = tbz * kD2ZC, nzb = min(kD2ZC, g.nz - z0);
  const bool col = i < g.nx + g.ng && j < g.ny + g.ng;
  const bool live = i < g.nx && j < g.ny;
  const int64_t sf = g.sf, sz = g.sz;
  const int64_t pc = col ? g.at(i + g.ng, j + g.ng, g.ng + z0) : 0;  // column at plane z0
  int hx[2], hy[2];
  bool hok[2];
  int64_t hp[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int h = tid + 256 * r;
    int lx = 0, ly = 0;
    if (h < 2 * LX) {
      ly = h / LX;
      lx = h % LX;
    } else if (h < 4 * LX) {
      ly = kD2H + TY + (h - 2 * LX) / LX;
      lx = (h - 2 * LX) % LX;
    } else if (h < NH) {
      const int q = h - 4 * LX, c = q % 4;
      ly = kD2H + q / 4;
      lx = c < 2 ? c : TX + c;
    }
    const int gi = tbx * TX + lx - kD2H, gj = tby * TY + ly - kD2H;
    hx[r] = lx;
    hy[r] = ly;
    hok[r] = h < NH && gi >= -g.ng && gj >= -g.ng && gi < g.nx + g.ng && gj < g.ny + g.ng;
    hp[r] = hok[r] ? g.at(gi + g.ng, gj + g.ng, g.ng + z0) : 0;
  }
  const int nst = nzb + 4;  // staged planes z0-2 .. z0+nzb+1
  // fields in the order of the per-point kernel: gt_ij, chi, alpha, beta^i
  const int fld[11] = {0, 1, 2, 3, 4, 5, 12, 18, 19, 20, 21};
  // pipeline: own and halo values of the next staged plane
  double own = col ? U[pc - 2 * sz] : 0.0, hv[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) hv[r] = hok[r] ? U[hp[r] - 2 * sz] : 0.0;
  int buf = 0;
#pragma unroll 1
  for (int fi = 0; fi < 11; ++fi) {
    const double* __restrict__ u = U + (int64_t)fld[fi] * sf;
    double qu[5] = {0, 0, 0, 0, 0}, qx[5] = {0, 0, 0, 0, 0}, qy[5] = {0, 0, 0, 0, 0};
    double hxx[3] = {0, 0, 0}, hyy[3] = {0, 0, 0}, hxy[3] = {0, 0, 0};
#pragma unroll 1
    for (int st = 0; st < nst; ++st) {
      const int zs = st - 2;  // staged plane, relative to z0
      lds[buf][ty + kD2H][tx + kD2H] = own;
#pragma unroll
      for (int r = 0; r < 2; ++r)
        if (hok[r]) lds[buf][hy[r]][hx[r]] = hv[r];
#pragma unroll
      for (int m = 0; m < 4; ++m) qu[m] = qu[m + 1];
      qu[4] = own;
      if (st + 1 < nst) {
        own = col ? u[pc + (int64_t)(zs + 1) * sz] : 0.0;
#pragma unroll
        for (int r = 0; r < 2; ++r) hv[r] = hok[r] ? u[hp[r] + (int64_t)(zs + 1) * sz] : 0.0;
      } else if (fi + 1 < 11) {
        const double* __restrict__ un = U + (int64_t)fld[fi + 1] * sf;
        own = col ? un[pc - 2 * sz] : 0.0;
#pragma unroll
        for (int r = 0; r < 2; ++r) hv[r] = hok[r] ? un[hp[r] - 2 * sz] : 0.0;
      }
      __syncthreads();
      if (live) {
        const double(*L)[LX] = lds[buf];
        const int cy = ty + kD2H, cx = tx + kD2H;
        // D_x u and D_y u at the staged plane
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          qx[m] = qx[m + 1];
          qy[m] = qy[m + 1];
        }
        qx[4] = d1of5(L[cy][cx - 2], L[cy][cx - 1], L[cy][cx + 1], L[cy][cx + 2], g.i12[0]);
        qy[4] = d1of5(L[cy - 2][cx], L[cy - 1][cx], L[cy + 1][cx], L[cy + 2][cx], g.i12[1]);
        // in-plane second derivatives of the staged plane, held two steps
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          hxx[m] = hxx[m + 1];
          hyy[m] = hyy[m + 1];
          hxy[m] = hxy[m + 1];
        }
        hxx[2] = d2of5(L[cy][cx - 2], L[cy][cx - 1], L[cy][cx], L[cy][cx + 1], L[cy][cx + 2], g.i12s[0]);
        hyy[2] = d2of5(L[cy - 2][cx], L[cy - 1][cx], L[cy][cx], L[cy + 1][cx], L[cy + 2][cx], g.i12s[1]);
        {
          const double a1 = d1of5(L[cy + 1][cx - 2], L[cy + 1][cx - 1], L[cy + 1][cx + 1], L[cy + 1][cx + 2], g.i12[0]);
          const double b1 = d1of5(L[cy - 1][cx - 2], L[cy - 1][cx - 1], L[cy - 1][cx + 1], L[cy - 1][cx + 2], g.i12[0]);
          const double a2 = d1of5(L[cy + 2][cx - 2], L[cy + 2][cx - 1], L[cy + 2][cx + 1], L[cy + 2][cx + 2], g.i12[0]);
          const double b2 = d1of5(L[cy - 2][cx - 2], L[cy - 2][cx - 1], L[cy - 2][cx + 1], L[cy - 2][cx + 2], g.i12[0]);
          hxy[2] = (8.0 * (a1 - b1) - (a2 - b2)) * g.i12[1];
        }
        if (st >= 4) {  // output plane z = zs - 2
          const int64_t po = pc + (int64_t)(zs - 2) * sz;
          const double xx = hxx[0], yy = hyy[0], xy = hxy[0];
          const double zz = d2of5(qu[0], qu[1], qu[2], qu[3], qu[4], g.i12s[2]);
          const double xz = (8.0 * (qx[3] - qx[1]) - (qx[4] - qx[0])) * g.i12[2];
          const double yz = (8.0 * (qy[3] - qy[1]) - (qy[4] - qy[0])) * g.i12[2];
          double* __restrict__ Wp = W + po;
          if (fi == 6 || fi == 7) {  // chi, alpha: 6 values each
            double* o = Wp + (int64_t)(6 + 6 * (fi - 6)) * sf;
            o[0 * sf] = xx;
            o[1 * sf] = xy;
            o[2 * sf] = xz;
            o[3 * sf] = yy;
            o[4 * sf] = yz;
            o[5 * sf] = zz;
          } else {
            double gt[6], gtu[6];
#pragma unroll
            for (int b = 0; b < 6; ++b) gt[b] = U[(int64_t)b * sf + po];
            sym_inv(gt, gtu);
            if (fi < 6) {
              Wp[(int64_t)fi * sf] = d2_gt_contract(gtu, xx, yy, zz, xy, xz, yz);
            } else {  // beta^ci
              const int ci = fi - 8;
              const double v[6] = {xx, xy, xz, yy, yz, zz};
              Wp[(int64_t)(18 + ci) * sf] = d2_beta_lap(gtu, v);
#pragma unroll
              for (int jj = 0; jj < 3; ++jj) {
                const double add = v[sym(jj, ci)];
                double* dv = Wp + (int64_t)(21 + jj) * sf;
                *dv = (ci == 0 ? 0.0 : *dv) + add;
              }
            }
          }
        }
      }
      buf ^= 1;
    }
  }
}

constexpr int kD2TX = 64, kD2TY = 4;  // patch tiles of the second-derivative kernel

__global__ void __launch_bounds__(256) k_ccz4_d2_lds(Ccz4Args a, double* __restrict__ W, D2Tile T) {
  __shared__ double lds[2][kD2TY + 2 * kD2H][kD2TX + 2 * kD2H];
  const TileXYZ t = tile_of_block(T.nbx, T.nby, T.nzc, a.strip);
  if (t.bx < 0) return;  // whole block
  d2_lds_tile<kD2TX, kD2TY>(a.g, a.U, W, t.bx, t.by, t.bz, lds);
}

__global__ void __launch_bounds__(256) k_ccz4_d2_lds_lv(LevelArgs L) {
  __shared__ double lds[2][kLvT + 2 * kD2H][kLvT + 2 * kD2H];
  int b;
  TileXYZ t;
  if (!level_lds_tile(L, b, t)) return;  // whole block
  const BoxDev& B = L.boxes[b];
  d2_lds_tile<kLvT, kLvT>(B.g, L.src ? B.Us : B.U, B.ws + 33 * B.g.sf, t.bx, t.by, t.bz, lds);
}

// ------------------------------------------------------------------ At_ij, Khat, Theta

__device__ __forceinline__ void ccz4_curv_at(const Ccz4Args& a, const double* __restrict__ W, const PointIdx& q) {
  const Geom& g = a.g;
  const double* __restrict__ U = a.U;
  const int64_t sf = q.sf, p = q.p;

  Conf c;
  conf_point(U, q, g, c);
  const double chi = ldf(U + (12) * sf, q.voff), Kh = ldf(U + (13) * sf, q.voff), Th = ldf(U + (14) * sf, q.voff);
  const double Gh[3] = {ldf(U + (15) * sf, q.voff), ldf(U + (16) * sf, q.voff), ldf(U + (17) * sf, q.voff)};
  const double alp = ldf(U + (18) * sf, q.voff);
  const double ichi = 1.0 / chi;
  double Z[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) Z[i] = 0.5 * chi * (Gh[i] - c.Gt[i]);

  double dchi[3], dalp[3], ddchi[6], ddalp[6];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    dchi[d] = fd1(U + 12 * sf, q.st[d], q.voff, g.i12[d]);
    dalp[d] = fd1(U + 18 * sf, q.st[d], q.voff, g.i12[d]);
  }
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    ddchi[b] = ldf(W + (6 + b) * sf, q.voff);
    ddalp[b] = ldf(W + (12 + b) * sf, q.voff);
  }
  // raised gradients: Gt^k_ij d_k f = c1[l][ij] (gt^{lk} d_k f)
  double uchi[3], ualp[3];
  sym_mv(c.gtu, dchi, uchi);
  sym_mv(c.gtu, dalp, ualp);

  // Rs_ij = Rhat_ij + Rhat^chi_ij
  double Rs[6];
  {
    // Q[k][n][i] = gt^{mn} Gamma^k_{mi},  Gamma^k_{mi} = gt^{kl} c1[l][mi]
    double Q[3][3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double c2k[6];
#pragma unroll
      for (int b = 0; b < 6; ++b)
        c2k[b] = c.gtu[sym(k, 0)] * c.c1[0][b] + c.gtu[sym(k, 1)] * c.c1[1][b] + c.gtu[sym(k, 2)] * c.c1[2][b];
#pragma unroll
      for (int n = 0; n < 3; ++n)
#pragma unroll
        for (int i = 0; i < 3; ++i)
          Q[k][n][i] = c.gtu[sym(0, n)] * c2k[sym(0, i)] + c.gtu[sym(1, n)] * c2k[sym(1, i)] +
                       c.gtu[sym(2, n)] * c2k[sym(2, i)];
    }
    double trchi = 0.0;  // gt^{km}(d_k d_m chi - 3/(2chi) d_k chi d_m chi) - Ghat^k d_k chi
#pragma unroll
    for (int b = 0; b < 6; ++b) trchi += wsym(b) * c.gtu[b] * ddchi[b];
    trchi -= 1.5 * ichi * (dchi[0] * uchi[0] + dchi[1] * uchi[1] + dchi[2] * uchi[2]);
    trchi -= Gh[0] * dchi[0] + Gh[1] * dchi[1] + Gh[2] * dchi[2];

    double dGh[3][3];  // d_d Ghat^k
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int k = 0; k < 3; ++k) dGh[d][k] = fd1(U + (15 + k) * sf, q.st[d], q.voff, g.i12[d]);

#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        const int b = sym(i, j);
        // -1/2 gt^{mn} d_m d_n gt_ij
        double r = ldf(W + b * sf, q.voff);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          r += 0.5 * (c.gt[sym(k, i)] * dGh[j][k] + c.gt[sym(k, j)] * dGh[i][k]);  // gt_k(i d_j) Ghat^k
          r += 0.5 * Gh[k] * (c.c1[i][sym(j, k)] + c.c1[j][sym(i, k)]);          // Ghat^k Gt_(ij)k
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int n = 0; n < 3; ++n)
            r += Q[k][n][i] * (c.c1[j][sym(k, n)] + c.c1[k][sym(n, j)]) + Q[k][n][j] * c.c1[i][sym(k, n)];
        // chi Rhat^chi_ij
        double rc = 0.5 * ddchi[b] - 0.25 * ichi * dchi[i] * dchi[j] + 0.5 * c.gt[b] * trchi;
        rc -= 0.5 * (c.c1[0][b] * uchi[0] + c.c1[1][b] * uchi[1] + c.c1[2][b] * uchi[2]);
#pragma unroll
        for (int k = 0; k < 3; ++k) rc += ichi * Z[k] * (c.gt[sym(k, i)] * dchi[j] + c.gt[sym(k, j)] * dchi[i]);
        Rs[b] = r + rc * ichi;
      }
  }
  double Rtr = 0.0;  // R + 2 D_i Z^i = chi gt^{ij} Rs_ij
#pragma unroll
  for (int b = 0; b < 6; ++b) Rtr += wsym(b) * c.gtu[b] * Rs[b];
  Rtr *= chi;

  // D_i D_j alpha with the physical Christoffels
  double DDa[6];
  {
    const double dad = dalp[0] * uchi[0] + dalp[1] * uchi[1] + dalp[2] * uchi[2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        const int b = sym(i, j);
        DDa[b] = ddalp[b] - (c.c1[0][b] * ualp[0] + c.c1[1][b] * ualp[1] + c.c1[2][b] * ualp[2]) +
                 0.5 * ichi * (dalp[i] * dchi[j] + dalp[j] * dchi[i] - c.gt[b] * dad);
      }
  }
  // Laplacian as printed: chi gt^{ij} d_i d_j alpha - chi Gt^k d_k alpha - 1/2 gt^{ij} d_i alpha d_j chi
  double lapA = 0.0;
#pragma unroll
  for (int b = 0; b < 6; ++b) lapA += wsym(b) * c.gtu[b] * ddalp[b];
  lapA = chi * lapA - chi * (c.Gt[0] * dalp[0] + c.Gt[1] * dalp[1] + c.Gt[2] * dalp[2]) -
         0.5 * (dalp[0] * uchi[0] + dalp[1] * uchi[1] + dalp[2] * uchi[2]);

  Matter m;
  const bool couple = (a.par.flags & MHD_COUPLE_MATTER) != 0;
  if (couple) {
    matter_point(U, a.P, a.m1P, q, c, chi, true, m);
  } else {
    m.E = m.Str = 0.0;
#pragma unroll
    for (int b = 0; b < 6; ++b) m.Sij[b] = 0.0;
  }

  double At[6], Amix[3][3];
#pragma unroll
  for (int b = 0; b < 6; ++b) At[b] = ldf(U + ((6 + b)) * sf, q.voff);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Amix[i][j] = c.gtu[sym(i, 0)] * At[sym(0, j)] + c.gtu[sym(i, 1)] * At[sym(1, j)] + c.gtu[sym(i, 2)] * At[sym(2, j)];
  const double trA = Amix[0][0] + Amix[1][1] + Amix[2][2];
  double AA = 0.0;  // At_ij At^ij = At^i_j At^j_i
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) AA += Amix[i][j] * Amix[j][i];

  double db[3][3];  // d_d beta^k
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int k = 0; k < 3; ++k) db[d][k] = fd1(U + (19 + k) * sf, q.st[d], q.voff, g.i12[d]);
  const double divb = db[0][0] + db[1][1] + db[2][2];

  double X[6], trX = 0.0;
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    X[b] = alp * (Rs[b] - 8.0 * kPi * m.Sij[b]) - DDa[b];
    trX += wsym(b) * c.gtu[b] * X[b];
  }
  double* __restrict__ R = a.rhs + p;
  const double kc = a.par.kappa_c;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const int b = sym(i, j);
      double la = -2.0 / 3.0 * At[b] * divb - alp / 3.0 * kc * c.gt[b] * trA + chi * (X[b] - 1.0 / 3.0 * c.gt[b] * trX) +
                  alp * Kh * At[b];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        la += At[sym(i, k)] * db[j][k] + At[sym(k, j)] * db[i][k];
        la -= 2.0 * alp * At[sym(i, k)] * Amix[k][j];
      }
      R[(6 + b) * sf] += la;
    }
  const double Kf = Kh + 2.0 * Th;
  const double Zda = Z[0] * dalp[0] + Z[1] * dalp[1] + Z[2] * dalp[2];
  R[13 * sf] += -lapA + alp * (1.0 / 3.0 * Kf * Kf + AA + 4.0 * kPi * (m.E + m.Str) +
                               a.par.kappa_z * (1.0 - a.par.kappa_2) * Th) + 2.0 * Zda;
  R[14 * sf] += 0.5 * alp * (Rtr + 2.0 / 3.0 * Kh * Kh + 2.0 / 3.0 * Th * (Kh - 2.0 * Th) - AA) - Zda -
                alp * (8.0 * kPi * m.E + a.par.kappa_z * (2.0 + a.par.kappa_2) * Th);
}

// ------------------------------------------------------------------ gt_ij, chi, Ghat^i, gauge

__device__ __forceinline__ void ccz4_gauge_at(const Ccz4Args& a, const double* __restrict__ W, const PointIdx& q) {
  const Geom& g = a.g;
  const double* __restrict__ U = a.U;
  const int64_t sf = q.sf, p = q.p;

  Conf c;
  conf_point(U, q, g, c);
  const double chi = ldf(U + (12) * sf, q.voff), Kh = ldf(U + (13) * sf, q.voff), Th = ldf(U + (14) * sf, q.voff);
  const double Gh[3] = {ldf(U + (15) * sf, q.voff), ldf(U + (16) * sf, q.voff), ldf(U + (17) * sf, q.voff)};
  const double alp = ldf(U + (18) * sf, q.voff);
  const double beta[3] = {ldf(U + (19) * sf, q.voff), ldf(U + (20) * sf, q.voff), ldf(U + (21) * sf, q.voff)};
  const double ichi = 1.0 / chi;
  const double Kf = Kh + 2.0 * Th;

  double At[6], Au[6];
#pragma unroll
  for (int b = 0; b < 6; ++b) At[b] = ldf(U + ((6 + b)) * sf, q.voff);
  double trA = 0.0;
  {
    double Amix[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Amix[i][j] = c.gtu[sym(i, 0)] * At[sym(0, j)] + c.gtu[sym(i, 1)] * At[sym(1, j)] + c.gtu[sym(i, 2)] * At[sym(2, j)];
    trA = Amix[0][0] + Amix[1][1] + Amix[2][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j)
        Au[sym(i, j)] = Amix[i][0] * c.gtu[sym(0, j)] + Amix[i][1] * c.gtu[sym(1, j)] + Amix[i][2] * c.gtu[sym(2, j)];
  }

  double db[3][3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int k = 0; k < 3; ++k) db[d][k] = fd1(U + (19 + k) * sf, q.st[d], q.voff, g.i12[d]);
  const double divb = db[0][0] + db[1][1] + db[2][2];
  double* __restrict__ R = a.rhs + p;

  // d_t gt_ij
  {
    const double lndet = log(c.det);
    const double kc = a.par.kappa_c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        const int b = sym(i, j);
        double lg = -2.0 / 3.0 * c.gt[b] * divb - 2.0 * alp * (At[b] - 1.0 / 3.0 * c.gt[b] * trA) -
                    alp / 3.0 * kc * c.gt[b] * lndet;
#pragma unroll
        for (int k = 0; k < 3; ++k) lg += c.gt[sym(i, k)] * db[j][k] + c.gt[sym(k, j)] * db[i][k];
        R[b * sf] += lg;
      }
  }
  // d_t chi
  R[12 * sf] += 2.0 / 3.0 * chi * (alp * Kf - divb);

  // d_t Ghat^i
  {
    double dchi[3], dalp[3], dKh[3], dTh[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      dchi[d] = fd1(U + 12 * sf, q.st[d], q.voff, g.i12[d]);
      dKh[d] = fd1(U + 13 * sf, q.st[d], q.voff, g.i12[d]);
      dTh[d] = fd1(U + 14 * sf, q.st[d], q.voff, g.i12[d]);
      dalp[d] = fd1(U + 18 * sf, q.st[d], q.voff, g.i12[d]);
    }
    double Sm[3] = {0.0, 0.0, 0.0};
    if (a.par.flags & MHD_COUPLE_MATTER) {
      Matter m;
      matter_point(U, a.P, a.m1P, q, c, chi, false, m);
      Sm[0] = m.S[0];
      Sm[1] = m.S[1];
      Sm[2] = m.S[2];
    }
    double Auda[3], Audchi[3], vK[3], vT[3], va[3], vS[3];
    sym_mv(Au, dalp, Auda);
    sym_mv(Au, dchi, Audchi);
    sym_mv(c.gtu, dKh, vK);
    sym_mv(c.gtu, dTh, vT);
    sym_mv(c.gtu, dalp, va);
    sym_mv(c.gtu, Sm, vS);
    double lapb[3], ddivb[3];  // gt^{jk} d_j d_k beta^i, d_i d_k beta^k
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      lapb[i] = ldf(W + (18 + i) * sf, q.voff);
      ddivb[i] = ldf(W + (21 + i) * sf, q.voff);
    }
    double gddivb[3];
    sym_mv(c.gtu, ddivb, gddivb);
    const double zfac = a.par.kappa_z + 2.0 / 3.0 * Kf;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      // Gt^i_jk At^jk with Gt^i_jk = gt^{il} c1[l][jk]
      double t0 = 0.0;
#pragma unroll
      for (int b = 0; b < 6; ++b)
        t0 += wsym(b) * (c.gtu[sym(i, 0)] * c.c1[0][b] + c.gtu[sym(i, 1)] * c.c1[1][b] + c.gtu[sym(i, 2)] * c.c1[2][b]) *
              Au[b];
      const double Zi = 0.5 * chi * (Gh[i] - c.Gt[i]);
      const double r = -(Gh[0] * db[0][i] + Gh[1] * db[1][i] + Gh[2] * db[2][i]) + 2.0 / 3.0 * Gh[i] * divb + lapb[i] +
                       1.0 / 3.0 * gddivb[i] - 2.0 * Auda[i];
      const double t1 = t0 - 1.5 * ichi * Audchi[i] - 2.0 / 3.0 * vK[i] - 8.0 * kPi * vS[i];
      const double t2 = -(1.0 / 3.0 * vT[i] + Th / alp * va[i]) - ichi * Zi * zfac;
      R[(15 + i) * sf] += r + 2.0 * alp * (t1 + t2);
    }
  }
  // gauge
  const double falpha = (a.par.f_alpha_kind == MHD_FALPHA_HARMONIC) ? 0.5 * alp : 1.0;
  R[18 * sf] += -2.0 * alp * falpha * Kh;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    R[(19 + i) * sf] += 0.75 * a.par.f_beta * Gh[i] - a.par.eta * (beta[i] - a.par.beta0[i]);
}

// ------------------------------------------------------------------ kernels

__global__ void __launch_bounds__(256) k_ccz4_curv(Ccz4Args a, const double* __restrict__ W) {
  const PointIdx q = point_index(a);
  if (!q.live) return;
  ccz4_curv_at(a, W, q);
}

template <bool IMEX>
__global__ void __launch_bounds__(256) k_ccz4_curv_lv(LevelArgs L) {
  for_each_level_point(L, kRegionInterior, [&](const BoxDev& B, int i, int j, int k, bool live) {
    if (!live) return;
    const Ccz4Args a{B.g, L.par, L.src ? B.Us : B.U, B.P, level_rhs<IMEX>(B, L), 0, 0, 0, 0, L.m1 ? B.ws_m1 : nullptr};
    ccz4_curv_at(a, B.ws + 33 * B.g.sf, point_at(B.g, i, j, k));
  });
}

__global__ void __launch_bounds__(256) k_ccz4_gauge(Ccz4Args a, const double* __restrict__ W) {
  const PointIdx q = point_index(a);
  if (!q.live) return;
  ccz4_gauge_at(a, W, q);
}

template <bool IMEX>
__global__ void __launch_bounds__(256) k_ccz4_gauge_lv(LevelArgs L) {
  for_each_level_point(L, kRegionInterior, [&](const BoxDev& B, int i, int j, int k, bool live) {
    if (!live) return;
    const Ccz4Args a{B.g, L.par, L.src ? B.Us : B.U, B.P, level_rhs<IMEX>(B, L), 0, 0, 0, 0, L.m1 ? B.ws_m1 : nullptr};
    ccz4_gauge_at(a, B.ws + 33 * B.g.sf, point_at(B.g, i, j, k));
  });
}

int ccz4_workspace_fields() { return kD2Fields; }

int launch_ccz4(const Geom& g, const mhd_params_t& par, const double* U, const double* P, double* rhs, double* ws,
                int strip, const double* m1P, hipStream_t s) {
  const int nbx = (g.nx + 63) / 64, nby = (g.ny + 3) / 4, nbz = g.nz;
  Ccz4Args a{g, par, U, P, rhs, nbx, nby, nbz, strip, m1P};
  dim3 blk(64, 4, 1);
  const int nblk = nbx * nby * nbz;
  dim3 grd(8 * ((nblk + 7) / 8), 1, 1);
  {
    const StencilTile T{nbx, nby, (g.nz + kStZC - 1) / kStZC};
    Ccz4Args as = a;
    as.nbz = T.nzc;
    const int nst = nbx * nby * T.nzc;
    MHD_LAUNCH(KID_CCZ4_STENCIL, k_ccz4_stencil_lds, dim3(8 * ((nst + 7) / 8)), blk, 0, s, as, T);
  }
  {
    const D2Tile T{(g.nx + kD2TX - 1) / kD2TX, (g.ny + kD2TY - 1) / kD2TY, (g.nz + kD2ZC - 1) / kD2ZC};
    const int nd2 = T.nbx * T.nby * T.nzc;
    MHD_LAUNCH(KID_CCZ4_D2, k_ccz4_d2_lds, dim3(8 * ((nd2 + 7) / 8)), dim3(kD2TX, kD2TY, 1), 0, s, a, ws, T);
  }
  MHD_LAUNCH(KID_CCZ4_CURV, k_ccz4_curv, grd, blk, 0, s, a, (const double*)ws);
  MHD_LAUNCH(KID_CCZ4_GAUGE, k_ccz4_gauge, grd, blk, 0, s, a, (const double*)ws);
  return (int)hipGetLastError();
}

int launch_ccz4_level(const LevelArgs& L, int grid, int block, int grid_lds, hipStream_t s) {
  static_assert(kStZC == kLevelLdsZ && kD2ZC == kLevelLdsZ, "one LDS tile space for both staged kernels");
  const dim3 blk_lds(kLvT, kLvT, 1);
  if (L.slot >= 0)
    MHD_LAUNCH(KID_CCZ4_STENCIL, k_ccz4_stencil_lds_lv<true>, dim3(grid_lds), blk_lds, 0, s, L);
  else
    MHD_LAUNCH(KID_CCZ4_STENCIL, k_ccz4_stencil_lds_lv<false>, dim3(grid_lds), blk_lds, 0, s, L);
  MHD_LAUNCH(KID_CCZ4_D2, k_ccz4_d2_lds_lv, dim3(grid_lds), blk_lds, 0, s, L);
  if (L.slot >= 0) {
    MHD_LAUNCH(KID_CCZ4_CURV, k_ccz4_curv_lv<true>, dim3(grid), dim3(block), 0, s, L);
    MHD_LAUNCH(KID_CCZ4_GAUGE, k_ccz4_gauge_lv<true>, dim3(grid), dim3(block), 0, s, L);
  } else {
    MHD_LAUNCH(KID_CCZ4_CURV, k_ccz4_curv_lv<false>, dim3(grid), dim3(block), 0, s, L);
    MHD_LAUNCH(KID_CCZ4_GAUGE, k_ccz4_gauge_lv<false>, dim3(grid), dim3(block), 0, s, L);
  }
  return (int)hipGetLastError();
}

}  // namespace mhd
