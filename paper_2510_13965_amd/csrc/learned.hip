// Learned starting guess for the con2prim root solves, and its training.
//
// The recovery of App. D solves f_a(mu_+) = 0 on (0, 1/h0] and then
// f(mu) = 0 on (0, mu_+] by bracketed iterations.  Here a small MLP
// (8 -> 64 -> 64 -> 2, ReLU) maps 8 metric-invariant scalars of the state
// (log D, log q, log r^2, log calB^2, (r.calB)^2/(r^2 calB^2), log(1+q),
// log r^2/(1+q)^2, log calB^2/(1+q)) to corrections of closed-form
// approximations of log(mu_+ h0) and log(mu/mu_+) (c2p_baseline); their sum
// is a guess for mu itself.  Newton's method in FP64 polishes it for at most
// three updates, and a point is accepted only if the residual of f falls below
// 1e-12 mu, one evaluation on the far side of the corrected root shows a sign
// change within 1e-12 of it, and f_a <= 0 there.  f_a is strictly increasing
// (mu^2 (h0^2 + rbar^2) is a sum of products of nonnegative increasing
// functions of mu), so that last check places the root in (0, mu_+] without
// solving for mu_+.  Every other point goes to a queue that the bracketed
// solver then finishes, so the plain solver decides and the answer is the
// root either way.
//
// Network arithmetic: the two hidden layers run on the bf16 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation) with inputs, weights and
// hidden activations rounded to bf16 (nearest-even); biases, ReLU and the
// 64 -> 2 output layer are FP32 on the vector ALU.
//
// Data layout on the matrix cores (one wavefront = 64 points, lane l owns
// point l).  Each layer is computed transposed, H^T = W X^T, so that the
// accumulator of a 32x32 tile holds, in lane l, the column m = l%32 (a point)
// and rows 8(i/4) + 4(l/32) + i%4, i = 0..15 (hidden units).  The next layer's
// B operand needs, in lane l, column m and 8 consecutive k; instead of moving
// data between lanes, the hidden units are relabelled: B-operand index
// kappa = 16 ks + 8 g + j (g = l/32) stands for hidden unit pi(kappa), the
// unit the lane already holds in accumulator slot idx = 8 ks + j, and the
// weight matrix is loaded with its columns permuted by pi.
#include <mutex>

#include "c2p_dev.hpp"
#include "prof.hpp"

namespace mhd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// parameter block (float32): same offsets as the oracle's
constexpr int kOW1 = 0, kOB1 = 512, kOW2 = 576, kOB2 = 4672, kOW3 = 4736, kOB3 = 4864;
constexpr int kOMean = 4866, kOIstd = 4874, kNTrain = 4866;
constexpr int kLd = 72;  // padded LDS row stride (bf16 elements) of 64-wide matrices

// binary32 -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ __bf16 to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
}
__device__ __forceinline__ float from_bf16(__bf16 b) {
  return __uint_as_float(((uint32_t)__builtin_bit_cast(unsigned short, b)) << 16);
}

// hidden unit held in B-operand index kappa (see the header comment)
__host__ __device__ constexpr int mlp_pi(int kappa) {
  const int idx = 8 * (kappa >> 4) + (kappa & 7);  // accumulator slot 16 nt + i
  const int g = (kappa >> 3) & 1;                   // lane half
  return 32 * (idx >> 4) + 8 * ((idx & 15) >> 2) + 4 * g + (idx & 3);
}
// row (hidden unit) of accumulator slot i in a lane of half g, tile nt
__device__ __forceinline__ constexpr int acc_row(int nt, int i, int g) { return 32 * nt + 8 * (i >> 2) + 4 * g + (i & 3); }

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// bf16 matrices are read 16 bytes at a time (ds_read_b128): 16-byte aligned rows
struct MlpLds {
  alignas(16) __bf16 w1[64 * 16];   // [n][k], k = 8..15 zero
  alignas(16) __bf16 w2p[64 * kLd]; // [n2][kappa] = W2[n2][pi(kappa)]
  float b1[64], b2[64], w3[128], b3[2], mean[8], istd[8];
};

__device__ void mlp_stage(const float* __restrict__ prm, MlpLds& s) {
  const int t = threadIdx.x, nt = blockDim.x;
  for (int e = t; e < 64 * 16; e += nt) {
    const int n = e >> 4, k = e & 15;
    s.w1[e] = to_bf16(k < 8 ? prm[kOW1 + n * 8 + k] : 0.0f);
  }
  for (int e = t; e < 64 * 64; e += nt) {
    const int n = e >> 6, kap = e & 63;
    s.w2p[n * kLd + kap] = to_bf16(prm[kOW2 + n * 64 + mlp_pi(kap)]);
  }
  for (int e = t; e < 64; e += nt) {
    s.b1[e] = prm[kOB1 + e];
    s.b2[e] = prm[kOB2 + e];
  }
  for (int e = t; e < 128; e += nt) s.w3[e] = prm[kOW3 + e];
  for (int e = t; e < 8; e += nt) {
    s.mean[e] = prm[kOMean + e];
    s.istd[e] = prm[kOIstd + e];
  }
  if (t < 2) s.b3[t] = prm[kOB3 + t];
}

__device__ __forceinline__ bf16x8 lds8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

struct MlpFwd {
  bf16x8 xb[2];      // layer-1 B operands, per point tile mt
  f32x16 a1[2][2];   // layer-1 pre-activations (with bias) [nt][mt]
  bf16x8 hb[2][4];   // layer-2 B operands [mt][ks]
  f32x16 a2[2][2];   // layer-2 pre-activations (with bias) [nt][mt]
};

// standardized features of this lane's point -> network outputs of this lane's point
__device__ __forceinline__ void mlp_forward(const MlpLds& s, const float z[8], MlpFwd& f, float y[2]) {
#pragma clang fp contract(off)
  const int l = lane_id(), g = l >> 5, c = l & 31;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float other = __shfl(z[j], c + 32, 64);
    f.xb[0][j] = to_bf16(g ? 0.0f : z[j]);
    f.xb[1][j] = to_bf16(g ? 0.0f : other);
  }
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const bf16x8 aw = lds8(&s.w1[(32 * nt + c) * 16 + 8 * g]);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const f32x16 zero = {};
      f.a1[nt][mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw, f.xb[mt], zero, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 16; ++i) f.a1[nt][mt][i] += s.b1[acc_row(nt, i, g)];
    }
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float v = f.a1[(8 * ks + j) >> 4][mt][(8 * ks + j) & 15];
        f.hb[mt][ks][j] = to_bf16(v > 0.0f ? v : 0.0f);
      }
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    f32x16 acc[2] = {{}, {}};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const bf16x8 aw = lds8(&s.w2p[(32 * nt + c) * kLd + 16 * ks + 8 * g]);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw, f.hb[mt][ks], acc[mt], 0, 0, 0);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int i = 0; i < 16; ++i) f.a2[nt][mt][i] = acc[mt][i] + s.b2[acc_row(nt, i, g)];
  }
  float part[2][2];
#pragma unroll
  for (int o = 0; o < 2; ++o)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      float sacc = 0.0f;
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const float h = f.a2[nt][mt][i];
          sacc += s.w3[o * 64 + acc_row(nt, i, g)] * (h > 0.0f ? h : 0.0f);
        }
      part[o][mt] = sacc;
    }
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    const float mine = g ? part[o][1] : part[o][0];
    const float send = g ? part[o][0] : part[o][1];
    y[o] = mine + __shfl_xor(send, 32, 64) + s.b3[o];
  }
}

// The same network for inference only: identical operations in the same
// order (so the same outputs bit for bit), without keeping the layers'
// pre-activations for a backward pass: layer 2 is formed one 32-unit tile at
// a time and folded into the output sums at once, which keeps the register
// footprint small enough for several waves per SIMD.
__device__ __forceinline__ void mlp_infer(const MlpLds& s, const float z[8], float y[2]) {
#pragma clang fp contract(off)
  const int l = lane_id(), g = l >> 5, c = l & 31;
  float part[2][2] = {{0.0f, 0.0f}, {0.0f, 0.0f}};
  // one 32-point tile (mt) at a time: layer 1 for both 32-unit halves of the
  // hidden layer, then layer 2 half by half, folded into the output sums
#pragma unroll 1
  for (int mt = 0; mt < 2; ++mt) {
    bf16x8 xb;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float v = __shfl(z[j], c + 32 * mt, 64);
      xb[j] = to_bf16(g ? 0.0f : v);
    }
    bf16x8 hb[4];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const bf16x8 aw = lds8(&s.w1[(32 * nt + c) * 16 + 8 * g]);
      const f32x16 zero = {};
      const f32x16 a1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw, xb, zero, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float v = a1[i] + s.b1[acc_row(nt, i, g)];
        // accumulator slot 16 nt + i is B-operand entry (ks, j) = ((16 nt + i) / 8, (16 nt + i) % 8)
        hb[(16 * nt + i) >> 3][(16 * nt + i) & 7] = to_bf16(v > 0.0f ? v : 0.0f);
      }
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      f32x16 acc = {};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const bf16x8 aw = lds8(&s.w2p[(32 * nt + c) * kLd + 16 * ks + 8 * g]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw, hb[ks], acc, 0, 0, 0);
      }
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        float sacc = part[o][mt];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const float h = acc[i] + s.b2[acc_row(nt, i, g)];
          sacc += s.w3[o * 64 + acc_row(nt, i, g)] * (h > 0.0f ? h : 0.0f);
        }
        part[o][mt] = sacc;
      }
    }
  }
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    const float mine = g ? part[o][1] : part[o][0];
    const float send = g ? part[o][0] : part[o][1];
    y[o] = mine + __shfl_xor(send, 32, 64) + s.b3[o];
  }
}

// --------------------------------------------------------------- features

// The network's inputs are binary32 (then bf16 on the matrix cores), so the
// logarithms are taken in binary32 of the FP64 quantities rounded to it; the
// ratio x4 is formed in FP64 (its tiny guard would underflow in binary32).
__device__ __forceinline__ void c2p_features(const C2pInv& c, float x[8]) {
#pragma clang fp contract(off)
  const double onep = 1.0 + c.q;
  x[0] = log10f((float)c.D);
  x[1] = log10f((float)fmax(c.q, 1e-30));
  x[2] = log10f((float)(c.r2 + 1e-30));
  x[3] = log10f((float)(c.B2 + 1e-30));
  x[4] = (float)(c.rB * c.rB / (c.r2 * c.B2 + 1e-300));
  x[5] = log10f((float)onep);
  x[6] = log10f((float)(c.r2 / (onep * onep) + 1e-30));
  x[7] = log10f((float)(c.B2 / onep + 1e-30));
}

// Closed-form approximations of the two log fractions, corrected by the
// network: exact for the auxiliary root without magnetic field (rbar = r, so
// mu_+ = 1/sqrt(h0^2 + r^2)); mu ~ 1/(1 + q) for the second root (D (1 + q)
// is the energy density, about rho h W^2 for a cold, weakly magnetised fluid).
// In binary32: they only place the starting guesses.
__device__ __forceinline__ void c2p_baseline(const C2pInv& c, double h0, float b[2]) {
#pragma clang fp contract(off)
  const float l = 0.5f * logf((float)(h0 * h0 + c.r2));
  b[0] = logf((float)h0) - l;
  b[1] = -logf((float)(1.0 + c.q)) + l;
}

__device__ __forceinline__ void standardize(const MlpLds& s, const float x[8], float z[8]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int k = 0; k < 8; ++k) z[k] = (x[k] - s.mean[k]) * s.istd[k];
}


struct FeatArgs {
  Geom g;
  mhd_eos_t eos;
  const double* __restrict__ U;
  const double* __restrict__ mu;
  float* __restrict__ X;
  float* __restrict__ T;
  int Nx, Ny;
  int64_t npts;
};

// features (and targets) at every padded point, rows in linear padded order;
// points below the density threshold get NaN rows
__global__ void __launch_bounds__(256) k_mlp_features(FeatArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.npts) return;
  const int i = (int)(t % a.Nx), j = (int)((t / a.Nx) % a.Ny), k = (int)(t / ((int64_t)a.Nx * a.Ny));
  const int64_t p = a.g.at(i, j, k);
  C2pPoint pt;
  load_point(a.U, a.g.sf, p, pt);
  C2pInv c;
  if (!c2p_setup(a.eos, pt, c)) {
    const float nan = __builtin_nanf("");
#pragma unroll
    for (int q = 0; q < 8; ++q) a.X[t * 8 + q] = nan;
    if (a.T) a.T[t * 2] = a.T[t * 2 + 1] = nan;
    return;
  }
  float x[8];
  c2p_features(c, x);
#pragma unroll
  for (int q = 0; q < 8; ++q) a.X[t * 8 + q] = x[q];
  if (a.T && a.mu) {
    const double mup = a.mu[p], mu = a.mu[a.g.sf + p];
    float b[2];
    c2p_baseline(c, a.eos.h0, b);
    a.T[t * 2] = (float)(log(mup * a.eos.h0) - (double)b[0]);
    a.T[t * 2 + 1] = (float)(log(mu / mup) - (double)b[1]);
  }
}

// mean and inverse standard deviation of each feature over the non-NaN rows (one block)
__global__ void __launch_bounds__(256) k_mlp_normalize(float* __restrict__ prm, const float* __restrict__ X, int64_t n) {
  __shared__ double red[3][8][256];
  const int t = threadIdx.x;
  double s1[8] = {0}, s2[8] = {0}, cnt = 0.0;
  for (int64_t r = t; r < n; r += 256) {
    if (isnan(X[r * 8])) continue;
    cnt += 1.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double v = X[r * 8 + q];
      s1[q] += v;
      s2[q] += v * v;
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    red[0][q][t] = s1[q];
    red[1][q][t] = s2[q];
    red[2][q][t] = cnt;
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int q = 0; q < 8; ++q) {
        red[0][q][t] += red[0][q][t + w];
        red[1][q][t] += red[1][q][t + w];
        red[2][q][t] += red[2][q][t + w];
      }
    __syncthreads();
  }
  if (t < 8) {
    const double N = red[2][t][0] > 0.0 ? red[2][t][0] : 1.0;
    const double m = red[0][t][0] / N;
    const double var = fmax(red[1][t][0] / N - m * m, 0.0);
    prm[kOMean + t] = (float)m;
    prm[kOIstd + t] = var > 1e-12 ? (float)(1.0 / sqrt(var)) : 1.0f;
  }
}

// network outputs for n raw feature rows (NaN rows give NaN)
__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ prm, const float* __restrict__ X, int64_t n,
                                                     float* __restrict__ Y) {
  __shared__ MlpLds s;
  mlp_stage(prm, s);
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // whole waves run the MFMA
  const bool live = r < n && !isnan(X[(r < n ? r : 0) * 8]);
  float x[8], z[8], y[2];
#pragma unroll
  for (int q = 0; q < 8; ++q) x[q] = live ? X[r * 8 + q] : 0.0f;
  standardize(s, x, z);
  MlpFwd f;
  mlp_forward(s, z, f, y);
  if (r < n) {
    Y[r * 2] = live ? y[0] : __builtin_nanf("");
    Y[r * 2 + 1] = live ? y[1] : __builtin_nanf("");
  }
}

// --------------------------------------------------------------- training

struct MlpLdsTrain {
  MlpLds s;
  alignas(16) __bf16 w2tp[64 * kLd];  // [k][kappa] = W2[pi(kappa)][k]  (A operand of W2^T g2)
  alignas(16) __bf16 G[64 * kLd];     // [hidden][sample] staging of bf16 back-propagated signals
  alignas(16) __bf16 H[64 * kLd];     // [hidden][sample] staging of bf16 layer-1 activations
  alignas(16) __bf16 XT[32 * kLd];    // [feature][sample] staging of bf16 inputs (rows 8..31 zero)
  float acc[kNTrain];     // this block's gradient
  double loss;
};

// half-wave (32-lane) butterfly sum
__device__ __forceinline__ float half_sum(float v) {
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per-block gradient of L = 1/(2n) sum (y - t)^2 over the rows [0, n) the
// block owns (chunks of 64 rows, grid-strided); written to part[block][.] so
// that the reduction over blocks has a fixed order.  One wavefront per block.
__global__ void __launch_bounds__(64) k_mlp_grad(const float* __restrict__ prm, const float* __restrict__ X,
                                                 const float* __restrict__ T, int64_t n, float* __restrict__ part,
                                                 double* __restrict__ loss_part) {
#pragma clang fp contract(off)
  __shared__ MlpLdsTrain L;
  MlpLds& s = L.s;
  mlp_stage(prm, s);
  const int l = lane_id(), g = l >> 5, c = l & 31;
  for (int e = l; e < 64 * 64; e += 64) {
    const int k = e >> 6, kap = e & 63;
    L.w2tp[k * kLd + kap] = to_bf16(prm[kOW2 + mlp_pi(kap) * 64 + k]);
  }
  for (int e = l; e < kNTrain; e += 64) L.acc[e] = 0.0f;
  for (int e = l; e < 32 * kLd; e += 64) L.XT[e] = to_bf16(0.0f);
  double lsum = 0.0;
  __syncthreads();
  const float inv_n = 1.0f / (float)n;
  for (int64_t chunk = blockIdx.x; chunk * 64 < n; chunk += gridDim.x) {
    const int64_t r = chunk * 64 + l;
    const bool live = r < n && !isnan(X[(r < n ? r : 0) * 8]);
    float x[8], z[8], y[2];
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = live ? X[r * 8 + q] : 0.0f;
    standardize(s, x, z);
    MlpFwd f;
    mlp_forward(s, z, f, y);
    float dy[2];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      const float res = live ? y[o] - T[r * 2 + o] : 0.0f;
      lsum += 0.5 * (double)res * (double)res;
      dy[o] = res * inv_n;
    }
    // dy of the two points of this lane's column (tiles mt = 0, 1)
    float dym[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int o = 0; o < 2; ++o) dym[mt][o] = __shfl(dy[o], 32 * mt + c, 64);
    // output layer: dW3, db3, and g2 = (W3^T dy) relu'(a2)
    f32x16 g2[2][2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int n2 = acc_row(nt, i, g);
        float w0 = 0.0f, w1 = 0.0f, gb = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          const float a = f.a2[nt][mt][i];
          const float h = a > 0.0f ? a : 0.0f;
          w0 += dym[mt][0] * h;
          w1 += dym[mt][1] * h;
          const float gg = dym[mt][0] * s.w3[n2] + dym[mt][1] * s.w3[64 + n2];
          g2[nt][mt][i] = a > 0.0f ? gg : 0.0f;
          gb += g2[nt][mt][i];
        }
        w0 = half_sum(w0);
        w1 = half_sum(w1);
        gb = half_sum(gb);
        if (c == 0) {
          L.acc[kOW3 + n2] += w0;
          L.acc[kOW3 + 64 + n2] += w1;
          L.acc[kOB2 + n2] += gb;
        }
      }
    {
      float d0 = dy[0], d1 = dy[1];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        d0 += __shfl_xor(d0, off, 64);
        d1 += __shfl_xor(d1, off, 64);
      }
      if (l == 0) {
        L.acc[kOB3] += d0;
        L.acc[kOB3 + 1] += d1;
      }
    }
    // stage bf16 g2 and layer-1 activations as [hidden][sample]
    bf16x8 g2b[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int i = 0; i < 16; ++i) L.G[acc_row(nt, i, g) * kLd + 32 * mt + c] = to_bf16(g2[nt][mt][i]);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int idx = 8 * ks + j;
          g2b[mt][ks][j] = to_bf16(g2[idx >> 4][mt][idx & 15]);
          L.H[mlp_pi(16 * ks + 8 * g + j) * kLd + 32 * mt + c] = f.hb[mt][ks][j];
        }
    }
    if (g == 0)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int q = 0; q < 8; ++q) L.XT[q * kLd + 32 * mt + c] = f.xb[mt][q];
    __syncthreads();
    // dW2[n2][k] = sum_m g2b[n2][m] h1b[k][m]
#pragma unroll
    for (int na = 0; na < 2; ++na)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        f32x16 acc = {};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const bf16x8 a = lds8(&L.G[(32 * na + c) * kLd + 16 * ks + 8 * g]);
          const bf16x8 b = lds8(&L.H[(32 * nb + c) * kLd + 16 * ks + 8 * g]);
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) L.acc[kOW2 + acc_row(na, i, g) * 64 + 32 * nb + c] += acc[i];
      }
    // g1[k][m] = (sum_n2 W2[n2][k] g2b[n2][m]) relu'(a1)
    f32x16 g1[2][2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      f32x16 acc[2] = {{}, {}};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const bf16x8 a = lds8(&L.w2tp[(32 * nt + c) * kLd + 16 * ks + 8 * g]);
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, g2b[mt][ks], acc[mt], 0, 0, 0);
      }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int i = 0; i < 16; ++i) g1[nt][mt][i] = f.a1[nt][mt][i] > 0.0f ? acc[mt][i] : 0.0f;
    }
    __syncthreads();  // every lane is done reading L.G
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        float gb = 0.0f;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
          gb += g1[nt][mt][i];
          L.G[acc_row(nt, i, g) * kLd + 32 * mt + c] = to_bf16(g1[nt][mt][i]);
        }
        gb = half_sum(gb);
        if (c == 0) L.acc[kOB1 + acc_row(nt, i, g)] += gb;
      }
    __syncthreads();
    // dW1[k][q] = sum_m g1b[k][m] xb[q][m]
#pragma unroll
    for (int na = 0; na < 2; ++na) {
      f32x16 acc = {};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const bf16x8 a = lds8(&L.G[(32 * na + c) * kLd + 16 * ks + 8 * g]);
        const bf16x8 b = lds8(&L.XT[c * kLd + 16 * ks + 8 * g]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
      if (c < 8)
#pragma unroll
        for (int i = 0; i < 16; ++i) L.acc[kOW1 + acc_row(na, i, g) * 8 + c] += acc[i];
    }
    __syncthreads();
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
  for (int e = l; e < kNTrain; e += 64) part[(int64_t)blockIdx.x * kNTrain + e] = L.acc[e];
  if (l == 0) loss_part[blockIdx.x] = lsum / (double)n;
}

// grad[i] = sum over blocks (fixed order); loss likewise
__global__ void __launch_bounds__(256) k_mlp_grad_reduce(const float* __restrict__ part, const double* __restrict__ loss_part,
                                                         int nblk, float* __restrict__ grad, float* __restrict__ loss) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < kNTrain) {
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * kNTrain + e];
    grad[e] = s;
  }
  if (e == 0 && loss) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += loss_part[b];
    *loss = (float)s;
  }
}

__global__ void __launch_bounds__(256) k_mlp_adam(float* __restrict__ prm, const float* __restrict__ grad,
                                                  float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                  float b2, float eps, float c1, float c2) {
#pragma clang fp contract(off)
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kNTrain) return;
  const float gr = grad[e];
  const float mn = b1 * m[e] + (1.0f - b1) * gr;
  const float vn = b2 * v[e] + (1.0f - b2) * gr * gr;
  m[e] = mn;
  v[e] = vn;
  prm[e] -= lr * (mn / c1) / (sqrtf(vn / c2) + eps);
}

// --------------------------------------------------------------- con2prim with the learned guess

struct LearnedArgs {
  Geom g;
  mhd_eos_t eos;
  const float* __restrict__ prm;
  double* __restrict__ U;
  double* __restrict__ P;
  uint8_t* __restrict__ flags;
  double* __restrict__ mu;
  int64_t* __restrict__ stats;
  uint32_t* __restrict__ qcount;  // [0]: points to solve, [1]: points for the bracketed solver
  uint32_t* __restrict__ queue;   // linear padded indices of the points to solve
  uint32_t* __restrict__ fqueue;  // linear padded indices of the rejected points
  float* __restrict__ feat;        // per solve-queue slot: 8 raw features, then the 2 network outputs in place
  int Nx, Ny;
  int64_t npts;
};

constexpr int kNewtonIt = 3;

// mu_+ (App. D): the root of f_a on (0, hi], hi = 1/h0, or hi itself where
// f_a(hi) <= 0.  Newton on f_a from x0 with at most kNewtonIt updates, iterates
// kept in (0, hi]; accepted once |f_a(x)| <= 1e-12, returning the Newton
// correction of x.  f_a costs one division and one square root: no EoS.
__device__ __forceinline__ bool newton_mup(const C2pInv& c, double x, double hi, double& out, int& nev) {
#pragma clang fp contract(off)
  for (int it = 0; it <= kNewtonIt; ++it) {
    const Dual r = fa_t<Dual>(c, Dual{x, 1.0});
    ++nev;
    if (x == hi && r.v <= 0.0) {  // f_a(hi) <= 0: the bracket's end itself
      out = hi;
      return true;
    }
    if (!(r.d > 0.0)) return false;
    const double x1 = x - r.v / r.d;
    if (fabs(r.v) <= 1e-12) {
      out = fmin(x1, hi);
      return out > 0.0;
    }
    if (it == kNewtonIt) return false;
    x = fmin(x1, hi);
    if (!(x > 0.0)) return false;
  }
  return false;
}

// Newton on f from x0 with at most kNewtonIt updates, iterates kept in
// (0, mup] (an update past mup restarts from it: roots close to mup are
// common, and above it the velocity clamp of App. D changes f's branch).
// At an iterate x with |f(x)| <= 1e-12 x the Newton correction x1 is taken;
// one more evaluation at y, 5e-13 x1 beyond x1 on the side away from x, must
// have the sign opposite to f(x), and |y - x| <= 1e-12 x1: a root of f then
// lies between x and y, within 1e-12 x1 of x1.  That interval must lie below
// f_a's root (f_a is increasing): taken as shown when its upper end is below
// mup (1 - 1e-9), mup being f_a's root to ~1e-12, else checked by f_a <= 0
// there.  nev counts the root-function evaluations, f_a's included.
template <class FnD, class Fn>
__device__ __forceinline__ bool newton_mu(const FnD& F, const Fn& Fv, const C2pInv& c, double x, double mup,
                                          double& out, int& nev) {
#pragma clang fp contract(off)
  for (int it = 0; it <= kNewtonIt; ++it) {
    const Dual r = F(Dual{x, 1.0});
    ++nev;
    if (!(r.d != 0.0)) return false;
    const double x1 = x - r.v / r.d;
    if (fabs(r.v) <= 1e-12 * x) {
      double up = x;
      if (r.v != 0.0) {
        const double dir = (r.v < 0.0) == (r.d > 0.0) ? 1.0 : -1.0;
        const double y = x1 + dir * 5e-13 * x1;
        const double fy = Fv(y);
        ++nev;
        if (!((fy > 0.0) != (r.v > 0.0) || fy == 0.0)) return false;
        if (!(fabs(y - x) <= 1e-12 * x1)) return false;
        up = fmax(x, y);
      }
      if (!(up < mup * (1.0 - 1e-9))) {
        const double fa = fa_t<double>(c, up);
        ++nev;
        if (!(fa <= 0.0)) return false;
      }
      if (!(x1 > 0.0)) return false;
      out = r.v != 0.0 ? x1 : x;
      return true;
    }
    if (it == kNewtonIt) return false;
    x = fmin(x1, mup);
    if (!(x > 0.0)) return false;
  }
  return false;
}

struct FDual {
  const mhd_eos_t& e;
  const C2pInv& c;
  __device__ Dual operator()(Dual mu) const { return f_t<Dual>(e, c, mu); }
};

// log fraction (baseline + network output) -> fraction of the bracket's upper end, in (0, 1]
__device__ __forceinline__ double frac_of(float y) { return (double)expf(fminf(y, 0.0f)); }

struct LearnedOut {
  bool fallback;
  int64_t nfatal, ncorr, nit;
};

// con2prim of padded point (i, j, k), one that needs a root solve, from the
// network's two outputs y: Newton for mu_+ and then mu (no matrix cores here,
// so the kernel is not held to the network's register budget).  Returns
// whether the point needs the bracketed solver (then nothing is stored).
__device__ __forceinline__ LearnedOut newton_point(const mhd_eos_t& eos, const Geom& g, double* U, double* P,
                                                   uint8_t* flags, double* mu, int i, int j, int k, float y0,
                                                   float y1) {
  LearnedOut r{false, 0, 0, 0};
  const int64_t p = g.at(i, j, k);
  C2pPoint pt;
  load_point(U, g.sf, p, pt);
  C2pInv c;
  if (!c2p_setup(eos, pt, c)) {  // not reached for queued points
    r.fallback = true;
    return r;
  }
  C2pOut o;
  o.flags = 0;
  o.iters = 0;
  int nev = 0;
  float b[2];
  c2p_baseline(c, c.h0, b);
  const double hi = 1.0 / c.h0;
  double mup = hi, m = hi;
  bool ok = newton_mup(c, frac_of(b[0] + y0) * hi, hi, mup, nev);
  if (ok) ok = newton_mu(FDual{eos, c}, FFn{eos, c}, c, frac_of(b[1] + y1) * mup, mup, m, nev);
  r.nit = nev;
  if (!ok) {
    r.fallback = true;
    return r;
  }
  o.mup = mup;
  o.mu = m;
  c2p_finish(eos, pt, c, m, o);
  store_point(U, P, flags, mu, g.sf, p, pt, o);
  r.nfatal = (o.flags & MHD_FLAG_FATAL) ? 1 : 0;
  r.ncorr = (o.flags & C2P_CORRECTED) ? 1 : 0;
  return r;
}

// First pass: every padded point is loaded once; points below the density
// threshold get the atmosphere (as in the bracketed path); for the others the
// network's 8 raw features are computed (binary32).  No network here: the
// pass runs at full occupancy.  Returns whether the point needs a solve.
__device__ __forceinline__ bool classify_point(const mhd_eos_t& eos, const Geom& g, double* U, double* P,
                                               uint8_t* flags, double* mu, int i, int j, int k, float x[8]) {
  const int64_t p = g.at(i, j, k);
  C2pPoint pt;
  load_point(U, g.sf, p, pt);
  C2pInv c;
  if (!c2p_setup(eos, pt, c)) {
    C2pOut o;
    o.iters = 0;
    o.mup = o.mu = 0.0;
    atmosphere_prims(eos, o.prim);
    o.flags = MHD_FLAG_ATMO;
    double Wn;
    const double zv[3] = {0.0, 0.0, 0.0};
    prim_to_cons(pt.gd, o.prim[0], o.prim[1], o.prim[2], zv, o.prim[7], pt.B, o.cons, Wn);
    store_point(U, P, flags, mu, g.sf, p, pt, o);
    return false;
  }
  c2p_features(c, x);
  return true;
}

// wave-aggregated append of `entry` for the lanes with `take` set; returns the
// lane's slot (meaningful where take is set)
template <class T>
__device__ __forceinline__ uint32_t queue_append(bool take, T entry, uint32_t* count, T* queue) {
  const uint64_t mask = __ballot(take);
  if (!mask) return 0u;
  const int l = lane_id();
  const int leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if (l == leader) base = atomicAdd(count, (uint32_t)__popcll(mask));
  base = __shfl(base, leader, 64);
  const uint32_t slot = base + (uint32_t)__popcll(mask & ((1ull << l) - 1ull));
  if (take) queue[slot] = entry;
  return slot;
}

// block-aggregated append (every thread of the block calls it, with a
// block-uniform trip count): one atomic per block and call instead of one per
// wavefront, since appends from every wavefront to one counter serialise in
// L2 when most points are queued.  Returns the lane's slot where take is set.
template <class T>
__device__ __forceinline__ uint32_t block_queue_append(bool take, T entry, uint32_t* count, T* queue) {
  __shared__ uint32_t wsum[4], bbase;
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int w = tid >> 6, l = tid & 63;
  const uint64_t mask = __ballot(take);
  if (l == 0) wsum[w] = (uint32_t)__popcll(mask);
  __syncthreads();
  if (tid == 0) {
    const int nw = (int)((blockDim.x * blockDim.y + 63) / 64);
    uint32_t tot = 0;
    for (int v = 0; v < nw; ++v) {
      const uint32_t c = wsum[v];
      wsum[v] = tot;
      tot += c;
    }
    bbase = tot ? atomicAdd(count, tot) : 0u;
  }
  __syncthreads();
  const uint32_t slot = bbase + wsum[w] + (uint32_t)__popcll(mask & ((1ull << l) - 1ull));
  if (take) queue[slot] = entry;
  __syncthreads();  // wsum and bbase are reused by the next call
  return slot;
}

__device__ __forceinline__ void store_features(float* feat, uint32_t slot, const float x[8]) {
  float4* f = reinterpret_cast<float4*>(feat + (int64_t)slot * 8);
  f[0] = make_float4(x[0], x[1], x[2], x[3]);
  f[1] = make_float4(x[4], x[5], x[6], x[7]);
}

__global__ void __launch_bounds__(256) k_c2p_classify(LearnedArgs a) {
  __shared__ mhd_eos_t seos;
  const mhd_eos_t& eos = stage_eos(a.eos, seos);
  int64_t ncorr = 0;
  // block-uniform trip count (the append synchronises the block)
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < a.npts; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = base + threadIdx.x;
    float x[8];
    bool solve = false;
    if (t < a.npts) {
      const int i = (int)(t % a.Nx), j = (int)((t / a.Nx) % a.Ny), k = (int)(t / ((int64_t)a.Nx * a.Ny));
      solve = classify_point(eos, a.g, a.U, a.P, a.flags, a.mu, i, j, k, x);
      ncorr += solve ? 0 : 1;
    }
    const uint32_t slot = block_queue_append<uint32_t>(solve, (uint32_t)t, &a.qcount[0], a.queue);
    if (solve) store_features(a.feat, slot, x);
  }
  if (a.stats) block_add_stats(a.stats, 0, ncorr, 0, 0);
}

// Second pass: the network on the queued feature rows, whole wavefronts of
// them (blocks stride over chunks of 256 rows, so the trip count is uniform
// over the block); the two outputs overwrite the row's first two features.
__global__ void __launch_bounds__(256) k_c2p_mlp(const float* __restrict__ prm, const uint32_t* __restrict__ qcount,
                                                 float* __restrict__ feat) {
  const int64_t nq = qcount[0];
  if ((int64_t)blockIdx.x * blockDim.x >= nq) return;  // whole block: no work
  __shared__ MlpLds s;
  mlp_stage(prm, s);
  __syncthreads();
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nq; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = base + threadIdx.x;
    const bool live = q < nq;
    float x[8] = {0, 0, 0, 0, 0, 0, 0, 0}, z[8] = {0, 0, 0, 0, 0, 0, 0, 0}, y[2];
    if (live) {
      const float4* f = reinterpret_cast<const float4*>(feat + q * 8);
      const float4 f0 = f[0], f1 = f[1];
      x[0] = f0.x, x[1] = f0.y, x[2] = f0.z, x[3] = f0.w, x[4] = f1.x, x[5] = f1.y, x[6] = f1.z, x[7] = f1.w;
      standardize(s, x, z);
    }
    mlp_infer(s, z, y);
    if (live) *reinterpret_cast<float2*>(feat + q * 8) = make_float2(y[0], y[1]);
  }
}

// Third pass: Newton from the network's guesses on the queued points;
// rejected points go to the fallback queue
__global__ void __launch_bounds__(256) k_c2p_newton(LearnedArgs a) {
  __shared__ mhd_eos_t seos;
  const mhd_eos_t& eos = stage_eos(a.eos, seos);
  const int64_t nq = a.qcount[0];
  int64_t nfatal = 0, ncorr = 0, nfb = 0, nit = 0;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nq; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = base + threadIdx.x;
    const bool live = q < nq;
    LearnedOut r{false, 0, 0, 0};
    int64_t t = 0;
    if (live) {
      t = (int64_t)a.queue[q];
      const int i = (int)(t % a.Nx), j = (int)((t / a.Nx) % a.Ny), k = (int)(t / ((int64_t)a.Nx * a.Ny));
      const float2 y = *reinterpret_cast<const float2*>(a.feat + q * 8);
      r = newton_point(eos, a.g, a.U, a.P, a.flags, a.mu, i, j, k, y.x, y.y);
    }
    queue_append<uint32_t>(r.fallback, (uint32_t)t, &a.qcount[1], a.fqueue);
    nfatal += r.nfatal;
    ncorr += r.ncorr;
    nfb += r.fallback ? 1 : 0;
    nit += r.nit;
  }
  if (a.stats) block_add_stats(a.stats, nfatal, ncorr, nfb, nit);
}

// level versions: queue entries are (box << 32) | linear padded point of the box
__device__ __forceinline__ uint64_t level_entry(const LevelArgs& L, const BoxDev& B, int i, int j, int k) {
  const int Nx = B.g.nx + 2 * B.g.ng, Ny = B.g.ny + 2 * B.g.ng;
  const uint64_t box = (uint64_t)(&B - L.boxes);
  return (box << 32) | (uint64_t)((int64_t)i + (int64_t)Nx * ((int64_t)j + (int64_t)Ny * k));
}
__device__ __forceinline__ const BoxDev& level_point(const LevelArgs& L, uint64_t e, int& i, int& j, int& k) {
  const BoxDev& B = L.boxes[(int)(e >> 32)];
  const int64_t t = (int64_t)(e & 0xffffffffull);
  const int Nx = B.g.nx + 2 * B.g.ng, Ny = B.g.ny + 2 * B.g.ng;
  i = (int)(t % Nx);
  j = (int)((t / Nx) % Ny);
  k = (int)(t / ((int64_t)Nx * Ny));
  return B;
}

__global__ void __launch_bounds__(256) k_c2p_classify_lv(LevelArgs L) {
  __shared__ mhd_eos_t seos;
  const mhd_eos_t& eos = stage_eos(L.eos, seos);
  int64_t ncorr = 0;
  for_each_level_point(L, kRegionPadded, [&](const BoxDev& B, int i, int j, int k, bool live) {
    float x[8];
    const bool solve = live && classify_point(eos, B.g, L.src ? B.Us : B.U, B.P, B.flags, nullptr, i, j, k, x);
    ncorr += (live && !solve) ? 1 : 0;
    const uint32_t slot =
        block_queue_append<uint64_t>(solve, solve ? level_entry(L, B, i, j, k) : 0ull, &L.qcount[0], L.queue);
    if (solve) store_features(L.feat, slot, x);
  });
  if (L.stats) block_add_stats(L.stats, 0, ncorr, 0, 0);
}

__global__ void __launch_bounds__(256) k_c2p_newton_lv(LevelArgs L) {
  __shared__ mhd_eos_t seos;
  const mhd_eos_t& eos = stage_eos(L.eos, seos);
  const int64_t nq = L.qcount[0];
  int64_t nfatal = 0, ncorr = 0, nfb = 0, nit = 0;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nq; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = base + threadIdx.x;
    const bool live = q < nq;
    LearnedOut r{false, 0, 0, 0};
    uint64_t e = 0;
    if (live) {
      e = L.queue[q];
      int i, j, k;
      const BoxDev& B = level_point(L, e, i, j, k);
      const float2 y = *reinterpret_cast<const float2*>(L.feat + q * 8);
      r = newton_point(eos, B.g, L.src ? B.Us : B.U, B.P, B.flags, nullptr, i, j, k, y.x, y.y);
    }
    queue_append<uint64_t>(r.fallback, e, &L.qcount[1], L.fqueue);
    nfatal += r.nfatal;
    ncorr += r.ncorr;
    nfb += r.fallback ? 1 : 0;
    nit += r.nit;
  }
  if (L.stats) block_add_stats(L.stats, nfatal, ncorr, nfb, nit);
}

__global__ void __launch_bounds__(256) k_c2p_fallback_lv(LevelArgs L) {
  __shared__ mhd_eos_t seos;
  const mhd_eos_t& eos = stage_eos(L.eos, seos);
  const uint32_t nq = L.qcount[1];
  int64_t nfatal = 0, ncorr = 0, nit = 0;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
    int i, j, k;
    const BoxDev& B = level_point(L, L.fqueue[q], i, j, k);
    const int64_t p = B.g.at(i, j, k);
    double* U = L.src ? B.Us : B.U;
    C2pPoint pt;
    load_point(U, B.g.sf, p, pt);
    C2pOut o;
    c2p_plain(eos, pt, o);
    o.flags |= MHD_FLAG_FALLBACK;
    store_point(U, B.P, B.flags, nullptr, B.g.sf, p, pt, o);
    nfatal += (o.flags & MHD_FLAG_FATAL) ? 1 : 0;
    ncorr += (o.flags & C2P_CORRECTED) ? 1 : 0;
    nit += o.iters;
  }
  if (L.stats) block_add_stats(L.stats, nfatal, ncorr, 0, nit);
}

// the bracketed solver on the queued points (grid-strided over the queue)
__global__ void __launch_bounds__(256) k_c2p_fallback(LearnedArgs a) {
  __shared__ mhd_eos_t seos;
  const mhd_eos_t& eos = stage_eos(a.eos, seos);
  const uint32_t nq = a.qcount[1];
  int64_t nfatal = 0, ncorr = 0, nit = 0;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
    const int64_t t = a.fqueue[q];
    const int i = (int)(t % a.Nx), j = (int)((t / a.Nx) % a.Ny), k = (int)(t / ((int64_t)a.Nx * a.Ny));
    const int64_t p = a.g.at(i, j, k);
    C2pPoint pt;
    load_point(a.U, a.g.sf, p, pt);
    C2pOut o;
    c2p_plain(eos, pt, o);
    o.flags |= MHD_FLAG_FALLBACK;
    store_point(a.U, a.P, a.flags, a.mu, a.g.sf, p, pt, o);
    nfatal += (o.flags & MHD_FLAG_FATAL) ? 1 : 0;
    ncorr += (o.flags & C2P_CORRECTED) ? 1 : 0;
    nit += o.iters;
  }
  if (a.stats) block_add_stats(a.stats, nfatal, ncorr, 0, nit);
}

__global__ void k_zero_u32(uint32_t* p) {
  p[0] = 0u;
  p[1] = 0u;
}

// ------------------------------------------------------------------ launchers

int launch_mlp_features(const Geom& g, const mhd_eos_t& eos, const double* U, const double* mu, float* X, float* T,
                        hipStream_t s) {
  const int Nx = g.nx + 2 * g.ng, Ny = g.ny + 2 * g.ng, Nz = g.nz + 2 * g.ng;
  FeatArgs a{g, eos, U, mu, X, T, Nx, Ny, (int64_t)Nx * Ny * Nz};
  MHD_LAUNCH(KID_MLP_FEATURES, k_mlp_features, dim3((unsigned)((a.npts + 255) / 256)), dim3(256), 0, s, a);
  return (int)hipGetLastError();
}

int launch_mlp_normalize(float* prm, const float* X, int64_t n, hipStream_t s) {
  MHD_LAUNCH(KID_MLP_NORMALIZE, k_mlp_normalize, dim3(1), dim3(256), 0, s, prm, X, n);
  return (int)hipGetLastError();
}

int launch_mlp_forward(const float* prm, const float* X, int64_t n, float* Y, hipStream_t s) {
  MHD_LAUNCH(KID_MLP_FORWARD, k_mlp_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, prm, X, n, Y);
  return (int)hipGetLastError();
}

int mlp_grad_blocks(int64_t n) {
  const int64_t chunks = (n + 63) / 64;
  return (int)(chunks < 1024 ? chunks : 1024);
}

int launch_mlp_grad(const float* prm, const float* X, const float* T, int64_t n, float* grad, float* loss, void* ws,
                    hipStream_t s) {
  const int nblk = mlp_grad_blocks(n);
  double* lpart = reinterpret_cast<double*>(ws);
  float* part = reinterpret_cast<float*>(lpart + 1024);
  MHD_LAUNCH(KID_MLP_GRAD, k_mlp_grad, dim3(nblk), dim3(64), 0, s, prm, X, T, n, part, lpart);
  MHD_LAUNCH(KID_MLP_GRAD_REDUCE, k_mlp_grad_reduce, dim3((kNTrain + 255) / 256), dim3(256), 0, s, part, lpart, nblk, grad,
             loss);
  return (int)hipGetLastError();
}

int launch_mlp_adam(float* prm, const float* grad, float* m, float* v, int step, float lr, float b1, float b2,
                    float eps, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  MHD_LAUNCH(KID_MLP_ADAM, k_mlp_adam, dim3((kNTrain + 255) / 256), dim3(256), 0, s, prm, grad, m, v, lr, b1, b2, eps,
             c1, c2);
  return (int)hipGetLastError();
}

int launch_con2prim_learned(const Geom& g, const mhd_eos_t& eos, const float* prm, double* U, double* P,
                            uint8_t* flags, double* mu, int64_t* stats, void* ws, hipStream_t s) {
  const int Nx = g.nx + 2 * g.ng, Ny = g.ny + 2 * g.ng, Nz = g.nz + 2 * g.ng;
  const int64_t npts = (int64_t)Nx * Ny * Nz;
  uint32_t* qcount = reinterpret_cast<uint32_t*>(ws);
  uint32_t* queue = qcount + 64;  // 256-byte offset
  // the feature rows start on the next 256-byte boundary after the two queues
  const uintptr_t fb = (reinterpret_cast<uintptr_t>(queue + 2 * npts) + 255u) & ~uintptr_t(255u);
  float* feat = reinterpret_cast<float*>(fb);
  LearnedArgs a{g, eos, prm, U, P, flags, mu, stats, qcount, queue, queue + npts, feat, Nx, Ny, npts};
  MHD_LAUNCH(KID_ZERO, k_zero_u32, dim3(1), dim3(1), 0, s, qcount);
  const int64_t nblk = (a.npts + 255) / 256;
  const unsigned grid = (unsigned)(nblk < 2048 ? nblk : 2048);
  MHD_LAUNCH(KID_C2P_CLASSIFY, k_c2p_classify, dim3(grid), dim3(256), 0, s, a);
  MHD_LAUNCH(KID_MLP_FORWARD, k_c2p_mlp, dim3(grid), dim3(256), 0, s, prm, qcount, feat);
  MHD_LAUNCH(KID_C2P_LEARNED, k_c2p_newton, dim3(grid), dim3(256), 0, s, a);
  MHD_LAUNCH(KID_C2P_FALLBACK, k_c2p_fallback, dim3(grid), dim3(256), 0, s, a);
  return (int)hipGetLastError();
}

// ---------------------------------------------- allocation-free entry point
// The queues and network rows of mhd_con2prim_learned_noalloc live in this
// file-scope device array, laid out as the workspace of mhd_con2prim_learned:
// the two count words padded to 256 bytes, the solve queue and the fallback
// queue (4 bytes per padded point each), then from the next 256-byte boundary
// an 8-float row per padded point (features, then the network's outputs).
// 512 B + 40 B per point covers patches of at most kNoAllocMaxPoints padded
// points (160 MiB per device, held until the process ends).  In host code the array's name is not a device
// address: the address comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is passed to kernels.
// Every call on a device shares its array; calls that overlap on one device
// race.
constexpr int64_t kNoAllocMaxPoints = int64_t(1) << 22;
static __device__ __align__(256) uint32_t scratch[128 + 10 * kNoAllocMaxPoints];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int64_t noalloc_max_points() { return kNoAllocMaxPoints; }

// Device address of `scratch` on the current device (looked up on the first
// call per device).  Returns a hipError_t.
int noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return (int)hipSuccess;
}

int launch_con2prim_learned_noalloc(const Geom& g, const mhd_eos_t& eos, const float* prm, double* U, double* P,
                                    uint8_t* flags, double* mu, int64_t* stats, hipStream_t s) {
  void* ws = nullptr;
  const int e = noalloc_scratch(&ws);
  if (e != (int)hipSuccess) return e;
  // same kernels as mhd_con2prim_learned; the first one clears the queue count
  return launch_con2prim_learned(g, eos, prm, U, P, flags, mu, stats, ws, s);
}

int launch_con2prim_learned_level(const LevelArgs& L, int grid, int block, int grid_q, hipStream_t s) {
  MHD_LAUNCH(KID_ZERO, k_zero_u32, dim3(1), dim3(1), 0, s, L.qcount);
  MHD_LAUNCH(KID_C2P_CLASSIFY, k_c2p_classify_lv, dim3(grid), dim3(block), 0, s, L);
  MHD_LAUNCH(KID_MLP_FORWARD, k_c2p_mlp, dim3(grid_q), dim3(256), 0, s, L.mlp, L.qcount, L.feat);
  MHD_LAUNCH(KID_C2P_LEARNED, k_c2p_newton_lv, dim3(grid_q), dim3(256), 0, s, L);
  MHD_LAUNCH(KID_C2P_FALLBACK, k_c2p_fallback_lv, dim3(grid_q), dim3(256), 0, s, L);
  return (int)hipGetLastError();
}

}  // namespace mhd
