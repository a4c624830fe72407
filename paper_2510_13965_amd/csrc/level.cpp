// Batched levels: all boxes of a refinement level through one persistent
// kernel per phase, an optional hipGraph of the whole RK4 step, and an
// autotuner for the launch shape (chunk size, strip height, persistent grid).
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mhd.h"
#include "dev_common.hpp"

namespace mhd {
int launch_con2prim_level(const LevelArgs& L, int grid, int block, hipStream_t s);
int launch_ccz4_level(const LevelArgs& L, int grid, int block, int grid_lds, hipStream_t s);
int launch_mhd_level(const LevelArgs& L, int grid_pad, int grid_int, int block, hipStream_t s);
int launch_rk4_level(const LevelArgs& L, int grid, int block, hipStream_t s);
int launch_zero_u64(unsigned long long* p, hipStream_t s);
int launch_con2prim_learned_level(const LevelArgs& L, int grid, int block, int grid_fb, hipStream_t s);
int launch_m1_point_level(const LevelArgs& L, int grid, int block, hipStream_t s);
int launch_m1_update_level(const LevelArgs& L, int grid, int block, hipStream_t s);
int launch_imex_combine_level(const LevelArgs& L, int grid, int block, hipStream_t s);
int launch_m1_implicit_level(const LevelArgs& L, int grid, int block, hipStream_t s);
int ccz4_workspace_fields();
int les_workspace_fields();
int abi_fail(int code, const char* msg);
int abi_hip(int rc, const char* what);
Geom abi_geom(const mhd_patch_t* p);
int abi_check_patch(const mhd_patch_t* p, int need_ng, const char* fn);
}  // namespace mhd

struct mhd_level {
  std::vector<mhd_box_t> boxes;
  std::vector<mhd::BoxDev> host;
  mhd::BoxDev* dev = nullptr;
  mhd_params_t par;
  mhd_eos_t eos;
  mhd_tuning_t tun;
  int64_t ntile_int = 0, ntile_pad = 0, ntile_h1 = 0, ntile_lds = 0;
  int ncu = 256;
  // graphs of one RK4 step and of one IMEX step, each valid for the arguments
  // it was captured with
  struct Graph {
    hipGraphExec_t exec = nullptr;
    double dt = 0.0;
    const void* a = nullptr;
    const void* b = nullptr;
  };
  hipStream_t cap = nullptr;
  Graph g_rk, g_imex;
  bool imex = false;  // per-box IMEX stage arrays attached
  // learned con2prim guess (nullptr: bracketed solver) and its fallback queue
  const float* mlp = nullptr;
  void* lws = nullptr;
  int64_t npad = 0;
};

namespace {

using mhd::abi_fail;
using mhd::abi_hip;

int block_threads(const mhd_tuning_t& t) { return t.block_threads ? t.block_threads : 256; }

void drop_graphs(mhd_level_t* lv) {
  for (mhd_level::Graph* g : {&lv->g_rk, &lv->g_imex}) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    *g = mhd_level::Graph{};
  }
}

// tile prefix sums for the current chunk size, uploaded to the device array
int layout(mhd_level_t* lv) {
  // kernels of earlier calls may still read the descriptor array
  int rc0 = abi_hip((int)hipDeviceSynchronize(), "mhd_level: synchronize");
  if (rc0) return rc0;
  const int T = block_threads(lv->tun);
  int64_t ti = 0, tp = 0, th = 0, tl = 0;
  for (size_t b = 0; b < lv->boxes.size(); ++b) {
    mhd::BoxDev& B = lv->host[b];
    const mhd::Geom& g = B.g;
    const int64_t plane_i = (int64_t)g.nx * g.ny;
    const int64_t plane_p = (int64_t)(g.nx + 2 * g.ng) * (g.ny + 2 * g.ng);
    const int64_t plane_h = (int64_t)(g.nx + 2) * (g.ny + 2);
    B.cpp_int = (int)((plane_i + T - 1) / T);
    B.cpp_pad = (int)((plane_p + T - 1) / T);
    B.cpp_h1 = (int)((plane_h + T - 1) / T);
    B.t0_int = ti;
    B.t0_pad = tp;
    B.t0_h1 = th;
    ti += (int64_t)B.cpp_int * g.nz;
    tp += (int64_t)B.cpp_pad * (g.nz + 2 * g.ng);
    th += (int64_t)B.cpp_h1 * (g.nz + 2);
    B.ntx_lds = (g.nx + mhd::kLevelLdsTile - 1) / mhd::kLevelLdsTile;
    B.nty_lds = (g.ny + mhd::kLevelLdsTile - 1) / mhd::kLevelLdsTile;
    B.nzc_lds = (g.nz + mhd::kLevelLdsZ - 1) / mhd::kLevelLdsZ;
    B.t0_lds = tl;
    tl += (int64_t)B.ntx_lds * B.nty_lds * B.nzc_lds;
  }
  if (ti >= ((int64_t)1 << 31) || tp >= ((int64_t)1 << 31) || th >= ((int64_t)1 << 31) || tl >= ((int64_t)1 << 31))
    return abi_fail(MHD_EINVAL, "mhd_level: too many tiles for one launch");
  lv->ntile_int = ti;
  lv->ntile_pad = tp;
  lv->ntile_h1 = th;
  lv->ntile_lds = tl;
  drop_graphs(lv);
  return abi_hip((int)hipMemcpy(lv->dev, lv->host.data(), sizeof(mhd::BoxDev) * lv->host.size(), hipMemcpyHostToDevice),
                 "mhd_level: upload");
}

int grid_for(const mhd_level_t* lv, int64_t ntile) {
  int64_t g = (ntile + 7) / 8 * 8;
  if (lv->tun.grid_per_cu > 0) {
    const int64_t cap = ((int64_t)lv->ncu * lv->tun.grid_per_cu + 7) / 8 * 8;
    if (cap < g) g = cap;
  }
  return (int)(g > 0 ? g : 8);
}

mhd::LevelArgs args_of(const mhd_level_t* lv, int src, int stage, double dt, double* max_speed, int64_t* stats) {
  mhd::LevelArgs L;
  L.boxes = lv->dev;
  L.nboxes = (int)lv->boxes.size();
  L.strip = lv->tun.strip;
  L.src = src;
  L.stage = stage;
  L.slot = -1;
  L.adt = 0.0;
  L.nfail = nullptr;
  L.m1 = (lv->par.flags & MHD_EVOLVE_M1) ? 1 : 0;
  L.nd = (L.m1 && (lv->par.flags & MHD_EVOLVE_M1N)) ? 1 : 0;
  L.nfields = L.nd ? MHD_NU_M1N : (L.m1 ? MHD_NU_M1 : MHD_NU);
  L.ntile_int = lv->ntile_int;
  L.ntile_pad = lv->ntile_pad;
  L.ntile_h1 = lv->ntile_h1;
  L.ntile_lds = lv->ntile_lds;
  L.dt = dt;
  L.par = lv->par;
  L.eos = lv->eos;
  L.max_speed = reinterpret_cast<unsigned long long*>(max_speed);
  L.stats = stats;
  L.mlp = lv->mlp;
  L.qcount = static_cast<uint32_t*>(lv->lws);
  L.queue = lv->lws ? reinterpret_cast<uint64_t*>(static_cast<char*>(lv->lws) + 256) : nullptr;
  L.fqueue = lv->lws ? L.queue + lv->npad : nullptr;
  L.feat = lv->lws ? reinterpret_cast<float*>(L.fqueue + lv->npad) : nullptr;
  return L;
}

// con2prim of every box at U (src 0) or Us (src 1)
int enqueue_c2p(const mhd_level_t* lv, int src, int64_t* stats, hipStream_t s) {
  const mhd::LevelArgs L = args_of(lv, src, 0, 0.0, nullptr, stats);
  const int T = block_threads(lv->tun);
  const int gp = grid_for(lv, lv->ntile_pad);
  if (lv->mlp) {
    const int64_t fb = (lv->npad + 255) / 256;
    return mhd::launch_con2prim_learned_level(L, gp, T, (int)(fb < 2048 ? fb : 2048), s);
  }
  return mhd::launch_con2prim_level(L, gp, T, s);
}

// L(U) of every box at U (src 0) or Us (src 1), into k (slot -1) or into the
// IMEX stage arrays F[slot], R[slot]
int enqueue_rhs_only(const mhd_level_t* lv, int src, double* max_speed, int slot, hipStream_t s) {
  mhd::LevelArgs L = args_of(lv, src, 0, 0.0, max_speed, nullptr);
  L.slot = slot;
  const int T = block_threads(lv->tun);
  const int gi = grid_for(lv, lv->ntile_int), gp = grid_for(lv, lv->ntile_pad);
  int rc;
  // the order of mhd_rhs: M1 closure and point fluxes (the CCZ4 matter terms read
  // the closure), CCZ4, GRMHD, then the M1 update (which adds the radiation's
  // exchange to the fluid's right-hand side)
  if (L.m1 && (rc = mhd::launch_m1_point_level(L, grid_for(lv, lv->ntile_h1), T, s))) return rc;
  if ((rc = mhd::launch_ccz4_level(L, gi, T, (int)((lv->ntile_lds + 7) / 8 * 8), s))) return rc;
  if ((rc = mhd::launch_mhd_level(L, gp, gi, T, s))) return rc;
  return L.m1 ? mhd::launch_m1_update_level(L, gi, T, s) : 0;
}

// con2prim + RHS of every box at U (src 0) or Us (src 1)
int enqueue_rhs(const mhd_level_t* lv, int src, double* max_speed, int64_t* stats, hipStream_t s) {
  const int rc = enqueue_c2p(lv, src, stats, s);
  return rc ? rc : enqueue_rhs_only(lv, src, max_speed, -1, s);
}

// implicit diagonal of Table I's I42L tableau
constexpr double kImexAii[4] = {0.0, 0.25, 1.0 / 3.0, 1.0 / 6.0};

// one IMEX(4,4,2) step (Table I): per stage, the combination into Us, con2prim,
// the implicit collision solve (a_ii != 0), and the split RHS into F[s], R[s];
// then the final combination into U
int enqueue_imex_step(const mhd_level_t* lv, double dt, double* max_speed, uint64_t* nfail, hipStream_t s) {
  int rc;
  if (max_speed && (rc = mhd::launch_zero_u64(reinterpret_cast<unsigned long long*>(max_speed), s))) return rc;
  const int T = block_threads(lv->tun);
  const int gi = grid_for(lv, lv->ntile_int);
  for (int st = 0; st <= 4; ++st) {
    const mhd::LevelArgs C = args_of(lv, 1, st, dt, nullptr, nullptr);
    if ((rc = mhd::launch_imex_combine_level(C, gi, T, s))) return rc;
    if (st == 4) break;
    if ((rc = enqueue_c2p(lv, 1, nullptr, s))) return rc;
    if (kImexAii[st] != 0.0) {
      mhd::LevelArgs I = args_of(lv, 1, st, dt, nullptr, nullptr);
      I.adt = kImexAii[st] * dt;
      I.nfail = reinterpret_cast<unsigned long long*>(nfail);
      if ((rc = mhd::launch_m1_implicit_level(I, gi, T, s))) return rc;
    }
    if ((rc = enqueue_rhs_only(lv, 1, max_speed, st, s))) return rc;
  }
  return 0;
}

// replays `g` (captured again when its arguments changed) on `s`
template <class Enqueue>
int graph_launch(mhd_level_t* lv, mhd_level::Graph& g, double dt, const void* a, const void* b, hipStream_t s,
                 Enqueue&& enqueue) {
  if (!g.exec || g.dt != dt || g.a != a || g.b != b) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = mhd_level::Graph{};
    hipGraph_t graph = nullptr;
    int rc = abi_hip((int)hipStreamBeginCapture(lv->cap, hipStreamCaptureModeThreadLocal), "mhd_level: capture");
    if (rc) return rc;
    const int erc = enqueue(lv->cap);
    const hipError_t e2 = hipStreamEndCapture(lv->cap, &graph);
    if (erc || e2 != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return abi_hip(erc ? erc : (int)e2, "mhd_level: capture of the step");
    }
    const hipError_t e3 = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
      g.exec = nullptr;
      return abi_hip((int)e3, "mhd_level: graph instantiate");
    }
    g.dt = dt;
    g.a = a;
    g.b = b;
  }
  return abi_hip((int)hipGraphLaunch(g.exec, s), "mhd_level: graph launch");
}

int enqueue_stage(const mhd_level_t* lv, int stage, double dt, hipStream_t s) {
  const mhd::LevelArgs L = args_of(lv, 0, stage, dt, nullptr, nullptr);
  return mhd::launch_rk4_level(L, grid_for(lv, lv->ntile_int), block_threads(lv->tun), s);
}

int enqueue_step(const mhd_level_t* lv, double dt, double* max_speed, hipStream_t s) {
  int rc;
  if (max_speed && (rc = mhd::launch_zero_u64(reinterpret_cast<unsigned long long*>(max_speed), s))) return rc;
  for (int st = 0; st < 4; ++st) {
    if ((rc = enqueue_rhs(lv, st > 0, max_speed, nullptr, s))) return rc;
    if ((rc = enqueue_stage(lv, st, dt, s))) return rc;
  }
  return 0;
}

int check_tuning(const mhd_tuning_t* t) {
  if (t->strip < 1 || t->strip > 1024) return abi_fail(MHD_EINVAL, "mhd_level: strip must be 1..1024");
  if (t->block_threads != 0 && t->block_threads != 64 && t->block_threads != 128 && t->block_threads != 256)
    return abi_fail(MHD_EINVAL, "mhd_level: block_threads must be 64, 128 or 256 (0: 256)");
  if (t->grid_per_cu < 0 || t->grid_per_cu > 64) return abi_fail(MHD_EINVAL, "mhd_level: grid_per_cu must be 0..64");
  return MHD_OK;
}

}  // namespace

extern "C" {

int mhd_level_create(const mhd_box_t* boxes, int nboxes, const mhd_params_t* par, const mhd_eos_t* eos,
                     mhd_level_t** out) {
  if (!out) return abi_fail(MHD_EINVAL, "mhd_level_create: out is NULL");
  *out = nullptr;
  if (!boxes || nboxes < 1) return abi_fail(MHD_EINVAL, "mhd_level_create: need at least one box");
  if (!par || !eos) return abi_fail(MHD_EINVAL, "mhd_level_create: params and eos are required");
  const uint32_t need = MHD_EVOLVE_SPACETIME | MHD_EVOLVE_MHD | MHD_COUPLE_MATTER;
  if ((par->flags & need) != need)
    return abi_fail(MHD_EINVAL, "mhd_level_create: a level evolves the full coupled system (all flags set)");
  if (par->les_cm != 0.0)
    return abi_fail(MHD_EINVAL, "mhd_level_create: the LES term (les_cm != 0) is evolved on single patches only");
  if (par->flags & MHD_COUPLE_EXCHANGE)
    return abi_fail(MHD_EINVAL, "mhd_level_create: the coupled exchange (MHD_COUPLE_EXCHANGE) runs on single patches only");
  if (par->flags & ~(need | MHD_EVOLVE_M1 | MHD_EVOLVE_M1N))
    return abi_fail(MHD_EINVAL, "mhd_level_create: unknown params flags");
  const bool m1 = (par->flags & MHD_EVOLVE_M1) != 0;
  const bool nd = (par->flags & MHD_EVOLVE_M1N) != 0;
  if (nd && !m1) return abi_fail(MHD_EINVAL, "mhd_level_create: MHD_EVOLVE_M1N needs MHD_EVOLVE_M1");
  if (nd && !std::isfinite(par->m_b)) return abi_fail(MHD_EINVAL, "mhd_level_create: m_b must be finite");
  if (par->f_alpha_kind != MHD_FALPHA_ONE && par->f_alpha_kind != MHD_FALPHA_HARMONIC)
    return abi_fail(MHD_EINVAL, "mhd_level_create: unknown f_alpha_kind");
  if (!(par->c_b > 0.0)) return abi_fail(MHD_EINVAL, "mhd_level_create: c_b must be > 0");
  if (eos->npieces < 1 || eos->npieces > 4) return abi_fail(MHD_EINVAL, "mhd_level_create: bad eos");
  for (int b = 0; b < nboxes; ++b) {
    const mhd_box_t& B = boxes[b];
    int rc;
    if ((rc = mhd::abi_check_patch(&B.patch, 3, "mhd_level_create"))) return rc;
    if (!B.U || !B.Us || !B.P || !B.k || !B.acc || !B.workspace)
      return abi_fail(MHD_EINVAL, "mhd_level_create: box arrays must be non-NULL (flags may be NULL)");
    if (B.workspace_bytes < (nd ? mhd_rhs_workspace_size_m1n(&B.patch)
                                : (m1 ? mhd_rhs_workspace_size_m1(&B.patch) : mhd_rhs_workspace_size(&B.patch))))
      return abi_fail(MHD_EWORKSPACE, "mhd_level_create: box workspace too small");
    if (m1 && !B.aux) return abi_fail(MHD_EINVAL, "mhd_level_create: aux is required with MHD_EVOLVE_M1");
    if (B.patch.sf > (int64_t)(INT32_MAX / 8))
      return abi_fail(MHD_EINVAL, "mhd_level_create: a padded field exceeds the 2^28-point limit");
  }
  mhd_level_t* lv = new (std::nothrow) mhd_level;
  if (!lv) return abi_fail(MHD_EINVAL, "mhd_level_create: out of host memory");
  lv->boxes.assign(boxes, boxes + nboxes);
  lv->host.resize(nboxes);
  for (int b = 0; b < nboxes; ++b) {
    mhd::BoxDev& D = lv->host[b];
    const mhd_box_t& B = boxes[b];
    D.g = mhd::abi_geom(&B.patch);
    D.U = B.U;
    D.Us = B.Us;
    D.P = B.P;
    D.k = B.k;
    D.acc = B.acc;
    D.ws = static_cast<double*>(B.workspace);
    D.flags = B.flags;
    D.aux = m1 ? B.aux : nullptr;
    D.ws_m1 = m1 ? D.ws + (int64_t)(33 + mhd::ccz4_workspace_fields() + mhd::les_workspace_fields()) * B.patch.sf
                 : nullptr;
    lv->npad += (int64_t)(B.patch.nx + 6) * (B.patch.ny + 6) * (B.patch.nz + 6);
  }
  lv->par = *par;
  lv->eos = *eos;
  lv->tun = mhd_tuning_t{};
  lv->tun.strip = 4;
  lv->tun.block_threads = 256;
  lv->tun.grid_per_cu = 0;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&lv->ncu, hipDeviceAttributeMultiprocessorCount, dev);
  int rc;
  if ((rc = abi_hip((int)hipMalloc(&lv->dev, sizeof(mhd::BoxDev) * nboxes), "mhd_level_create: hipMalloc")) ||
      (rc = layout(lv)) ||
      (rc = abi_hip((int)hipStreamCreateWithFlags(&lv->cap, hipStreamNonBlocking), "mhd_level_create: stream"))) {
    mhd_level_destroy(lv);
    return rc;
  }
  *out = lv;
  return MHD_OK;
}

int mhd_level_destroy(mhd_level_t* lv) {
  if (!lv) return MHD_OK;
  drop_graphs(lv);
  if (lv->cap) (void)hipStreamDestroy(lv->cap);
  if (lv->dev) (void)hipFree(lv->dev);
  delete lv;
  return MHD_OK;
}

int mhd_level_set_tuning(mhd_level_t* lv, const mhd_tuning_t* t) {
  if (!lv || !t) return abi_fail(MHD_EINVAL, "mhd_level_set_tuning: NULL");
  int rc;
  if ((rc = check_tuning(t))) return rc;
  lv->tun = *t;
  if (!lv->tun.block_threads) lv->tun.block_threads = 256;
  return layout(lv);
}

int mhd_level_get_tuning(const mhd_level_t* lv, mhd_tuning_t* t) {
  if (!lv || !t) return abi_fail(MHD_EINVAL, "mhd_level_get_tuning: NULL");
  *t = lv->tun;
  return MHD_OK;
}

size_t mhd_level_learned_workspace_size(const mhd_level_t* lv) {
  if (!lv) return 0;
  // counts, two 8-byte queues, then one 8-float row per padded point
  return 256 + 16 * (size_t)lv->npad + 32 * (size_t)lv->npad;
}

int mhd_level_set_learned(mhd_level_t* lv, const float* mlp, void* workspace, size_t workspace_bytes) {
  if (!lv) return abi_fail(MHD_EINVAL, "mhd_level_set_learned: NULL level");
  if (mlp && (!workspace || workspace_bytes < mhd_level_learned_workspace_size(lv)))
    return abi_fail(MHD_EWORKSPACE, "mhd_level_set_learned: workspace too small for the fallback queue");
  if (mlp && lv->npad >= ((int64_t)1 << 32))
    return abi_fail(MHD_EINVAL, "mhd_level_set_learned: more than 2^32 padded points in the level");
  int rc = abi_hip((int)hipDeviceSynchronize(), "mhd_level_set_learned: synchronize");
  if (rc) return rc;
  lv->mlp = mlp;
  lv->lws = mlp ? workspace : nullptr;
  drop_graphs(lv);
  return MHD_OK;
}

int mhd_level_rhs(mhd_level_t* lv, int src, double* max_speed, int64_t* stats, void* stream) {
  if (!lv) return abi_fail(MHD_EINVAL, "mhd_level_rhs: NULL level");
  if (src != 0 && src != 1) return abi_fail(MHD_EINVAL, "mhd_level_rhs: src must be 0 (U) or 1 (Us)");
  return abi_hip(enqueue_rhs(lv, src, max_speed, stats, (hipStream_t)stream), "mhd_level_rhs");
}

int mhd_level_rk4_step(mhd_level_t* lv, double dt, double* max_speed, int use_graph, void* stream) {
  if (!lv) return abi_fail(MHD_EINVAL, "mhd_level_rk4_step: NULL level");
  if (!(dt == dt) || dt > 1e300 || dt < -1e300) return abi_fail(MHD_EINVAL, "mhd_level_rk4_step: dt must be finite");
  hipStream_t s = (hipStream_t)stream;
  if (!use_graph) return abi_hip(enqueue_step(lv, dt, max_speed, s), "mhd_level_rk4_step");
  return graph_launch(lv, lv->g_rk, dt, max_speed, nullptr, s,
                      [&](hipStream_t cs) { return enqueue_step(lv, dt, max_speed, cs); });
}

int mhd_level_set_imex(mhd_level_t* lv, const mhd_imex_box_t* boxes, int nboxes) {
  if (!lv) return abi_fail(MHD_EINVAL, "mhd_level_set_imex: NULL level");
  if (!(lv->par.flags & MHD_EVOLVE_M1)) return abi_fail(MHD_EINVAL, "mhd_level_set_imex: the level must evolve M1");
  if (boxes && nboxes != (int)lv->boxes.size())
    return abi_fail(MHD_EINVAL, "mhd_level_set_imex: one entry per box of the level is needed");
  if (boxes)
    for (int b = 0; b < nboxes; ++b)
      for (int st = 0; st < 4; ++st)
        if (!boxes[b].F[st] || !boxes[b].R[st])
          return abi_fail(MHD_EINVAL, "mhd_level_set_imex: every F[s] and R[s] must be non-NULL");
  for (size_t b = 0; b < lv->host.size(); ++b)
    for (int st = 0; st < 4; ++st) {
      lv->host[b].F[st] = boxes ? boxes[b].F[st] : nullptr;
      lv->host[b].R[st] = boxes ? boxes[b].R[st] : nullptr;
    }
  lv->imex = boxes != nullptr;
  return layout(lv);  // waits for the device, uploads the descriptors, drops the graphs
}

int mhd_level_imex_step(mhd_level_t* lv, double dt, double* max_speed, uint64_t* nfail, int use_graph, void* stream) {
  if (!lv) return abi_fail(MHD_EINVAL, "mhd_level_imex_step: NULL level");
  if (!lv->imex) return abi_fail(MHD_EINVAL, "mhd_level_imex_step: no IMEX stage arrays (mhd_level_set_imex)");
  if (!(dt == dt) || dt > 1e300 || dt < -1e300) return abi_fail(MHD_EINVAL, "mhd_level_imex_step: dt must be finite");
  hipStream_t s = (hipStream_t)stream;
  if (!use_graph) return abi_hip(enqueue_imex_step(lv, dt, max_speed, nfail, s), "mhd_level_imex_step");
  return graph_launch(lv, lv->g_imex, dt, max_speed, nfail, s,
                      [&](hipStream_t cs) { return enqueue_imex_step(lv, dt, max_speed, nfail, cs); });
}

int mhd_level_autotune(mhd_level_t* lv, double dt, void* stream, mhd_tuning_t* chosen) {
  if (!lv) return abi_fail(MHD_EINVAL, "mhd_level_autotune: NULL level");
  hipStream_t s = (hipStream_t)stream;
  static const int kBlock[3] = {64, 128, 256};
  static const int kStrip[3] = {1, 4, 16};
  static const int kGrid[3] = {0, 4, 16};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return abi_fail(MHD_EHIP, "mhd_level_autotune: event");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return abi_fail(MHD_EHIP, "mhd_level_autotune: event");
  }
  mhd_tuning_t best = lv->tun;
  float best_ms = 1e30f;
  int rc = MHD_OK;
  for (int bi = 0; bi < 3 && !rc; ++bi)
    for (int si = 0; si < 3 && !rc; ++si)
      for (int gi = 0; gi < 3 && !rc; ++gi) {
        mhd_tuning_t t = mhd_tuning_t{};
        t.strip = kStrip[si];
        t.block_threads = kBlock[bi];
        t.grid_per_cu = kGrid[gi];
        if ((rc = mhd_level_set_tuning(lv, &t))) break;
        // timed unit: one evaluation at Us plus the stage-1 update (U is only read)
        float ms = 0.0f;
        for (int rep = 0; rep < 3 && !rc; ++rep) {
          if (rep == 1) rc = abi_hip((int)hipEventRecord(e0, s), "mhd_level_autotune: event");
          if (!rc) rc = abi_hip(enqueue_rhs(lv, 1, nullptr, nullptr, s), "mhd_level_autotune");
          if (!rc) rc = abi_hip(enqueue_stage(lv, 1, dt, s), "mhd_level_autotune");
        }
        if (!rc) rc = abi_hip((int)hipEventRecord(e1, s), "mhd_level_autotune: event");
        if (!rc) rc = abi_hip((int)hipEventSynchronize(e1), "mhd_level_autotune: sync");
        if (!rc) rc = abi_hip((int)hipEventElapsedTime(&ms, e0, e1), "mhd_level_autotune: time");
        if (!rc && ms < best_ms) {
          best_ms = ms;
          best = t;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if ((rc = mhd_level_set_tuning(lv, &best))) return rc;
  if (chosen) *chosen = best;
  return MHD_OK;
}

}  // extern "C"
