// Per-kernel event timing behind mhd_profile_start / mhd_profile_stop.
#include "prof.hpp"

#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/mhd.h"

namespace mhd {
namespace {

const char* const kNames[KID_COUNT] = {"k_ccz4_stencil", "k_ccz4_d2",  "k_ccz4_curv", "k_ccz4_gauge",
                                       "k_mhd_point",    "k_mhd_update", "k_con2prim", "k_prim2con",
                                       "k_rk4_stage",    "k_ghosts_periodic", "k_zero_interior", "k_mlp_features",
                                       "k_mlp_normalize", "k_mlp_forward", "k_mlp_grad", "k_mlp_grad_reduce",
                                       "k_mlp_adam", "k_c2p_learned", "k_c2p_fallback", "k_m1_point",
                                       "k_m1_update", "k_imex_combine", "k_m1_implicit", "k_prolong",
                                       "k_restrict", "k_dense_output", "k_ssprk3_stage", "k_constraints",
                                       "k_constraint_planes", "k_constraint_total", "k_c2p_classify", "k_les"};

struct Rec {
  int kid;
  hipEvent_t e0, e1;
};

constexpr size_t kMaxRecords = 1 << 16;

std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<hipEvent_t> g_pool;  // events owned by the profiler, reused across sessions
size_t g_used = 0;
std::vector<Rec> g_recs;
int64_t g_dropped = 0;

hipEvent_t take_event() {
  if (g_used == g_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_pool.push_back(e);
  }
  return g_pool[g_used++];
}

}  // namespace

int prof_begin(int kid, hipStream_t s) {
  if (!g_on.load(std::memory_order_relaxed)) return -1;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_recs.size() >= kMaxRecords) {
    ++g_dropped;
    return -1;
  }
  hipEvent_t e0 = take_event(), e1 = take_event();
  if (!e0 || !e1 || hipEventRecord(e0, s) != hipSuccess) return -1;
  g_recs.push_back(Rec{kid, e0, e1});
  return (int)g_recs.size() - 1;
}

void prof_end(int rec, hipStream_t s) {
  if (rec < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (hipEventRecord(g_recs[rec].e1, s) != hipSuccess) g_recs[rec].e1 = nullptr;
}

}  // namespace mhd

extern "C" {

int mhd_profile_start(void) {
  std::lock_guard<std::mutex> lk(mhd::g_mu);
  mhd::g_recs.clear();
  mhd::g_used = 0;
  mhd::g_dropped = 0;
  mhd::g_on.store(1);
  return MHD_OK;
}

int mhd_profile_stop(mhd_kernel_time_t* out, int max_entries, int* n_entries) {
  using namespace mhd;
  g_on.store(0);
  std::lock_guard<std::mutex> lk(g_mu);
  double tot[KID_COUNT] = {0};
  int64_t cnt[KID_COUNT] = {0};
  int rc = MHD_OK;
  for (const Rec& r : g_recs) {
    float ms = 0.f;
    if (!r.e1 || hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) {
      rc = MHD_EHIP;
      continue;
    }
    tot[r.kid] += ms;
    cnt[r.kid] += 1;
  }
  int n = 0;
  for (int k = 0; k < KID_COUNT; ++k) {
    if (!cnt[k]) continue;
    if (out && n < max_entries) {
      std::memset(&out[n], 0, sizeof(out[n]));
      std::strncpy(out[n].name, kNames[k], sizeof(out[n].name) - 1);
      out[n].launches = cnt[k];
      out[n].total_ms = tot[k];
    }
    ++n;
  }
  if (n_entries) *n_entries = n;
  g_recs.clear();
  g_used = 0;
  return g_dropped ? MHD_EINVAL : rc;
}

}  // extern "C"
