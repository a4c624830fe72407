// Optional per-kernel timing of the library's launches (host side).
//
// While profiling is switched on (mhd_profile_start), each launch site brackets
// its kernel with two HIP events recorded on the stream the kernel goes to, so
// the elapsed time between them is that kernel's duration on that stream.  When
// profiling is off, prof_begin is one relaxed atomic load.
#pragma once

#include <hip/hip_runtime.h>

namespace mhd {

enum KernelId : int {
  KID_CCZ4_STENCIL,
  KID_CCZ4_D2,
  KID_CCZ4_CURV,
  KID_CCZ4_GAUGE,
  KID_MHD_POINT,
  KID_MHD_UPDATE,
  KID_CON2PRIM,
  KID_PRIM2CON,
  KID_RK4_STAGE,
  KID_GHOSTS,
  KID_ZERO,
  KID_MLP_FEATURES,
  KID_MLP_NORMALIZE,
  KID_MLP_FORWARD,
  KID_MLP_GRAD,
  KID_MLP_GRAD_REDUCE,
  KID_MLP_ADAM,
  KID_C2P_LEARNED,
  KID_C2P_FALLBACK,
  KID_M1_POINT,
  KID_M1_UPDATE,
  KID_IMEX_COMBINE,
  KID_M1_IMPLICIT,
  KID_PROLONG,
  KID_RESTRICT,
  KID_DENSE,
  KID_SSPRK3_STAGE,
  KID_CONSTRAINTS,
  KID_CONSTRAINT_PLANES,
  KID_CONSTRAINT_TOTAL,
  KID_C2P_CLASSIFY,
  KID_LES,
  KID_COUNT
};

// returns a record handle (or -1 when profiling is off or the stream is being captured)
int prof_begin(int kid, hipStream_t s);
void prof_end(int rec, hipStream_t s);

}  // namespace mhd

// hipLaunchKernelGGL bracketed by the profiler's events
#define MHD_LAUNCH(kid, kernel, grid, block, shmem, stream, ...)                  \
  do {                                                                         \
    const int mhd_prof_rec_ = ::mhd::prof_begin((kid), (stream));              \
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);       \
    ::mhd::prof_end(mhd_prof_rec_, (stream));                                  \
  } while (0)
