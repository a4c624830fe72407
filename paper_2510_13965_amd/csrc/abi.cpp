// C ABI of the library (include/mhd.h): argument validation, geometry set-up
// and kernel launches.  No allocation happens here; every buffer is the
// caller's.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "../../include/mhd.h"
#include "dev_common.hpp"

namespace mhd {
int launch_ccz4(const Geom& g, const mhd_params_t& par, const double* U, const double* P, double* rhs, double* ws,
                int strip, const double* m1P, hipStream_t s);
int m1_workspace_fields(bool nd);
int les_workspace_fields();
int launch_les(const Geom& g, const mhd_eos_t& eos, double cm, const double* U, const double* P, double* ws,
               double* rhs, hipStream_t s);
int launch_m1_point(const Geom& g, const double* U, const double* P, const double* aux, double* ws, int nd,
                    hipStream_t s);
int launch_m1_update(const Geom& g, const double* U, const double* P, const double* aux, double* ws, double* rhs,
                     double* max_speed, double* stiff, int nd, double m_b, int coupled, hipStream_t s);
int launch_imex_combine(const Geom& g, int scheme, int nfields, int coupled, int stage, double dt, const double* Un,
                        const double* const* F, const double* const* R, double* Uout, hipStream_t s);
int launch_m1_implicit(const Geom& g, double* U, const double* P, const double* aux, double adt, int nd, int coupled,
                       double m_b, unsigned long long* nfail, hipStream_t s);
int ccz4_workspace_fields();
int launch_mhd(const Geom& g, const mhd_params_t& par, const mhd_eos_t& eos, const double* U, const double* P,
               double* ws, double* rhs, double* max_speed, int strip, hipStream_t s);
int launch_con2prim(const Geom& g, const mhd_eos_t& eos, double* U, double* P, uint8_t* flags, double* mu,
                    int64_t* stats, hipStream_t s);
int launch_prim2con(const Geom& g, const mhd_eos_t& eos, double* U, double* P, const double* EM, int eps_mode,
                    hipStream_t s);
int launch_rk4_stage(const Geom& g, int nfields, int stage, double dt, const double* Un, const double* k, double* acc,
                     double* Unext, hipStream_t s);
int launch_ghosts_periodic(const Geom& g, double* U, int nfields, hipStream_t s);
int launch_ssprk3_stage(const Geom& g, int nfields, int stage, double dt, const double* Un, const double* k,
                        double* acc, double* Unext, hipStream_t s);
int launch_zero_interior(const Geom& g, int f0, int nfields, double* A, hipStream_t s);
int launch_mlp_features(const Geom& g, const mhd_eos_t& eos, const double* U, const double* mu, float* X, float* T,
                        hipStream_t s);
int launch_mlp_normalize(float* prm, const float* X, int64_t n, hipStream_t s);
int launch_mlp_forward(const float* prm, const float* X, int64_t n, float* Y, hipStream_t s);
int mlp_grad_blocks(int64_t n);
int launch_prolong(const Geom& gc, const double* Uc, const Geom& gf, double* Uf, int nfields, const int off[3],
                   const int lo[3], const int n[3], hipStream_t s);
int launch_restrict(const Geom& gf, const double* Uf, const Geom& gc, double* Uc, int nfields, const int off[3],
                    const int lo[3], const int n[3], hipStream_t s);
int launch_constraints(const Geom& g, const double* U, double* C, double* sums, hipStream_t s);
int launch_dense_output(const Geom& g, int nfields, double dt, const double b[4], int add_un, double dtm,
                        const double* Un, const double* const* L, double* out, hipStream_t s);
int launch_mlp_grad(const float* prm, const float* X, const float* T, int64_t n, float* grad, float* loss, void* ws,
                    hipStream_t s);
int launch_mlp_adam(float* prm, const float* grad, float* m, float* v, int step, float lr, float b1, float b2,
                    float eps, hipStream_t s);
int launch_con2prim_learned(const Geom& g, const mhd_eos_t& eos, const float* prm, double* U, double* P,
                            uint8_t* flags, double* mu, int64_t* stats, void* ws, hipStream_t s);
int64_t noalloc_max_points();
int launch_con2prim_learned_noalloc(const Geom& g, const mhd_eos_t& eos, const float* prm, double* U, double* P,
                                    uint8_t* flags, double* mu, int64_t* stats, hipStream_t s);
}  // namespace mhd

namespace {

thread_local char g_err[512] = "";
// strip height (in 64x4 tiles) of the XCD-aware tile order of the stencil kernels
int g_strip = 4;

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_check(int rc, const char* what) {
  if (rc != (int)hipSuccess) return fail(MHD_EHIP, "%s: %s", what, hipGetErrorString((hipError_t)rc));
  g_err[0] = 0;
  return MHD_OK;
}

constexpr int64_t kMaxGridYZ = 65535;

int check_patch(const mhd_patch_t* pt, int need_ng, int nfields_z, const char* fn) {
  if (!pt) return fail(MHD_EINVAL, "%s: patch is NULL", fn);
  if (pt->nx < 1 || pt->ny < 1 || pt->nz < 1)
    return fail(MHD_EINVAL, "%s: interior extents must be >= 1 (got %d %d %d)", fn, pt->nx, pt->ny, pt->nz);
  if (pt->ng < 0 || pt->ng > 16) return fail(MHD_EINVAL, "%s: ghost width %d out of range", fn, pt->ng);
  if (need_ng >= 0 && pt->ng != need_ng) return fail(MHD_EINVAL, "%s: ghost width must be %d (got %d)", fn, need_ng, pt->ng);
  const int64_t Nx = pt->nx + 2 * pt->ng, Ny = pt->ny + 2 * pt->ng, Nz = pt->nz + 2 * pt->ng;
  if (pt->sy < Nx || pt->sz < pt->sy * Ny || pt->sf < pt->sz * Nz)
    return fail(MHD_EINVAL, "%s: strides (sy=%lld sz=%lld sf=%lld) too small for padded extents %lld x %lld x %lld", fn,
                (long long)pt->sy, (long long)pt->sz, (long long)pt->sf, (long long)Nx, (long long)Ny, (long long)Nz);
  if (!(pt->dx > 0.0 && pt->dy > 0.0 && pt->dz > 0.0)) return fail(MHD_EINVAL, "%s: spacings must be > 0", fn);
  if ((Ny + 3) / 4 > kMaxGridYZ || Nz * (int64_t)nfields_z > kMaxGridYZ)
    return fail(MHD_EINVAL, "%s: patch too large for one launch (Ny=%lld, Nz*fields=%lld)", fn, (long long)Ny,
                (long long)(Nz * nfields_z));
  return MHD_OK;
}

int check_eos(const mhd_eos_t* e, const char* fn) {
  if (!e) return fail(MHD_EINVAL, "%s: eos is NULL", fn);
  if (e->npieces < 1 || e->npieces > 4) return fail(MHD_EINVAL, "%s: eos npieces must be 1..4", fn);
  if (!(e->Gamma_th > 1.0)) return fail(MHD_EINVAL, "%s: Gamma_th must be > 1", fn);
  for (int i = 0; i < e->npieces; ++i)
    if (!(e->Gamma[i] > 1.0) || e->K[i] < 0.0) return fail(MHD_EINVAL, "%s: piece %d needs Gamma > 1, K >= 0", fn, i);
  for (int i = 0; i + 1 < e->npieces; ++i)
    if (!(e->rho_b[i] > 0.0) || (i > 0 && !(e->rho_b[i] > e->rho_b[i - 1])))
      return fail(MHD_EINVAL, "%s: piece boundaries must be positive and increasing", fn);
  if (!(e->rho_atm > 0.0 && e->rho_min >= e->rho_atm && e->rho_max > e->rho_min))
    return fail(MHD_EINVAL, "%s: need 0 < rho_atm <= rho_min < rho_max", fn);
  if (!(e->h0 > 0.0) || !(e->W_max > 1.0) || !(e->eps_max > 0.0))
    return fail(MHD_EINVAL, "%s: need h0 > 0, W_max > 1, eps_max > 0", fn);
  return MHD_OK;
}

mhd::Geom geom_of(const mhd_patch_t* pt) {
  mhd::Geom g;
  g.nx = pt->nx;
  g.ny = pt->ny;
  g.nz = pt->nz;
  g.ng = pt->ng;
  g.sy = pt->sy;
  g.sz = pt->sz;
  g.sf = pt->sf;
  g.idx[0] = 1.0 / pt->dx;
  g.idx[1] = 1.0 / pt->dy;
  g.idx[2] = 1.0 / pt->dz;
  const double h[3] = {pt->dx, pt->dy, pt->dz};
  for (int a = 0; a < 3; ++a) {
    g.h[a] = h[a];
    g.i12[a] = 1.0 / (12.0 * h[a]);
    g.i12s[a] = 1.0 / (12.0 * h[a] * h[a]);
  }
  return g;
}

}  // namespace

namespace mhd {
int abi_fail(int code, const char* msg) { return fail(code, "%s", msg); }
int abi_hip(int rc, const char* what) { return hip_check(rc, what); }
Geom abi_geom(const mhd_patch_t* p) { return geom_of(p); }
int abi_check_patch(const mhd_patch_t* p, int need_ng, const char* fn) { return check_patch(p, need_ng, 1, fn); }
}  // namespace mhd

extern "C" {

const char* mhd_last_error(void) { return g_err; }

int mhd_abi_version(void) { return MHD_ABI_VERSION; }

int mhd_set_tuning(const mhd_tuning_t* t) {
  if (!t) return fail(MHD_EINVAL, "mhd_set_tuning: NULL");
  if (t->strip < 1 || t->strip > 1024) return fail(MHD_EINVAL, "mhd_set_tuning: strip must be 1..1024");
  g_strip = t->strip;
  g_err[0] = 0;
  return MHD_OK;
}

int mhd_get_tuning(mhd_tuning_t* t) {
  if (!t) return fail(MHD_EINVAL, "mhd_get_tuning: NULL");
  *t = mhd_tuning_t{};
  t->strip = g_strip;
  t->block_threads = 256;
  return MHD_OK;
}

int mhd_eos_init_pwp(mhd_eos_t* e) {
  if (!e) return fail(MHD_EINVAL, "mhd_eos_init_pwp: eos is NULL");
  if (e->npieces < 1 || e->npieces > 4) return fail(MHD_EINVAL, "mhd_eos_init_pwp: npieces must be 1..4");
  e->a[0] = 0.0;
  for (int i = 1; i < e->npieces; ++i) {
    const double rb = e->rho_b[i - 1];
    const double Gm = e->Gamma[i - 1], G = e->Gamma[i];
    // p_cold continuous: K_i rb^G_i = K_{i-1} rb^G_{i-1}
    e->K[i] = e->K[i - 1] * std::pow(rb, Gm - G);
    // eps_cold continuous
    e->a[i] = e->a[i - 1] + e->K[i - 1] / (Gm - 1.0) * std::pow(rb, Gm - 1.0) - e->K[i] / (G - 1.0) * std::pow(rb, G - 1.0);
  }
  g_err[0] = 0;
  return MHD_OK;
}

int mhd_prim2con(const mhd_patch_t* patch, const mhd_eos_t* eos, double* U, double* P, const double* EM, int eps_mode,
                 void* stream) {
  int rc;
  if ((rc = check_patch(patch, -1, 1, "mhd_prim2con")) || (rc = check_eos(eos, "mhd_prim2con"))) return rc;
  if (!U || !P || !EM) return fail(MHD_EINVAL, "mhd_prim2con: U, P and EM must be non-NULL");
  if (eps_mode != 0 && eps_mode != 1) return fail(MHD_EINVAL, "mhd_prim2con: eps_mode must be 0 or 1");
  return hip_check(mhd::launch_prim2con(geom_of(patch), *eos, U, P, EM, eps_mode, (hipStream_t)stream),
                   "mhd_prim2con");
}

int mhd_con2prim(const mhd_patch_t* patch, const mhd_eos_t* eos, double* U, double* P, uint8_t* flags, double* mu,
                 int64_t* stats, void* stream) {
  int rc;
  if ((rc = check_patch(patch, -1, 1, "mhd_con2prim")) || (rc = check_eos(eos, "mhd_con2prim"))) return rc;
  if (!U || !P) return fail(MHD_EINVAL, "mhd_con2prim: U and P must be non-NULL");
  return hip_check(mhd::launch_con2prim(geom_of(patch), *eos, U, P, flags, mu, stats, (hipStream_t)stream),
                   "mhd_con2prim");
}

static int64_t padded_points(const mhd_patch_t* p) {
  return (int64_t)(p->nx + 2 * p->ng) * (p->ny + 2 * p->ng) * (p->nz + 2 * p->ng);
}

size_t mhd_con2prim_learned_workspace_size(const mhd_patch_t* patch) {
  if (!patch) return 0;
  // counts, two 4-byte queues, then (256-byte aligned) one 8-float row per point
  const size_t n = (size_t)padded_points(patch);
  return ((256 + 8 * n + 255) / 256) * 256 + 32 * n;
}

int mhd_con2prim_learned(const mhd_patch_t* patch, const mhd_eos_t* eos, const float* mlp, double* U, double* P,
                         uint8_t* flags, double* mu, int64_t* stats, void* workspace, size_t workspace_bytes,
                         void* stream) {
  int rc;
  if ((rc = check_patch(patch, -1, 1, "mhd_con2prim_learned")) || (rc = check_eos(eos, "mhd_con2prim_learned")))
    return rc;
  if (!U || !P || !mlp) return fail(MHD_EINVAL, "mhd_con2prim_learned: U, P and mlp must be non-NULL");
  if (padded_points(patch) >= ((int64_t)1 << 32))
    return fail(MHD_EINVAL, "mhd_con2prim_learned: the padded patch must have fewer than 2^32 points");
  if (!workspace || workspace_bytes < mhd_con2prim_learned_workspace_size(patch))
    return fail(MHD_EWORKSPACE, "mhd_con2prim_learned: workspace of %zu bytes needed (got %zu)",
                mhd_con2prim_learned_workspace_size(patch), workspace_bytes);
  return hip_check(mhd::launch_con2prim_learned(geom_of(patch), *eos, mlp, U, P, flags, mu, stats, workspace,
                                                (hipStream_t)stream),
                   "mhd_con2prim_learned");
}

int mhd_con2prim_learned_noalloc(const mhd_patch_t* patch, const mhd_eos_t* eos, const float* mlp, double* U,
                                 double* P, uint8_t* flags, double* mu, int64_t* stats, void* stream) {
  int rc;
  if ((rc = check_patch(patch, -1, 1, "mhd_con2prim_learned_noalloc")) ||
      (rc = check_eos(eos, "mhd_con2prim_learned_noalloc")))
    return rc;
  if (!U || !P || !mlp) return fail(MHD_EINVAL, "mhd_con2prim_learned_noalloc: U, P and mlp must be non-NULL");
  if (padded_points(patch) > mhd::noalloc_max_points())
    return fail(MHD_EINVAL, "mhd_con2prim_learned_noalloc: the padded patch has %lld points, at most %lld allowed",
                (long long)padded_points(patch), (long long)mhd::noalloc_max_points());
  return hip_check(mhd::launch_con2prim_learned_noalloc(geom_of(patch), *eos, mlp, U, P, flags, mu, stats,
                                                        (hipStream_t)stream),
                   "mhd_con2prim_learned_noalloc");
}

int mhd_mlp_features(const mhd_patch_t* patch, const mhd_eos_t* eos, const double* U, const double* mu, float* X,
                     float* T, void* stream) {
  int rc;
  if ((rc = check_patch(patch, -1, 1, "mhd_mlp_features")) || (rc = check_eos(eos, "mhd_mlp_features"))) return rc;
  if (!U || !X) return fail(MHD_EINVAL, "mhd_mlp_features: U and X must be non-NULL");
  return hip_check(mhd::launch_mlp_features(geom_of(patch), *eos, U, mu, X, T, (hipStream_t)stream),
                   "mhd_mlp_features");
}

int mhd_mlp_normalize(float* mlp, const float* X, int64_t n, void* stream) {
  if (!mlp || !X || n < 1) return fail(MHD_EINVAL, "mhd_mlp_normalize: need mlp, X and n >= 1");
  return hip_check(mhd::launch_mlp_normalize(mlp, X, n, (hipStream_t)stream), "mhd_mlp_normalize");
}

int mhd_mlp_forward(const float* mlp, const float* X, int64_t n, float* Y, void* stream) {
  if (!mlp || !X || !Y || n < 1) return fail(MHD_EINVAL, "mhd_mlp_forward: need mlp, X, Y and n >= 1");
  if (n > ((int64_t)1 << 31) - 256) return fail(MHD_EINVAL, "mhd_mlp_forward: n too large for one launch");
  return hip_check(mhd::launch_mlp_forward(mlp, X, n, Y, (hipStream_t)stream), "mhd_mlp_forward");
}

size_t mhd_mlp_grad_workspace_size(int64_t n) {
  if (n < 1) return 0;
  return 1024 * sizeof(double) + (size_t)mhd::mlp_grad_blocks(n) * MHD_MLP_NPARAM * sizeof(float);
}

int mhd_mlp_grad(const float* mlp, const float* X, const float* T, int64_t n, float* grad, float* loss,
                 void* workspace, size_t workspace_bytes, void* stream) {
  if (!mlp || !X || !T || !grad || n < 1) return fail(MHD_EINVAL, "mhd_mlp_grad: need mlp, X, T, grad and n >= 1");
  if (!workspace || workspace_bytes < mhd_mlp_grad_workspace_size(n))
    return fail(MHD_EWORKSPACE, "mhd_mlp_grad: workspace of %zu bytes needed (got %zu)", mhd_mlp_grad_workspace_size(n),
                workspace_bytes);
  return hip_check(mhd::launch_mlp_grad(mlp, X, T, n, grad, loss, workspace, (hipStream_t)stream), "mhd_mlp_grad");
}

int mhd_mlp_adam(float* mlp, const float* grad, float* m, float* v, int step, float lr, float beta1, float beta2,
                 float eps, void* stream) {
  if (!mlp || !grad || !m || !v) return fail(MHD_EINVAL, "mhd_mlp_adam: NULL array");
  if (step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return fail(MHD_EINVAL, "mhd_mlp_adam: need step >= 1, lr > 0, 0 <= beta < 1, eps > 0");
  return hip_check(mhd::launch_mlp_adam(mlp, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream),
                   "mhd_mlp_adam");
}

// fields of the base workspace: 33 of point fluxes and speeds (GRMHD), the CCZ4
// second derivatives, then the LES term's B^i and alpha G_B (6)
static int64_t base_workspace_fields() {
  return 33 + (int64_t)mhd::ccz4_workspace_fields() + (int64_t)mhd::les_workspace_fields();
}

size_t mhd_rhs_workspace_size(const mhd_patch_t* patch) {
  if (!patch) return 0;
  return (size_t)base_workspace_fields() * (size_t)patch->sf * sizeof(double);
}

size_t mhd_rhs_workspace_size_m1(const mhd_patch_t* patch) {
  if (!patch) return 0;
  return mhd_rhs_workspace_size(patch) + (size_t)mhd::m1_workspace_fields(false) * (size_t)patch->sf * sizeof(double);
}

size_t mhd_rhs_workspace_size_m1n(const mhd_patch_t* patch) {
  if (!patch) return 0;
  return mhd_rhs_workspace_size(patch) + (size_t)mhd::m1_workspace_fields(true) * (size_t)patch->sf * sizeof(double);
}

static int rhs_impl(const mhd_patch_t* patch, const mhd_params_t* params, const mhd_eos_t* eos, const double* U,
                    const double* P, const double* aux, double* rhs, double* stiff, double* max_speed, void* workspace,
                    size_t workspace_bytes, void* stream) {
  int rc;
  if ((rc = check_patch(patch, 3, MHD_NST, "mhd_rhs")) || (rc = check_eos(eos, "mhd_rhs"))) return rc;
  if (!params) return fail(MHD_EINVAL, "mhd_rhs: params is NULL");
  if (!U || !rhs) return fail(MHD_EINVAL, "mhd_rhs: U and rhs must be non-NULL");
  const uint32_t fl = params->flags;
  const bool m1 = (fl & MHD_EVOLVE_M1) != 0;
  const bool nd = m1 && (fl & MHD_EVOLVE_M1N) != 0;
  if ((fl & MHD_EVOLVE_M1N) && !m1) return fail(MHD_EINVAL, "mhd_rhs: MHD_EVOLVE_M1N needs MHD_EVOLVE_M1");
  if (nd && !std::isfinite(params->m_b)) return fail(MHD_EINVAL, "mhd_rhs: m_b must be finite");
  if ((fl & (MHD_EVOLVE_MHD | MHD_COUPLE_MATTER)) && !P)
    return fail(MHD_EINVAL, "mhd_rhs: P is required when the fluid is evolved or coupled");
  if (m1 && (!P || !aux)) return fail(MHD_EINVAL, "mhd_rhs: P and aux are required with MHD_EVOLVE_M1");
  if ((fl & MHD_EVOLVE_MHD) && !(params->c_b > 0.0)) return fail(MHD_EINVAL, "mhd_rhs: c_b must be > 0");
  if (!std::isfinite(params->les_cm)) return fail(MHD_EINVAL, "mhd_rhs: les_cm must be finite");
  if (params->f_alpha_kind != MHD_FALPHA_ONE && params->f_alpha_kind != MHD_FALPHA_HARMONIC)
    return fail(MHD_EINVAL, "mhd_rhs: unknown f_alpha_kind %d", params->f_alpha_kind);
  const size_t need = nd ? mhd_rhs_workspace_size_m1n(patch)
                        : (m1 ? mhd_rhs_workspace_size_m1(patch) : mhd_rhs_workspace_size(patch));
  if (!workspace || workspace_bytes < need)
    return fail(MHD_EWORKSPACE, "mhd_rhs: workspace of %zu bytes needed (got %zu)", need, workspace_bytes);
  if (patch->sf > (int64_t)(INT32_MAX / 8))
    return fail(MHD_EINVAL, "mhd_rhs: a padded field of %lld points exceeds the 2^28-point limit of one launch",
                (long long)patch->sf);
  const mhd::Geom g = geom_of(patch);
  hipStream_t s = (hipStream_t)stream;
  double* ws = (double*)workspace;
  double* ws_les = ws + (int64_t)(33 + mhd::ccz4_workspace_fields()) * patch->sf;
  double* ws_m1 = ws + base_workspace_fields() * patch->sf;
  if (m1 && (rc = hip_check(mhd::launch_m1_point(g, U, P, aux, ws_m1, nd ? 1 : 0, s), "mhd_rhs/m1 point"))) return rc;
  const bool radiation_matter = m1 && (fl & MHD_COUPLE_MATTER);
  if (fl & MHD_EVOLVE_SPACETIME) {
    if ((rc = hip_check(mhd::launch_ccz4(g, *params, U, P, rhs, ws + 33 * patch->sf, g_strip,
                                         radiation_matter ? ws_m1 : nullptr, s),
                        "mhd_rhs/ccz4")))
      return rc;
  } else {
    // frozen spacetime: the CCZ4 block of the RHS is zero at interior points
    if ((rc = hip_check(mhd::launch_zero_interior(g, 0, MHD_NST, rhs, s), "mhd_rhs/zero"))) return rc;
  }
  if (fl & MHD_EVOLVE_MHD) {
    if ((rc = hip_check(mhd::launch_mhd(g, *params, *eos, U, P, ws, rhs, max_speed, g_strip, s), "mhd_rhs/grmhd")))
      return rc;
    if (params->les_cm != 0.0 &&
        (rc = hip_check(mhd::launch_les(g, *eos, params->les_cm, U, P, ws_les, rhs, s), "mhd_rhs/les")))
      return rc;
  } else {
    if ((rc = hip_check(mhd::launch_zero_interior(g, MHD_NST, MHD_NMHD, rhs, s), "mhd_rhs/zero"))) return rc;
  }
  const int coupled = (stiff && (fl & MHD_COUPLE_EXCHANGE)) ? 1 : 0;
  if (m1 && (rc = hip_check(mhd::launch_m1_update(g, U, P, aux, ws_m1, rhs, max_speed, stiff, nd ? 1 : 0, params->m_b,
                                                  coupled, s),
                            "mhd_rhs/m1 update")))
    return rc;
  return MHD_OK;
}

int mhd_rhs(const mhd_patch_t* patch, const mhd_params_t* params, const mhd_eos_t* eos, const double* U,
            const double* P, const double* aux, double* rhs, double* max_speed, void* workspace,
            size_t workspace_bytes, void* stream) {
  return rhs_impl(patch, params, eos, U, P, aux, rhs, nullptr, max_speed, workspace, workspace_bytes, stream);
}

int mhd_rhs_split(const mhd_patch_t* patch, const mhd_params_t* params, const mhd_eos_t* eos, const double* U,
                  const double* P, const double* aux, double* rhs, double* stiff, double* max_speed, void* workspace,
                  size_t workspace_bytes, void* stream) {
  if (!params || !(params->flags & MHD_EVOLVE_M1) || !stiff)
    return fail(MHD_EINVAL, "mhd_rhs_split: needs MHD_EVOLVE_M1 and a stiff array");
  return rhs_impl(patch, params, eos, U, P, aux, rhs, stiff, max_speed, workspace, workspace_bytes, stream);
}

int mhd_imex_stiff_fields(int nfields, int coupled) {
  if (nfields != MHD_NU_M1 && nfields != MHD_NU_M1N)
    return fail(MHD_EINVAL, "mhd_imex_stiff_fields: nfields must be %d or %d", MHD_NU_M1, MHD_NU_M1N);
  const int nrad = nfields - 32;
  return coupled ? nrad + 4 + (nfields == MHD_NU_M1N ? 1 : 0) : nrad;
}

int mhd_imex_combine(const mhd_patch_t* patch, int scheme, int nfields, int coupled, int stage, double dt,
                     const double* Un, const double* const* F, const double* const* R, double* Uout, void* stream) {
  int rc;
  if (scheme != MHD_IMEX_442 && scheme != MHD_IMEX_332)
    return fail(MHD_EINVAL, "mhd_imex_combine: scheme must be MHD_IMEX_442 or MHD_IMEX_332");
  const int ns = scheme == MHD_IMEX_442 ? 4 : 3;
  if (nfields != MHD_NU_M1 && nfields != MHD_NU_M1N)
    return fail(MHD_EINVAL, "mhd_imex_combine: nfields must be %d or %d", MHD_NU_M1, MHD_NU_M1N);
  if ((rc = check_patch(patch, -1, nfields, "mhd_imex_combine"))) return rc;
  if (stage < 0 || stage > ns) return fail(MHD_EINVAL, "mhd_imex_combine: stage must be 0..%d", ns);
  if (!Un || !Uout || !F || !R) return fail(MHD_EINVAL, "mhd_imex_combine: NULL array");
  if (!std::isfinite(dt)) return fail(MHD_EINVAL, "mhd_imex_combine: dt must be finite");
  const int nread = stage < ns ? stage : ns;
  const double* f4[4] = {nullptr, nullptr, nullptr, nullptr};
  const double* r4[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int j = 0; j < nread; ++j) {
    if (!F[j] || !R[j]) return fail(MHD_EINVAL, "mhd_imex_combine: stage arrays %d missing", j);
    f4[j] = F[j];
    r4[j] = R[j];
  }
  if (Uout == Un && stage < ns) return fail(MHD_EINVAL, "mhd_imex_combine: Uout may alias Un only at the final stage");
  return hip_check(
      mhd::launch_imex_combine(geom_of(patch), scheme, nfields, coupled ? 1 : 0, stage, dt, Un, f4, r4, Uout,
                               (hipStream_t)stream),
      "mhd_imex_combine");
}

int mhd_m1_implicit(const mhd_patch_t* patch, const double* aux, double* U, const double* P, double adt,
                    unsigned flags, double m_b, uint64_t* nfail, void* stream) {
  int rc;
  if ((rc = check_patch(patch, -1, 1, "mhd_m1_implicit"))) return rc;
  if (!aux || !U || !P) return fail(MHD_EINVAL, "mhd_m1_implicit: aux, U and P are required");
  if (!(adt >= 0.0) || !std::isfinite(adt)) return fail(MHD_EINVAL, "mhd_m1_implicit: adt must be finite and >= 0");
  if (flags & ~(MHD_IMPLICIT_N | MHD_IMPLICIT_COUPLED)) return fail(MHD_EINVAL, "mhd_m1_implicit: unknown flags");
  if (!std::isfinite(m_b)) return fail(MHD_EINVAL, "mhd_m1_implicit: m_b must be finite");
  return hip_check(mhd::launch_m1_implicit(geom_of(patch), U, P, aux, adt, (flags & MHD_IMPLICIT_N) ? 1 : 0,
                                           (flags & MHD_IMPLICIT_COUPLED) ? 1 : 0, m_b,
                                           reinterpret_cast<unsigned long long*>(nfail), (hipStream_t)stream),
                   "mhd_m1_implicit");
}

int mhd_rk_stage(const mhd_patch_t* patch, int nfields, int stage, double dt, const double* Un, const double* k,
                 double* acc, double* Unext, void* stream) {
  int rc;
  if ((rc = check_patch(patch, -1, nfields > 0 ? nfields : 1, "mhd_rk_stage"))) return rc;
  if (nfields < 1) return fail(MHD_EINVAL, "mhd_rk_stage: nfields must be >= 1");
  if (stage < 0 || stage > 3) return fail(MHD_EINVAL, "mhd_rk_stage: stage must be 0..3");
  if (!Un || !k || !acc || !Unext) return fail(MHD_EINVAL, "mhd_rk_stage: NULL array");
  if (Unext == Un && stage != 3) return fail(MHD_EINVAL, "mhd_rk_stage: Unext may alias Un only at stage 3");
  if (!std::isfinite(dt)) return fail(MHD_EINVAL, "mhd_rk_stage: dt must be finite");
  return hip_check(mhd::launch_rk4_stage(geom_of(patch), nfields, stage, dt, Un, k, acc, Unext, (hipStream_t)stream),
                   "mhd_rk_stage");
}

int mhd_ssprk3_stage(const mhd_patch_t* patch, int nfields, int stage, double dt, const double* Un, const double* k,
                     double* acc, double* Unext, void* stream) {
  int rc;
  if ((rc = check_patch(patch, -1, nfields > 0 ? nfields : 1, "mhd_ssprk3_stage"))) return rc;
  if (nfields < 1) return fail(MHD_EINVAL, "mhd_ssprk3_stage: nfields must be >= 1");
  if (stage < 0 || stage > 2) return fail(MHD_EINVAL, "mhd_ssprk3_stage: stage must be 0..2");
  if (!Un || !k || !acc || !Unext) return fail(MHD_EINVAL, "mhd_ssprk3_stage: NULL array");
  if (Unext == Un && stage != 2) return fail(MHD_EINVAL, "mhd_ssprk3_stage: Unext may alias Un only at stage 2");
  if (!std::isfinite(dt)) return fail(MHD_EINVAL, "mhd_ssprk3_stage: dt must be finite");
  return hip_check(mhd::launch_ssprk3_stage(geom_of(patch), nfields, stage, dt, Un, k, acc, Unext, (hipStream_t)stream),
                   "mhd_ssprk3_stage");
}

// padded extent of a patch along axis a
static int64_t padded(const mhd_patch_t* p, int a) {
  const int n = a == 0 ? p->nx : (a == 1 ? p->ny : p->nz);
  return (int64_t)n + 2 * p->ng;
}

static double spacing(const mhd_patch_t* p, int a) { return a == 0 ? p->dx : (a == 1 ? p->dy : p->dz); }

// floor(t / 2) for any sign
static int64_t floor_half(int64_t t) { return t >= 0 ? t / 2 : -((-t + 1) / 2); }

int mhd_prolong(const mhd_patch_t* coarse, const double* Uc, const mhd_patch_t* fine, double* Uf, int nfields,
                const int32_t* offset, const int32_t* lo, const int32_t* hi, void* stream) {
  int rc;
  const char* fn = "mhd_prolong";
  if ((rc = check_patch(coarse, -1, 1, fn)) || (rc = check_patch(fine, -1, 1, fn))) return rc;
  if (nfields < 1 || !Uc || !Uf || !offset || !lo || !hi)
    return fail(MHD_EINVAL, "%s: need nfields >= 1 and non-NULL arrays", fn);
  if (Uc == Uf) return fail(MHD_EINVAL, "%s: coarse and fine arrays must differ", fn);
  int o3[3], l3[3], n3[3];
  for (int a = 0; a < 3; ++a) {
    if (!(spacing(coarse, a) == 2.0 * spacing(fine, a)))
      return fail(MHD_EINVAL, "%s: the coarse spacing must be twice the fine one on every axis", fn);
    if (lo[a] < 0 || hi[a] <= lo[a] || hi[a] > padded(fine, a))
      return fail(MHD_EINVAL, "%s: fine box [%d, %d) out of the padded fine patch on axis %d", fn, lo[a], hi[a], a);
    // coarse nodes needed over the box: copies at even t = I - off, six points around odd t
    const int64_t t0 = (int64_t)lo[a] - offset[a], t1 = (int64_t)hi[a] - 1 - offset[a];
    int64_t need_lo = INT64_MAX, need_hi = INT64_MIN;
    for (int64_t t : {t0, t0 + 1, t1 - 1, t1}) {
      if (t < t0 || t > t1) continue;
      const int64_t first = (t % 2 == 0) ? floor_half(t) : floor_half(t - 1) - 2;
      const int64_t last = (t % 2 == 0) ? floor_half(t) : floor_half(t - 1) + 3;
      need_lo = first < need_lo ? first : need_lo;
      need_hi = last > need_hi ? last : need_hi;
    }
    if (need_lo < 0 || need_hi >= padded(coarse, a))
      return fail(MHD_EINVAL, "%s: the box needs coarse nodes %lld..%lld on axis %d, outside the padded coarse patch",
                  fn, (long long)need_lo, (long long)need_hi, a);
    o3[a] = offset[a];
    l3[a] = lo[a];
    n3[a] = hi[a] - lo[a];
  }
  if ((n3[1] + 3) / 4 > kMaxGridYZ || n3[2] > kMaxGridYZ) return fail(MHD_EINVAL, "%s: box too large for one launch", fn);
  return hip_check(mhd::launch_prolong(geom_of(coarse), Uc, geom_of(fine), Uf, nfields, o3, l3, n3, (hipStream_t)stream),
                   fn);
}

int mhd_restrict(const mhd_patch_t* fine, const double* Uf, const mhd_patch_t* coarse, double* Uc, int nfields,
                 const int32_t* offset, const int32_t* lo, const int32_t* hi, void* stream) {
  int rc;
  const char* fn = "mhd_restrict";
  if ((rc = check_patch(coarse, -1, 1, fn)) || (rc = check_patch(fine, -1, 1, fn))) return rc;
  if (nfields < 1 || !Uc || !Uf || !offset || !lo || !hi)
    return fail(MHD_EINVAL, "%s: need nfields >= 1 and non-NULL arrays", fn);
  if (Uc == Uf) return fail(MHD_EINVAL, "%s: coarse and fine arrays must differ", fn);
  int o3[3], l3[3], n3[3];
  for (int a = 0; a < 3; ++a) {
    if (!(spacing(coarse, a) == 2.0 * spacing(fine, a)))
      return fail(MHD_EINVAL, "%s: the coarse spacing must be twice the fine one on every axis", fn);
    if (lo[a] < 0 || hi[a] <= lo[a] || hi[a] > padded(coarse, a))
      return fail(MHD_EINVAL, "%s: coarse box [%d, %d) out of the padded coarse patch on axis %d", fn, lo[a], hi[a], a);
    const int64_t f0 = 2 * (int64_t)lo[a] + offset[a], f1 = 2 * ((int64_t)hi[a] - 1) + offset[a];
    if (f0 < 0 || f1 >= padded(fine, a))
      return fail(MHD_EINVAL, "%s: the box maps to fine points %lld..%lld on axis %d, outside the padded fine patch",
                  fn, (long long)f0, (long long)f1, a);
    o3[a] = offset[a];
    l3[a] = lo[a];
    n3[a] = hi[a] - lo[a];
  }
  if ((n3[1] + 3) / 4 > kMaxGridYZ || n3[2] > kMaxGridYZ) return fail(MHD_EINVAL, "%s: box too large for one launch", fn);
  return hip_check(mhd::launch_restrict(geom_of(fine), Uf, geom_of(coarse), Uc, nfields, o3, l3, n3, (hipStream_t)stream),
                   fn);
}

int mhd_dense_output(const mhd_patch_t* patch, int nfields, double theta, double dt, int deriv, const double* Un,
                     const double* const* L, double* out, void* stream) {
  int rc;
  const char* fn = "mhd_dense_output";
  if ((rc = check_patch(patch, -1, nfields > 0 ? nfields : 1, fn))) return rc;
  if (nfields < 1 || !L || !out) return fail(MHD_EINVAL, "%s: need nfields >= 1, L and out", fn);
  if (deriv < 0 || deriv > 3) return fail(MHD_EINVAL, "%s: deriv must be 0..3", fn);
  if (deriv == 0 && !Un) return fail(MHD_EINVAL, "%s: Un is required for the value (deriv 0)", fn);
  if (!std::isfinite(theta) || !std::isfinite(dt) || (deriv > 0 && dt == 0.0))
    return fail(MHD_EINVAL, "%s: theta and dt must be finite (dt != 0 for derivatives)", fn);
  const double* l4[4];
  for (int j = 0; j < 4; ++j) {
    if (!L[j] || L[j] == out) return fail(MHD_EINVAL, "%s: stage array %d missing or aliasing out", fn, j);
    l4[j] = L[j];
  }
  // b_j(theta) of RK4's third-order dense output and their theta-derivatives
  // (Sec. 3.1): b1 = t - 3/2 t^2 + 2/3 t^3, b2 = b3 = t^2 - 2/3 t^3,
  // b4 = -1/2 t^2 + 2/3 t^3
  const double t = theta, t2 = t * t, t3 = t2 * t;
  double b[4];
  switch (deriv) {
    case 0:
      b[0] = t - 1.5 * t2 + 2.0 / 3.0 * t3;
      b[1] = b[2] = t2 - 2.0 / 3.0 * t3;
      b[3] = -0.5 * t2 + 2.0 / 3.0 * t3;
      break;
    case 1:
      b[0] = 1.0 - 3.0 * t + 2.0 * t2;
      b[1] = b[2] = 2.0 * t - 2.0 * t2;
      b[3] = -t + 2.0 * t2;
      break;
    case 2:
      b[0] = -3.0 + 4.0 * t;
      b[1] = b[2] = 2.0 - 4.0 * t;
      b[3] = -1.0 + 4.0 * t;
      break;
    default:
      b[0] = 4.0;
      b[1] = b[2] = -4.0;
      b[3] = 4.0;
  }
  const double dtm = deriv == 0 ? 1.0 : std::pow(dt, (double)deriv);
  return hip_check(mhd::launch_dense_output(geom_of(patch), nfields, dt, b, deriv == 0 ? 1 : 0, dtm, Un, l4, out,
                                            (hipStream_t)stream),
                   fn);
}

int mhd_fill_ghosts_periodic(const mhd_patch_t* patch, double* U, int nfields, void* stream) {
  int rc;
  if ((rc = check_patch(patch, -1, nfields > 0 ? nfields : 1, "mhd_fill_ghosts_periodic"))) return rc;
  if (nfields < 1 || !U) return fail(MHD_EINVAL, "mhd_fill_ghosts_periodic: need nfields >= 1 and U");
  if (patch->ng == 0) return MHD_OK;
  return hip_check(mhd::launch_ghosts_periodic(geom_of(patch), U, nfields, (hipStream_t)stream),
                   "mhd_fill_ghosts_periodic");
}

int mhd_constraints(const mhd_patch_t* patch, const double* U, double* C, double* sums, void* stream) {
  int rc;
  const char* fn = "mhd_constraints";
  if ((rc = check_patch(patch, -1, 1, fn))) return rc;
  if (patch->ng < 2) return fail(MHD_EINVAL, "%s: ghost width must be >= 2 (got %d)", fn, patch->ng);
  if (!U || !C || !sums) return fail(MHD_EINVAL, "%s: U, C and sums are required", fn);
  if (C == U) return fail(MHD_EINVAL, "%s: C must not alias U", fn);
  if (patch->sf > (int64_t)(INT32_MAX / 8))
    return fail(MHD_EINVAL, "%s: a padded field of %lld points exceeds the 2^28-point limit of one launch", fn,
                (long long)patch->sf);
  return hip_check(mhd::launch_constraints(geom_of(patch), U, C, sums, (hipStream_t)stream), fn);
}

}  // extern "C"
