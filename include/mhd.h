/*
 * mhd.h -- C ABI of the MI355X (gfx950) implementation of the MHDuet
 * method-of-lines right-hand side on one mesh patch (arXiv:2510.13965).
 *
 * The library evaluates d_t U = L(U) (Sec. 3, method of lines) for
 *   - the CCZ4 spacetime system with 1+log / Gamma-freezing gauge (Sec. 2.1),
 *     4th-order centred derivatives, one-sided advection derivatives and
 *     Kreiss-Oliger dissipation (Sec. 3.2);
 *   - the GRMHD balance laws with hyperbolic divergence cleaning (Sec. 2.2),
 *     in conservative form with Lax-Friedrichs flux splitting and MP5
 *     reconstruction (Sec. 3.3), characteristic speeds from App. B;
 *   - the per-point conserved-to-primitive recovery (App. D);
 *   - the explicit RK4 stage update of Table I.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * Memory: every array argument is a DEVICE pointer owned by the caller; the
 *   library never frees or retains it past the call (work is enqueued on
 *   `stream`, a hipStream_t; NULL means the default stream).  Struct
 *   arguments (mhd_patch_t, mhd_params_t, mhd_eos_t) are HOST pointers read
 *   during the call only.
 * Layout: structure of arrays, field-major.  Element (f, i, j, k) of a patch
 *   array lives at base[f*sf + k*sz + j*sy + i] with padded indices
 *   0 <= i < nx+2ng etc.  Interior points are ng <= i < ng+nx.
 * Evolved fields U (MHD_NU = 32): gt_xx gt_xy gt_xz gt_yy gt_yz gt_zz (0-5),
 *   At_xx..At_zz (6-11), chi (12), Khat (13), Theta (14), Ghat^x,y,z (15-17),
 *   alpha (18), beta^x,y,z (19-21), Dbar (22), DYebar (23), taubar (24),
 *   Sbar_x,y,z (25-27), Bbar^x,y,z (28-30), phibar (31); the MHD fields are
 *   densitized by sqrt(gamma) (Sec. 2.2).  With MHD_EVOLVE_M1, 12 more fields:
 *   per species s = 0, 1, 2 the densitized neutrino energy and flux Ebar,
 *   Fbar_x,y,z at 32 + 4 s (Sec. 2.3), and an aux array of MHD_NAUX fields
 *   (kappa_a, kappa_s, eta of species s at 3 s, 3 s + 1, 3 s + 2).  With
 *   MHD_EVOLVE_M1N as well, 3 more: the densitized neutrino number density
 *   Nbar of species s at 44 + s (Sec. 2.3; MHD_NU_M1N fields), and the aux
 *   array has MHD_NAUX_N fields: after the 9 above, the number absorption
 *   opacity kappa0_a and emissivity eta0 of species s at 9 + 2 s, 10 + 2 s.
 *   Species 0 is the electron neutrino, 1 its antineutrino.
 * Primitive fields P (MHD_NP = 8): rho, eps, p, v^x, v^y, v^z, W, Ye.
 * Errors: 0 on success; a negative MHD_E* code otherwise, with a message
 *   available from mhd_last_error() (per host thread).  Argument errors are
 *   detected before any work is enqueued.
 */
#ifndef MHD_H
#define MHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MHD_ABI_VERSION 6

#define MHD_NST 22
#define MHD_NMHD 10
#define MHD_NU 32
#define MHD_NU_M1 44 /* with three grey M1 species (MHD_EVOLVE_M1) */
#define MHD_NAUX 9   /* per species kappa_a, kappa_s, eta */
#define MHD_NU_M1N 47 /* with the three number densities as well (MHD_EVOLVE_M1N) */
#define MHD_NAUX_N 15 /* and per species kappa0_a, eta0 */
#define MHD_NP 8
#define MHD_NEM 4

/* return codes */
#define MHD_OK 0
#define MHD_EINVAL (-1)     /* invalid argument (shape, stride, pointer, parameter) */
#define MHD_EHIP (-2)       /* a HIP runtime call failed */
#define MHD_EWORKSPACE (-3) /* workspace missing or too small */

/* con2prim per-point flag bits (App. D error policy) */
#define MHD_FLAG_ATMO 1u        /* rho < rho_min: reset to atmosphere */
#define MHD_FLAG_EPS_LO 2u      /* eps < eps_cold(rho): raised to it */
#define MHD_FLAG_EPS_HI 4u      /* eps > eps_max in a low-density / BH region: lowered */
#define MHD_FLAG_VEL_LIMIT 8u   /* W > W_max in a low-density / BH region: rescaled */
#define MHD_FLAG_YE_RESET 16u   /* Ye out of range in a low-density / BH region */
#define MHD_FLAG_FALLBACK 32u   /* learned guess rejected, bracketed solver used */
#define MHD_FLAG_NOT_CONVERGED 64u /* bracketed solver hit its iteration cap */
#define MHD_FLAG_FATAL 128u     /* error the paper treats as fatal (rho > rho_max, ...) */

/* con2prim statistics slots (int64 counters, accumulated atomically) */
#define MHD_STAT_FATAL 0
#define MHD_STAT_CORRECTED 1
#define MHD_STAT_FALLBACK 2
#define MHD_STAT_ITERATIONS 3 /* root-function evaluations (Newton or bracketed, bracket ends included) */
#define MHD_NSTAT 8

/* flags of mhd_params_t.flags */
#define MHD_EVOLVE_SPACETIME 1u
#define MHD_EVOLVE_MHD 2u
#define MHD_COUPLE_MATTER 4u
#define MHD_EVOLVE_M1 8u /* grey M1 radiation, three species (Sec. 2.3): U has MHD_NU_M1 fields */
#define MHD_EVOLVE_M1N 16u /* with MHD_EVOLVE_M1: the number densities too (Sec. 2.3): MHD_NU_M1N fields */
/* with MHD_EVOLVE_M1, for mhd_rhs_split: the fluid's share of the collision
 * exchange is stiff too (see mhd_rhs_split); single patches only */
#define MHD_COUPLE_EXCHANGE 32u

/* f_alpha_kind: the slicing function f_alpha(alpha) of the lapse equation */
#define MHD_FALPHA_ONE 0      /* 1+log slicing, f_alpha = 1 (the paper's standard) */
#define MHD_FALPHA_HARMONIC 1 /* f_alpha = alpha/2 (harmonic slicing) */

/* One vertex-centred patch (Sec. 4): nx*ny*nz interior points surrounded by
 * ng ghost layers.  The RHS needs ng = 3 (MP5 window, KO and upwind stencils);
 * con2prim and prim2con accept any ng >= 0 and process every padded point.
 * Strides are in elements: x is contiguous, sy >= nx+2ng, sz >= sy*(ny+2ng),
 * sf >= sz*(nz+2ng). */
typedef struct {
  int32_t nx, ny, nz;
  int32_t ng;
  double dx, dy, dz;
  double x0, y0, z0; /* coordinate of the first interior point (informational) */
  int64_t sy, sz, sf;
} mhd_patch_t;

/* Hybrid EoS of Sec. 2.2: p = K_i rho^Gamma_i + (Gamma_th - 1) rho (eps - eps_cold),
 * eps_cold = a_i + K_i/(Gamma_i - 1) rho^(Gamma_i - 1) on rho_{i-1} <= rho < rho_i.
 * The ideal gas p = (Gamma-1) rho eps is npieces = 1, K[0] = 0, Gamma_th = Gamma.
 * Fill K[0], Gamma[], rho_b[], Gamma_th and call mhd_eos_init_pwp() to derive
 * K_i, a_i (i > 0) by continuity.  Thresholds follow App. D. */
typedef struct {
  int32_t npieces;   /* 1..4 */
  int32_t reserved;
  double K[4];
  double Gamma[4];
  double rho_b[3];
  double a[4];
  double Gamma_th;
  double rho_atm, rho_min, rho_max, eps_max, W_max, rho_low, alpha_bh, h0;
  double ye_min, ye_max, ye_atm;
} mhd_eos_t;

/* Physics parameters (Sec. 2.1 gauge and damping, Sec. 2.2 cleaning,
 * Sec. 3.2 KO strength, Sec. 3.3 MP5 alpha). */
typedef struct {
  double kappa_z, kappa_c, kappa_2, eta;
  double beta0[3];
  double sigma_ko, c_b, kappa_b, alpha_mp5, f_beta;
  int32_t f_alpha_kind;
  uint32_t flags; /* MHD_EVOLVE_SPACETIME | MHD_EVOLVE_MHD | MHD_COUPLE_MATTER | MHD_EVOLVE_M1 | MHD_EVOLVE_M1N */
  double m_b;     /* reference baryon mass of the electron-fraction source (Sec. 2.2), with MHD_EVOLVE_M1N */
  double les_cm;  /* C_M of the gradient SGS (LES) term of the induction equation (App. A; the paper uses 8);
                     0 switches the term off.  Single patches only (mhd_level_create rejects it). */
} mhd_params_t;

/* Launch tuning.  The results never depend on it (bitwise).
 * strip: height, in tiles, of the strips in which each XCD walks its
 *   contiguous range of tiles (z fastest inside a strip); 1..1024.  Used by
 *   the single-patch stencil kernels (process-wide, set with mhd_set_tuning
 *   before enqueuing work, not concurrently with launches from other host
 *   threads) and per level (mhd_level_set_tuning).
 * block_threads: level kernels only: threads per workgroup = points per tile
 *   (a tile is that many consecutive points of one z plane); 64, 128 or 256.
 * grid_per_cu: level kernels only: persistent grid of grid_per_cu workgroups
 *   per compute unit, each looping over tiles; 0 launches one workgroup per
 *   tile. */
typedef struct {
  int32_t strip;
  int32_t block_threads;
  int32_t grid_per_cu;
  int32_t reserved[5];
} mhd_tuning_t;

int mhd_set_tuning(const mhd_tuning_t* t);
int mhd_get_tuning(mhd_tuning_t* t);

/* Per-kernel timing, for benchmarks.  Between mhd_profile_start() and
 * mhd_profile_stop() every kernel the library launches (outside stream
 * capture) is bracketed by two HIP events recorded on the stream it is launched
 * on; stop waits for the recorded events and returns, per kernel name, the
 * number of launches and the summed event-to-event time.  Up to 65536 launches
 * are recorded per session (more: stop returns MHD_EINVAL after filling `out`).
 * out: host array of max_entries records (may be NULL); *n_entries receives
 * the number of kernels seen.  Process-wide; not for concurrent sessions. */
typedef struct {
  char name[40];
  int64_t launches;
  double total_ms;
} mhd_kernel_time_t;

int mhd_profile_start(void);
int mhd_profile_stop(mhd_kernel_time_t* out, int max_entries, int* n_entries);

/* Message of the last failed call on this host thread ("" if none). */
const char* mhd_last_error(void);
int mhd_abi_version(void);

/* Derive K_i (i>0) and a_i from K[0], Gamma[], rho_b[] by continuity of
 * p_cold and eps_cold at the piece boundaries (Sec. 2.2, a_0 = 0).  Host only. */
int mhd_eos_init_pwp(mhd_eos_t* eos);

/* prim -> cons (definitions of Sec. 2.2, App. D) at every padded point.
 * In: U[0..21] (spacetime, read), P slots rho, eps, v^i, Ye, and EM (4 fields:
 *   undensitized B^x, B^y, B^z, phi; field stride patch->sf).
 * Out: U[22..31] (densitized conserved fields), P slots p and W.
 * eps_mode 0: P[eps] is the specific internal energy; 1: it is the thermal part
 *   and eps_cold(rho) is added (the total is written back to P[eps]). */
int mhd_prim2con(const mhd_patch_t* patch, const mhd_eos_t* eos, double* U, double* P,
                 const double* EM, int eps_mode, void* stream);

/* cons -> prim (App. D) at every padded point: mu_+ root of f_a on (0, 1/h0],
 * mu root of f on (0, mu_+], both by Brent's method to a few ulp, primitives
 * from mu, then the error policy.  Corrected points get their conserved fields
 * (U[22..27]) rewritten from the corrected primitives.
 * In/out: U.  Out: P (8 fields), flags (uint8 per padded point, may be NULL),
 *   mu (2 fields mu_+, mu with stride patch->sf, may be NULL),
 *   stats (MHD_NSTAT int64 device counters, accumulated, may be NULL).
 * Returns MHD_OK or an error code, not the number of fatal points: a count
 * returned to the host would need a device-to-host copy and a stream
 * synchronisation on every call (no asynchronous steps, no graph capture).
 * Points the paper treats as fatal (App. D: density above rho_max) get
 * MHD_FLAG_FATAL and are counted in stats[MHD_STAT_FATAL]; the caller reads
 * the counter when it decides to stop. */
int mhd_con2prim(const mhd_patch_t* patch, const mhd_eos_t* eos, double* U, double* P,
                 uint8_t* flags, double* mu, int64_t* stats, void* stream);

/* ---- learned starting guess for con2prim ------------------------------------
 * A small MLP (8 -> 64 -> 64 -> 2, ReLU; hidden layers on bf16 matrix cores with
 * FP32 accumulation) predicts the two roots of App. D from 8 metric-invariant
 * scalars of the state: log10 D, log10 q, log10 r^2, log10 calB^2,
 * (r.calB)^2 / (r^2 calB^2), log10(1+q), log10 r^2/(1+q)^2, log10 calB^2/(1+q)
 * (q = tau/D, r_i = S_i/D, calB^i = B^i/sqrt(D); tiny floors keep the logs
 * finite).  Outputs: corrections y0, y1 to closed-form approximations b0, b1
 * of log(mu_+ h0) and log(mu / mu_+) (log fractions of the upper ends of the
 * two brackets): b0 = log h0 - log(h0^2 + r^2)/2 (exact without magnetic
 * field), b1 = -log(1 + q) + log(h0^2 + r^2)/2 (mu ~ 1/(1 + q)); the guesses
 * are mu_+ = exp(min(b0 + y0, 0))/h0 and mu = mu_+ exp(min(b1 + y1, 0)).
 * Parameter block (float32, device, MHD_MLP_NBLOCK floats): W1[64][8] at 0,
 * b1[64] at 512, W2[64][64] at 576, b2[64] at 4672, W3[2][64] at 4736, b3[2] at
 * 4864 (the MHD_MLP_NPARAM trainable values), feature mean[8] at 4866 and
 * inverse standard deviation[8] at 4874. */
#define MHD_MLP_NPARAM 4866
#define MHD_MLP_NBLOCK 4882

/* con2prim (App. D) with the learned guess: per padded point, the network
 * guesses mu_+ and mu; each is polished by at most 3 Newton iterations in FP64
 * and accepted when the residual is <= 1e-12 (|f_a|, and |f| relative to mu)
 * with 0 < mu <= mu_+ and the function has the opposite sign 5e-13 (relative)
 * away on the side the residual points to, so an accepted root is within
 * 5e-13 relative of the bracketed one.  Rejected points are queued and finished by the same
 * bracketed solver as mhd_con2prim (their flag gets MHD_FLAG_FALLBACK).  The
 * error policy, outputs and U rewrite are those of mhd_con2prim; stats also
 * counts MHD_STAT_FALLBACK points and, in MHD_STAT_ITERATIONS, Newton
 * evaluations plus bracketed iterations.
 * workspace: device buffer of mhd_con2prim_learned_workspace_size() bytes
 * (the fallback queue); the padded patch must have < 2^32 points. */
size_t mhd_con2prim_learned_workspace_size(const mhd_patch_t* patch);
int mhd_con2prim_learned(const mhd_patch_t* patch, const mhd_eos_t* eos, const float* mlp, double* U, double* P,
                         uint8_t* flags, double* mu, int64_t* stats, void* workspace, size_t workspace_bytes,
                         void* stream);

/* Allocation-free variant of mhd_con2prim_learned, for callers that cannot
 * allocate device memory (code under stream or graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same kernels, arguments, outputs
 * and results as mhd_con2prim_learned, without the workspace: the two queues
 * and the network's rows live in a file-scope device array of the library,
 * 512 + 40 * 2^22 bytes (160 MiB) per device, held from the first call on a
 * device until the process ends.  The padded patch must have at most 2^22 points (4 194 304; a 155^3
 * padded patch fits), else MHD_EINVAL.  The call allocates nothing; its first
 * call on a device looks up the array's address (MHD_EHIP if that fails) with
 * that device current, and the stream must belong to the current device.
 * Every call on a device shares that device's array, whose queue counts the
 * call clears by a kernel on `stream` before use: calls that overlap on one device
 * (different streams, or threads without ordering between their streams)
 * race and give wrong answers. */
int mhd_con2prim_learned_noalloc(const mhd_patch_t* patch, const mhd_eos_t* eos, const float* mlp, double* U,
                                 double* P, uint8_t* flags, double* mu, int64_t* stats, void* stream);

/* Training set-up and steps (device arrays, row-major):
 * mhd_mlp_features: X[N][8] raw features (float32) of every padded point in
 *   linear padded order (i fastest); points with D < rho_min get NaN rows.
 *   If mu (2 fields mu_+, mu, as written by mhd_con2prim) and T are non-NULL,
 *   T[N][2] gets the targets log(mu_+ h0) - b0, log(mu/mu_+) - b1.
 * mhd_mlp_normalize: mean and inverse std of each feature over the non-NaN rows
 *   of X[n][8], written into the parameter block.
 * mhd_mlp_forward: Y[n][2] network outputs for raw features X[n][8].
 * mhd_mlp_grad: grad[MHD_MLP_NPARAM] = dL/dtheta and *loss = L (device float,
 *   may be NULL) for L = 1/(2n) sum over non-NaN rows of |y - t|^2; the same
 *   bf16 rounding as the forward pass; deterministic (fixed reduction order).
 *   workspace: mhd_mlp_grad_workspace_size(n) bytes.
 * mhd_mlp_adam: one Adam step (step counts from 1) on the trainable
 *   parameters, with moment buffers m, v[MHD_MLP_NPARAM] (zeroed before step 1). */
int mhd_mlp_features(const mhd_patch_t* patch, const mhd_eos_t* eos, const double* U, const double* mu, float* X,
                     float* T, void* stream);
int mhd_mlp_normalize(float* mlp, const float* X, int64_t n, void* stream);
int mhd_mlp_forward(const float* mlp, const float* X, int64_t n, float* Y, void* stream);
size_t mhd_mlp_grad_workspace_size(int64_t n);
int mhd_mlp_grad(const float* mlp, const float* X, const float* T, int64_t n, float* grad, float* loss,
                 void* workspace, size_t workspace_bytes, void* stream);
int mhd_mlp_adam(float* mlp, const float* grad, float* m, float* v, int step, float lr, float beta1, float beta2,
                 float eps, void* stream);

/* ---- batched levels ---------------------------------------------------------
 * All boxes of one refinement level (patches of any shape, ng = 3, each with its
 * own arrays) go through one persistent kernel per phase of the right-hand
 * side; an RK4 step is 33 launches (41 with M1) whatever the number of boxes, and can be
 * replayed as one hipGraph.  Per point the arithmetic is that of the
 * single-patch entry points, so results are bitwise equal to per-box calls of
 * mhd_con2prim, mhd_rhs and mhd_rk_stage.  Ghost values are taken as given
 * (frozen; the level does not exchange or fill them).  The level evolves the
 * full coupled system (params->flags must hold MHD_EVOLVE_SPACETIME,
 * MHD_EVOLVE_MHD and MHD_COUPLE_MATTER); with MHD_EVOLVE_M1 as well, every box
 * also evolves the three grey M1 species (Sec. 2.3, 3.4): U, Us, k and acc then
 * hold MHD_NU_M1 fields, aux is required and the workspace is
 * mhd_rhs_workspace_size_m1() bytes; the results are bitwise those of per-box
 * mhd_rhs with MHD_EVOLVE_M1 and mhd_rk_stage over 44 fields.  With
 * MHD_EVOLVE_M1N too, the three number densities as well (Sec. 2.3): MHD_NU_M1N
 * fields, MHD_NAUX_N aux fields, mhd_rhs_workspace_size_m1n() bytes, and
 * params->m_b finite.  The LES term (les_cm != 0) is rejected: single patches
 * only.
 * mhd_level_create copies the descriptors to the device (the only allocation,
 * with a capture stream); the arrays stay the caller's and must outlive it. */
typedef struct {
  mhd_patch_t patch;
  double* U;        /* state at t^n (32, 44 or 47 fields); the RK4 step updates it in place */
  double* Us;       /* stage state (as U) */
  double* P;        /* primitives (8 fields) */
  double* k;        /* right-hand side (as U) */
  double* acc;      /* RK4 accumulator (as U) */
  void* workspace;  /* mhd_rhs_workspace_size(&patch) bytes or more (_m1 with M1, _m1n with M1N) */
  size_t workspace_bytes;
  uint8_t* flags;   /* con2prim flags, may be NULL */
  const double* aux; /* MHD_NAUX fields (kappa_a, kappa_s, eta per species) with MHD_EVOLVE_M1, MHD_NAUX_N
                        with MHD_EVOLVE_M1N, else NULL */
} mhd_box_t;

typedef struct mhd_level mhd_level_t;

int mhd_level_create(const mhd_box_t* boxes, int nboxes, const mhd_params_t* params, const mhd_eos_t* eos,
                     mhd_level_t** level);
int mhd_level_destroy(mhd_level_t* level);
/* Tuning of the level's launches (see mhd_tuning_t); waits for the device. */
int mhd_level_set_tuning(mhd_level_t* level, const mhd_tuning_t* tuning);
int mhd_level_get_tuning(const mhd_level_t* level, mhd_tuning_t* tuning);
/* con2prim + L(U) of every box, evaluated at U (src 0) or Us (src 1), into k;
 * max_speed (device double, may be NULL) gets an atomic max as in mhd_rhs;
 * stats (may be NULL) accumulates the con2prim counters. */
int mhd_level_rhs(mhd_level_t* level, int src, double* max_speed, int64_t* stats, void* stream);
/* One RK4 step of size dt (Table I) of every box: four evaluations and stage
 * updates; U is advanced in place.  max_speed (may be NULL) is zeroed and then
 * receives the maximum over the four evaluations.  use_graph != 0: the step is
 * captured once into a hipGraph (again whenever dt or max_speed change) and
 * replayed on `stream`. */
int mhd_level_rk4_step(mhd_level_t* level, double dt, double* max_speed, int use_graph, void* stream);
/* Times the candidate tunings (block_threads 64/128/256 x strip 1/4/16 x
 * grid_per_cu 0/4/16) on one evaluation at Us plus a stage-1 update, and keeps
 * the fastest.  It overwrites Us, P, k, acc, flags and the workspaces; U is only
 * read.  chosen may be NULL. */
int mhd_level_autotune(mhd_level_t* level, double dt, void* stream, mhd_tuning_t* chosen);

/* Use the learned con2prim guess (as mhd_con2prim_learned, over all boxes, with
 * one fallback queue) in the level's con2prim phase; mlp = NULL returns to the
 * bracketed solver.  workspace: mhd_level_learned_workspace_size() bytes.  Both
 * must outlive their use by the level; waits for the device. */
size_t mhd_level_learned_workspace_size(const mhd_level_t* level);
int mhd_level_set_learned(mhd_level_t* level, const float* mlp, void* workspace, size_t workspace_bytes);

/* IMEX(4,4,2) on a batched level (Table I; App. C), for a level that evolves M1.
 * mhd_level_set_imex: per box (same order as at creation), the explicit parts
 *   F[s] (MHD_NU_M1 fields, MHD_NU_M1N with the number densities) and stiff
 *   parts R[s] (12 fields, 15 with the number densities) of the four
 *   stages, device arrays in the box's patch layout, caller-owned, outliving
 *   their use; boxes = NULL detaches them.  Waits for the device.
 * mhd_level_imex_step: one step of size dt of every box, per box and stage the
 *   sequence of the single-patch entry points (mhd_imex_combine into Us,
 *   mhd_con2prim or the learned guess, mhd_m1_implicit with a_ii dt where
 *   a_ii != 0, mhd_rhs_split into F[s] and R[s]), then the final combination
 *   into U (advanced in place); results are bitwise those per-box calls.
 *   Ghosts stay frozen.  max_speed (may be NULL) is zeroed and then receives the
 *   maximum over the four evaluations; nfail (device uint64, may be NULL) is
 *   incremented per collision solve that did not converge.  use_graph != 0:
 *   captured once (again when dt, max_speed or nfail change) and replayed. */
typedef struct {
  double* F[4];
  double* R[4];
} mhd_imex_box_t;

int mhd_level_set_imex(mhd_level_t* level, const mhd_imex_box_t* boxes, int nboxes);
int mhd_level_imex_step(mhd_level_t* level, double dt, double* max_speed, uint64_t* nfail, int use_graph,
                        void* stream);

/* Workspace bytes mhd_rhs needs for this patch (point fluxes and speeds). */
size_t mhd_rhs_workspace_size(const mhd_patch_t* patch);

/* Workspace of mhd_rhs with MHD_EVOLVE_M1 (closure, point fluxes, speeds). */
size_t mhd_rhs_workspace_size_m1(const mhd_patch_t* patch);

/* Workspace of mhd_rhs with MHD_EVOLVE_M1 | MHD_EVOLVE_M1N (as _m1, plus the
 * number densities' point fluxes and the factors Gamma). */
size_t mhd_rhs_workspace_size_m1n(const mhd_patch_t* patch);

/* L(U) at the interior points (Sec. 2.1, 2.2, 2.3, 3.2, 3.3, 3.4, App. B).
 * In: U (32 fields incl. ghosts, 44 with MHD_EVOLVE_M1, 47 with
 *   MHD_EVOLVE_M1N too), P (8 fields incl. ghosts; from con2prim), aux
 *   (MHD_NAUX fields with MHD_EVOLVE_M1, MHD_NAUX_N with MHD_EVOLVE_M1N;
 *   else ignored and may be NULL).
 * Out: rhs (32, 44 or 47 fields, interior points only; ghost entries untouched).
 *   With MHD_EVOLVE_M1 the radiation also enters the CCZ4 matter terms (if
 *   MHD_COUPLE_MATTER) and exchanges energy and momentum with the fluid.
 *   With MHD_EVOLVE_M1N the number densities are evolved (Sec. 2.3): number
 *   current N^a = n (u^a + H^a/J) of the closure's J and H^a, so the d_k-flux
 *   of Nbar is (-W beta^k + alpha W v^k + alpha H^k/J) Nbar/Gamma with
 *   Gamma = W (E - F_i v^i)/J and H^k = gamma^kj H_j + W (J - E + F_i v^i)
 *   beta^k/alpha; HO/LO interfaces as the energy moments' (Sec. 3.4, the
 *   species' speed and kappa_a + kappa_s); source alpha sqrt(gamma) C with
 *   C = eta0 - kappa0_a N/Gamma; and the electron fraction's DYebar gains
 *   -alpha sqrt(gamma) m_b (C_0 - C_1) (Sec. 2.2).
 *   With params->les_cm != 0 (and MHD_EVOLVE_MHD) the gradient SGS term of
 *   App. A enters the induction equation: the flux of Bbar^i along k gains
 *   -alpha G_B^{ki}, G_B^{ki} = -C_M xi sqrt(gamma) H_M^{ki}, xi = gamma^(1/3)
 *   Delta^2/24 with Delta^2 = (dx dy dz)^(2/3), H_M^{ki} = B^i H_v^k - B^k H_v^i
 *   + 2 (grad B^i . grad v^k - grad B^k . grad v^i) (dot products with
 *   gamma^jl), H_v the velocity part of the primitives' second-order response
 *   to filtering the conserved fields (the quantity App. A's closed forms
 *   abbreviate); first derivatives of the primitives by 4th-order centred
 *   differences, the divergence by 2nd-order centred ones.
 * max_speed: device double, max over interior points and axes of the point
 *   speed (fast magnetosonic bound and cleaning mode, and the M1 speed);
 *   updated with an atomic max, the caller initialises it (to 0).  May be NULL.
 * workspace: device buffer of mhd_rhs_workspace_size() bytes
 *   (mhd_rhs_workspace_size_m1() with MHD_EVOLVE_M1). */
int mhd_rhs(const mhd_patch_t* patch, const mhd_params_t* params, const mhd_eos_t* eos,
            const double* U, const double* P, const double* aux, double* rhs, double* max_speed,
            void* workspace, size_t workspace_bytes, void* stream);

/* ---- IMEX(4,4,2) of Table I for the stiff radiation collisions (App. C) -----
 * mhd_rhs_split: as mhd_rhs with MHD_EVOLVE_M1, but the radiation's collision
 *   terms alpha sqrt(gamma) (S_n, S_i) (the stiff part) go to `stiff` (12
 *   fields, species-major, patch layout; with MHD_EVOLVE_M1N 15, the number
 *   densities' alpha sqrt(gamma) C at 12 + s) instead of rhs; the fluid's
 *   opposite exchange and the electron fraction's source stay in rhs
 *   (explicit).  With MHD_COUPLE_EXCHANGE in params->flags they go to
 *   `stiff` too, after the radiation's: the fluid's share at 12 (15 with
 *   MHD_EVOLVE_M1N) + 0 (taubar) and + 1..3 (Sbar_i), summed over the
 *   species, and the electron fraction's at 15 + 4; mhd_imex_stiff_fields()
 *   gives the count (12, 15, 16 or 20).  Taken with mhd_imex_combine's
 *   coupled and mhd_m1_implicit's MHD_IMPLICIT_COUPLED, the exchange is then
 *   implicit for both sides and conserves energy, momentum and lepton number
 *   at every stage (the fluid's primitives are held during the solve, as App.
 *   C holds them).
 * mhd_imex_combine: for scheme MHD_IMEX_442 (Table I: explicit RK4 with the
 *   L-stable I42L, ns = 4 stages) or MHD_IMEX_332 (Table II's SSP-RK(3,3)
 *   with an L-stable I32L re-derived from Sec. 3.1's order and L-stability
 *   conditions, ns = 3: the printed implicit half is first order, its rows
 *   summing to (0, 1, 1) against its c = (0, 1, 1/2); the re-derived one keeps
 *   the printed first row, c and b, with diagonal gamma = 1 - 1/sqrt(2): rows
 *   (0,0,0), (1 - gamma, gamma, 0), (1/2 - gamma - a32, a32, gamma),
 *   a32 = 3 gamma (1 - 2 gamma)/4), at the interior points of all nfields
 *   fields (44, or 47 with the number densities), stage s = 0..ns-1:
 *   Uout = Un + dt sum_{j<s} AE[s][j] F[j], and on the radiation fields (32
 *   and up) also + dt sum_{j<s} AI[s][j] R[j] (the explicit state V* of the
 *   stage); s = ns: Uout = Un + dt sum_i (BE[i] F[i] + BI[i] R[i]) (radiation)
 *   and Un + dt sum_i BE[i] F[i] (other fields).  With coupled != 0 the
 *   fluid's taubar, Sbar_i (and DYe with the number densities) take their
 *   stiff slots as the radiation does.  F, R: host arrays of 4 device pointers
 *   to stage explicit (nfields fields) and stiff
 *   (mhd_imex_stiff_fields(nfields, coupled) fields) parts; only the entries
 *   the stage reads must be set.  Uout may
 *   alias Un only at s = ns.  The implicit solve of stage s takes
 *   adt = AI[s][s] dt.
 * mhd_m1_implicit: at the interior points, per species, replaces the radiation
 *   fields V* of U by the solution V of V = V* + adt alpha (S_n, S_i)(V)
 *   (undensitized), the fluid state from P, the closure's Eddington factor
 *   frozen at its value for V*; Newton's method with the exact Jacobian, at
 *   most 60 iterations, converged at |dV| <= 1e-15 (E + |F|) or once an update
 *   no larger than 1e-9 (E + |F|) is not below half of the previous one (the
 *   rounding floor: App. C leaves the stopping rule open).  A solve that does
 *   not converge (singular Jacobian, or 60 iterations) keeps the first Newton
 *   iterate, App. C's linearised implicit update about V*; nfail (device
 *   uint64, may be NULL) is incremented per such species solve.  flags:
 *   MHD_IMPLICIT_N (U of 47 fields, aux of MHD_NAUX_N): each species' number
 *   density then takes App. C's closed-form implicit update
 *   N = (N* + adt alpha eta0)/(1 + adt alpha kappa0_a/Gamma), Gamma from the
 *   updated E, F_i and their closure; MHD_IMPLICIT_COUPLED: the fluid's taubar
 *   and Sbar_i then lose what each species' Ebar and Fbar_i gained, and DYe
 *   (with MHD_IMPLICIT_N) loses m_b times the gain of (Nbar_nue -
 *   Nbar_nuebar).  m_b is read only then; it must be finite. */
int mhd_rhs_split(const mhd_patch_t* patch, const mhd_params_t* params, const mhd_eos_t* eos, const double* U,
                  const double* P, const double* aux, double* rhs, double* stiff, double* max_speed, void* workspace,
                  size_t workspace_bytes, void* stream);
#define MHD_IMEX_442 0
#define MHD_IMEX_332 1
int mhd_imex_stiff_fields(int nfields, int coupled);
int mhd_imex_combine(const mhd_patch_t* patch, int scheme, int nfields, int coupled, int stage, double dt,
                     const double* Un, const double* const* F, const double* const* R, double* Uout, void* stream);
#define MHD_IMPLICIT_N 1u
#define MHD_IMPLICIT_COUPLED 2u
int mhd_m1_implicit(const mhd_patch_t* patch, const double* aux, double* U, const double* P, double adt,
                    unsigned flags, double m_b, uint64_t* nfail, void* stream);

/* Explicit RK4 stage of Table I at the interior points of `nfields` fields:
 *   stage s (0..3): acc = (s ? acc : 0) + b_s k;  s < 3: Unext = Un + dt a_{s+1,s} k;
 *   s = 3: Unext = Un + dt acc.
 * Unext may alias Un only for s = 3.  Ghost entries of Unext are untouched. */
int mhd_rk_stage(const mhd_patch_t* patch, int nfields, int stage, double dt, const double* Un,
                 const double* k, double* acc, double* Unext, void* stream);

/* Explicit SSP-RK(3,3) stage of Shu and Osher (Sec. 3.1, the explicit half of
 * IMEX(3,3,2); c = (0, 1, 1/2), A = ((0), (1), (1/4, 1/4)), b = (1/6, 1/6, 2/3))
 * at the interior points of `nfields` fields:
 *   stage 0: acc = k/6, Unext = Un + dt k;
 *   stage 1: acc += k/6, Unext = Un + dt (3/2) acc  (= Un + dt (k0 + k1)/4);
 *   stage 2: Unext = Un + dt (acc + 2/3 k).
 * Unext may alias Un only for stage 2. */
int mhd_ssprk3_stage(const mhd_patch_t* patch, int nfields, int stage, double dt, const double* Un,
                     const double* k, double* acc, double* Unext, void* stream);

/* Periodic ghost fill of `nfields` fields (edges and corners included). */
int mhd_fill_ghosts_periodic(const mhd_patch_t* patch, double* U, int nfields, void* stream);

/* ---- mesh-refinement glue (Sec. 4.2; Sec. 3.1 dense output) ----------------
 * Two patches of a 2:1 vertex-centred hierarchy: the coarse spacing is twice
 * the fine one on every axis, and fine padded index I coincides with coarse
 * padded index i when I = 2 i + offset (per axis; offset is a host int32[3],
 * any sign).  Boxes are host int32[3] half-open ranges [lo, hi) of padded
 * indices.  The arrays hold nfields fields in their patch's layout and must not
 * alias.
 * mhd_prolong: every fine point of the box takes the symmetric six-point
 *   Lagrange interpolation of the coarse data (coincident points are copies,
 *   half points (3, -25, 150, 150, -25, 3)/256 over the six nearest coarse
 *   nodes), as a tensor product applied along x, then y, then z; polynomials
 *   of degree <= 5 in each variable are reproduced.  Rejected (MHD_EINVAL)
 *   when a needed coarse node lies outside the padded coarse patch.
 * mhd_restrict: restriction by direct copy: every coarse point of the box
 *   takes the coincident fine value, Uc(i) = Uf(2 i + offset).
 * mhd_dense_output: at the interior points, from the right-hand sides L[j]
 *   (host array of 4 device pointers) of the four stages of an RK4 step of
 *   size dt that started from Un, with k_j = dt L_j: deriv = 0 gives
 *   U(t^n + theta dt) = Un + sum_j b_j(theta) k_j, deriv = 1..3 the deriv-th
 *   time derivative (1/dt^deriv) sum_j b_j^(deriv)(theta) k_j (Un unused, may
 *   be NULL), for the third-order interpolant b_1 = t - 3/2 t^2 + 2/3 t^3,
 *   b_2 = b_3 = t^2 - 2/3 t^3, b_4 = -1/2 t^2 + 2/3 t^3.  out may alias Un. */
int mhd_prolong(const mhd_patch_t* coarse, const double* Uc, const mhd_patch_t* fine, double* Uf, int nfields,
                const int32_t* offset, const int32_t* lo, const int32_t* hi, void* stream);
int mhd_restrict(const mhd_patch_t* fine, const double* Uf, const mhd_patch_t* coarse, double* Uc, int nfields,
                 const int32_t* offset, const int32_t* lo, const int32_t* hi, void* stream);
int mhd_dense_output(const mhd_patch_t* patch, int nfields, double theta, double dt, int deriv, const double* Un,
                     const double* const* L, double* out, void* stream);

/* ---- constraint monitors (Sec. 2.1 constraints; Sec. 5 accuracy checks) ----
 * At every interior point of the patch (ghost width >= 2, the 4th-order
 * centred stencils of Sec. 3.2 reach two points out), from the 32 evolved
 * fields U:
 *   C[0] = H   = R + K^2 - K_ij K^ij - 16 pi E          (energy constraint)
 *   C[1..3] = M_i = D_j K^j_i - d_i K - 8 pi S_i         (momentum constraint)
 *   C[4] = Z_i Z^i,  Z^i = chi (Ghat^i - Gt^i) / 2,  Gt^i = gt^ij gt^kl d_l gt_jk
 * with the physical metric gamma_ij = gt_ij / chi, K_ij = (At_ij + gt_ij K/3)/chi,
 * K = Khat + 2 Theta, E = (taubar + Dbar)/sqrt(gamma), S_i = Sbar_i/sqrt(gamma),
 * R the Ricci scalar of gamma_ij; every derivative is the 4th-order centred
 * operator on the evolved fields, products by the product rule.  C is a device
 * array of 5 fields in the patch layout (interior points written, the rest
 * untouched); it must not alias U.
 * sums: device array of 7 (nz + 1) doubles.  sums[7 + 7 k + q] is the volume
 * integral (sum times dx dy dz) over interior plane k of
 *   q = 0: H^2,  1: M_1^2 + M_2^2 + M_3^2,  2: Dbar (baryonic mass),
 *   3: Theta^2,  4: Z_i Z^i,  5: phi^2 = (phibar/sqrt(gamma))^2,
 *   6: gamma_ij B^i B^j with B^i = Bbar^i/sqrt(gamma),
 * and sums[q] the total over the planes (so sqrt(sums[0]) is the L2 norm of
 * H over the patch).  Reductions run in a fixed order: the same input gives
 * the same bits on every call.  Three kernels, enqueued on `stream`. */
int mhd_constraints(const mhd_patch_t* patch, const double* U, double* C, double* sums, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MHD_H */
