/*
 * Plain FP64 CPU oracle for the MHDuet method-of-lines right-hand side.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library; it is
 * not a code path of the library.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load it.  It shares no source with the HIP
 * path (no common headers, helpers or constant generators).
 *
 * Everything is written pointwise, in plain loops, in double precision, in the
 * order of the equations of the paper (arXiv:2510.13965):
 *   Sec. 2.1  CCZ4 evolution equations, Ricci split, Laplacian of the lapse,
 *             matter projections, gauge (1+log, Gamma-freezing shift)
 *   Sec. 2.2  GRMHD balance laws with divergence cleaning, cons/prim
 *             definitions, hybrid piecewise-polytropic EoS
 *   Sec. 3.1  Runge-Kutta (Table I, explicit RK4)
 *   Sec. 3.2  4th-order centred, upwind and Kreiss-Oliger operators
 *   Sec. 3.3  Lax-Friedrichs flux splitting + MP5 reconstruction
 *   App. B    fast-magnetosonic speed bound
 *   App. D    conserved-to-primitive recovery (two Brent solves) and error policy
 *
 * Storage: structure of arrays, field-major, x fastest, contiguous:
 *   idx(i,j,k) = i + Nx*(j + Ny*k), Nx = nx+2ng, ...; field f at f*Nx*Ny*Nz.
 * Field order (evolved U): gt_xx,gt_xy,gt_xz,gt_yy,gt_yz,gt_zz (0-5),
 *   At_xx..At_zz (6-11), chi (12), Khat (13), Theta (14), Ghat^x,y,z (15-17),
 *   alpha (18), beta^x,y,z (19-21), Dbar (22), DYebar (23), taubar (24),
 *   Sbar_x,y,z (25-27), Bbar^x,y,z (28-30), phibar (31).
 * Primitive P: rho, eps, p, v^x, v^y, v^z, W, Ye (0-7).
 */
#ifndef ORC_H
#define ORC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" { /* the op-counting build compiles these sources as C++ */
#endif

/* Op-count hooks.  Empty in the oracle build; the op-counting build
 * (opcount.py, opcount.hpp) defines ORC_PHASE to attribute every counted
 * floating-point operation to the step of the path it belongs to. */
#ifndef ORC_PHASE
#define ORC_PHASE(id) ((void)0)
#endif
#define ORC_PH_OTHER 0
#define ORC_PH_CCZ4 1      /* CCZ4 point RHS incl. matter terms and KO */
#define ORC_PH_MHD_POINT 2 /* point fluxes and speeds */
#define ORC_PH_MHD_RECON 3 /* LF split + MP5 at one interface */
#define ORC_PH_MHD_UPD 4   /* conservative difference + geometric sources */
#define ORC_PH_C2P 5       /* con2prim incl. rewriting corrected points */
#define ORC_PH_RK 6        /* RK stage */
#define ORC_PH_P2C 7       /* prim -> cons */
#define ORC_PH_M1_POINT 8  /* M1 closure, point fluxes and speeds */
#define ORC_PH_M1_HOLO 9   /* M1 HO/LO flux at one interface */
#define ORC_PH_M1_UPD 10   /* M1 flux difference, geometric and collision sources */
#define ORC_PH_M1_RECL 11  /* closure re-evaluated for the sources (computed once per point above) */
#define ORC_NPHASE 12

#define ORC_NST 22
#define ORC_NMHD 10
#define ORC_NU 32
#define ORC_NP 8

/* con2prim flag bits */
#define ORC_F_ATMO 1u
#define ORC_F_EPS_LO 2u
#define ORC_F_EPS_HI 4u
#define ORC_F_VEL_LIMIT 8u
#define ORC_F_YE_RESET 16u
#define ORC_F_FALLBACK 32u
#define ORC_F_NOT_CONVERGED 64u
#define ORC_F_FATAL 128u

typedef struct {
  int n[3];      /* interior points per axis */
  int ng;        /* ghost width (3) */
  double dx[3];  /* spacing */
} orc_grid;

typedef struct {
  int npieces;          /* cold pieces, 1..4; a single piece with K=0 is the ideal gas */
  double K[4];          /* K_i */
  double Gamma[4];      /* Gamma_i */
  double rho_b[3];      /* piece boundaries rho_i */
  double a[4];          /* a_i */
  double Gamma_th;      /* thermal index */
  double rho_atm, rho_min, rho_max, eps_max, W_max, rho_low, alpha_bh, h0;
  double ye_min, ye_max, ye_atm;
} orc_eos;

typedef struct {
  double kappa_z, kappa_c, kappa_2, eta;
  double beta0[3];
  double sigma_ko, c_b, kappa_b, alpha_mp5, f_beta;
  int f_alpha_kind;     /* 0: f_alpha = 1 (1+log); 1: f_alpha = alpha/2 (harmonic) */
  int evolve_st;        /* CCZ4 block on/off */
  int evolve_mhd;       /* GRMHD block on/off */
  int couple_matter;    /* matter terms in the CCZ4 block on/off */
  int evolve_m1;        /* M1 radiation (fields 32..43, aux kappa_a, kappa_s, eta) on/off */
  int evolve_m1n;       /* with evolve_m1: neutrino number densities (fields 44..46, aux 9..14) on/off */
  double m_b;           /* reference baryon mass of the electron-fraction source */
  double les_cm;        /* C_M of the gradient SGS term of the induction equation (App. A); 0: off */
  int couple_exchange;  /* IMEX: the fluid's share of the collision exchange is stiff too (fluid slots of R,
                           and the implicit solve moves the exchanged energy, momentum and lepton number
                           out of the fluid); 0: it stays explicit */
} orc_par;

/* ---- EoS (Sec. 2.2, hybrid piecewise polytrope + thermal ideal gas) ---- */
void orc_eos_init_pwp(orc_eos* e, int npieces, double K0, const double* Gamma,
                      const double* rho_b, double Gamma_th);
double orc_eps_cold(const orc_eos* e, double rho);
double orc_press(const orc_eos* e, double rho, double eps);
double orc_cs2(const orc_eos* e, double rho, double eps);

/* ---- finite-difference operators of Sec. 3.2 at one point ---- */
double orc_d1(const double* u, int64_t p, int64_t s, double h);
double orc_d2(const double* u, int64_t p, int64_t s, double h);
double orc_d11(const double* u, int64_t p, int64_t s1, int64_t s2, double h1, double h2);
double orc_dup(const double* u, int64_t p, int64_t s, double h, double beta);
double orc_ko(const double* u, int64_t p, int64_t s, double h, double sigma);
double orc_mp5(const double* f5, double alpha);

/* ---- cons <-> prim (Sec. 2.2 definitions, App. D recovery) ---- */
/* eps_mode 0: P[eps] is the specific internal energy;
 *          1: P[eps] is the thermal part, eps_cold(rho) is added and written back. */
void orc_prim2con(const orc_grid* g, const orc_eos* e, double* U, double* P,
                  const double* EM, int eps_mode);
int64_t orc_con2prim(const orc_grid* g, const orc_eos* e, double* U, double* P,
                     uint8_t* flags, double* mu);
/* one-point recovery on undensitized conserved data, for pins */
unsigned orc_c2p_point(const orc_eos* e, const double cons[6], const double B[3],
                       const double gdn[6], const double gup[6], double alpha,
                       double prim[8], double mu[2], int* iters);
/* primitives and error-policy flags at a given mu[N] per padded point (no
 * root solve; U is only read) */
void orc_c2p_prims_at(const orc_grid* g, const orc_eos* e, const double* U, const double* mu,
                      double* P, uint8_t* flags);
/* f_a and f (steps 2 and 3 of the recovery) at a given mu[N] per padded point */
void orc_c2p_f_at(const orc_grid* g, const orc_eos* e, const double* U, const double* mu,
                  double* fa, double* f);

/* ---- learned con2prim starting guess (MLP 8 -> 64 -> 64 -> 2) ---- */
#define ORC_MLP_NPARAM 4866
#define ORC_MLP_NBLOCK 4882
float orc_bf16(float x);
void orc_mlp_features(const double cons[6], const double B[3], const double gdn[6],
                      const double gup[6], double x[8]);
void orc_mlp_baseline(double h0, const double cons[6], const double gup[6], double b[2]);
void orc_mlp_targets(double h0, const double b[2], const double mu[2], double t[2]);
/* features (and, if mu != NULL, targets) at every padded point; X is [N][8],
 * T is [N][2], binary32; points with D < rho_min get NaN rows */
void orc_c2p_features(const orc_grid* g, const orc_eos* e, const double* U, const double* mu,
                      float* X, float* T);
void orc_mlp_forward(const double* prm, const float* X, int64_t n, int emulate, double* Y);
double orc_mlp_grad(const double* prm, const float* X, const float* T, int64_t n, int emulate,
                    double* grad);
void orc_mlp_adam(double* prm, const double* grad, double* m, double* v, int step, double lr,
                  double beta1, double beta2, double eps);

/* ---- grey M1 radiation, three species (Sec. 2.3, 3.4, App. B) ---- */
double orc_m1_eddington(double xi);
double orc_m1_closure(double E, const double F[3], const double v[3], double W, const double gdn6[6],
                      const double gup6[6], double P6[6], double* J, double H[3], double* chi, int* iters);
void orc_m1_matter(const double* U, const double* P, int64_t N, int64_t p, double* E, double S[3],
                   double Sij[3][3]);
void orc_m1_rhs(const orc_grid* g, const orc_par* par, const double* U, const double* P, const double* aux,
                double* rhs, double* max_speed);
void orc_m1_rhs_split(const orc_grid* g, const orc_par* par, const double* U, const double* P,
                      const double* aux, double* rhs, double* stiff, double* max_speed);
/* gradient SGS (LES) term of the induction equation (App. A): rhs[28..30] +=
 * d_k (alpha G_B^{ki}) at interior points (called by orc_rhs when les_cm != 0) */
void orc_les_rhs(const orc_grid* g, const orc_par* par, const orc_eos* e, const double* U, const double* P,
                 double* rhs);
/* H_v^i and H_M^{xy,xz,yz} at every point two or more from the patch edge
 * (6 fields; for the pins) */
void orc_les_point_fields(const orc_grid* g, const orc_eos* e, const double* U, const double* P, double* out);
/* threads of the oracle's OpenMP loops (timing) */
void orc_set_threads(int n);
/* stiff fields of the split right-hand side for these parameters */
int orc_imex_stiff_fields(const orc_par* par);
int64_t orc_m1_implicit(const orc_grid* g, double* U, const double* P, const double* aux, double adt);
int64_t orc_m1_implicit_x(const orc_grid* g, double* U, const double* P, const double* aux, double adt,
                          int couple);
/* residual G and App. C Jacobian dG/dV (row-major 4x4) of the implicit M1
 * equation of one species at one point (undensitized; gd6 the physical metric) */
void orc_m1_implicit_point(const double gd6[6], const double v[3], double W, const double V[4], const double Vs[4],
                           double chi, double adt, double alp, double ka, double ks, double eta, double G[4],
                           double Jac[16]);
/* neutrino number densities (Sec. 2.3): rhs[44..46] written (their collision
 * sources to stiff[12..14] instead when stiff is non-NULL) and the
 * electron-fraction source added to rhs[23]; U has 47 fields, aux 15 */
void orc_m1n_rhs(const orc_grid* g, const orc_par* par, const double* U, const double* P, const double* aux,
                 double* rhs, double* stiff);
/* the analytic implicit number-density update of App. C, after E and F_i of
 * the stage are updated */
void orc_m1n_implicit(const orc_grid* g, double* U, const double* P, const double* aux, double adt);
void orc_m1n_implicit_x(const orc_grid* g, double* U, const double* P, const double* aux, double adt, int couple,
                        double m_b);
/* explicit part F (44 fields) and stiff radiation part R (12 fields) of L(U) */
void orc_rhs_split(const orc_grid* g, const orc_par* par, const orc_eos* e, const double* U, const double* P,
                   const double* aux, double* F, double* R, double* max_speed);
/* one IMEX(4,4,2) step of Table I (44 fields, 47 with the number densities, frozen
 * ghosts); returns the number
 * of implicit point solves that did not converge */
int64_t orc_imex_step(const orc_grid* g, const orc_par* par, const orc_eos* e, double* U, const double* aux,
                      double dt, int periodic);
/* the same for scheme 0 (IMEX(4,4,2)) or 1 (IMEX(3,3,2): SSP-RK(3,3) with the
 * re-derived L-stable I32L); orc_imex_tableau returns a scheme's tableaux
 * (4x4 row-major, stages in *stages) */
int64_t orc_imex_step_scheme(const orc_grid* g, const orc_par* par, const orc_eos* e, double* U, const double* aux,
                             double dt, int periodic, int scheme);
void orc_imex_tableau(int scheme, double AE[16], double AI[16], double BE[4], double BI[4], int* stages);
/* orc_rhs plus, if par->evolve_m1, the M1 part (U has 44 fields) */
void orc_rhs_full(const orc_grid* g, const orc_par* par, const orc_eos* e, const double* U, const double* P,
                  const double* aux, double* rhs, double* max_speed);

/* ---- right-hand side ---- */
void orc_rhs(const orc_grid* g, const orc_par* par, const orc_eos* e,
             const double* U, const double* P, double* rhs, double* max_speed);

/* ---- Runge-Kutta stage (Table I, explicit RK4, low-storage form) ---- */
void orc_rk4_stage(int stage, double dt, int64_t n, const double* Un,
                   const double* k, double* acc, double* Unext);
void orc_rk4_stage_interior(const orc_grid* g, int nfields, int stage, double dt,
                            const double* Un, const double* k, double* acc,
                            double* Unext);

/* SSP-RK(3,3) (Sec. 3.1): the printed tableau, and one stage combination in
 * Butcher form from the stored stage right-hand sides (K1, K2 may be NULL when
 * the stage does not read them) */
void orc_ssprk3_tableau(double A[9], double b[3]);
void orc_ssprk3_combine(const orc_grid* g, int nfields, int stage, double dt, const double* Un,
                        const double* K0, const double* K1, const double* K2, double* Unext);

/* ---- ghost fill ---- */
void orc_fill_periodic(const orc_grid* g, double* U, int nfields);

/* ---- mesh-refinement glue (amr.c): 2:1 vertex-centred prolongation by the
 * six-point Lagrange interpolation, restriction by copy, RK4 dense output ---- */
void orc_lagrange_half(double w[6]);
int orc_prolong(const orc_grid* gc, const double* Uc, const orc_grid* gf, double* Uf, int nfields,
                const int off[3], const int lo[3], const int hi[3]);
int orc_restrict(const orc_grid* gf, const double* Uf, const orc_grid* gc, double* Uc, int nfields,
                 const int off[3], const int lo[3], const int hi[3]);
void orc_dense_weights(double theta, int m, double b[4]);
void orc_dense_output(const orc_grid* g, int nfields, double theta, double dt, int m, const double* Un,
                      const double* L0, const double* L1, const double* L2, const double* L3, double* out);

/* ---- constraint monitors (diag.c): energy and momentum constraints, Z4
 * variables, baryonic mass, cleaning field ---- */
void orc_constraints_point(const double* U, int64_t N, int64_t p, const int64_t st[3], const double h[3],
                           double out[5], double* sqrtg, double gdn[3][3]);
void orc_constraints(const orc_grid* g, const double* U, double* C, double* sums);

#ifdef __cplusplus
}
#endif
#endif
