/*
 * Oracle (test infrastructure only): hybrid equation of state, Sec. 2.2.
 *   p = p_cold(rho) + (Gamma_th - 1) rho (eps - eps_cold(rho))
 *   p_cold = K_i rho^Gamma_i,  eps_cold = a_i + K_i/(Gamma_i-1) rho^(Gamma_i-1)
 *   for rho_{i-1} <= rho <= rho_i; a_0 = 0, K_i and a_i (i>0) by continuity.
 * The ideal gas p = (Gamma-1) rho eps is the one-piece case with K_0 = 0 and
 * Gamma_th = Gamma.
 */
#include <math.h>
#include "orc.h"

/* index of the piece containing rho: first i with rho < rho_i, else the last */
static int piece_of(const orc_eos* e, double rho) {
  int i;
  for (i = 0; i < e->npieces - 1; ++i)
    if (rho < e->rho_b[i]) return i;
  return e->npieces - 1;
}

void orc_eos_init_pwp(orc_eos* e, int npieces, double K0, const double* Gamma,
                      const double* rho_b, double Gamma_th) {
  int i;
  e->npieces = npieces;
  e->K[0] = K0;
  e->a[0] = 0.0;
  for (i = 0; i < npieces; ++i) e->Gamma[i] = Gamma[i];
  for (i = 0; i < npieces - 1; ++i) e->rho_b[i] = rho_b[i];
  for (i = 1; i < npieces; ++i) {
    double rb = e->rho_b[i - 1];
    /* continuity of p_cold at rho_{i-1} */
    e->K[i] = e->K[i - 1] * pow(rb, e->Gamma[i - 1]) / pow(rb, e->Gamma[i]);
    /* continuity of eps_cold at rho_{i-1} */
    e->a[i] = e->a[i - 1] + e->K[i - 1] / (e->Gamma[i - 1] - 1.0) * pow(rb, e->Gamma[i - 1] - 1.0)
              - e->K[i] / (e->Gamma[i] - 1.0) * pow(rb, e->Gamma[i] - 1.0);
  }
  e->Gamma_th = Gamma_th;
}

double orc_eps_cold(const orc_eos* e, double rho) {
  int i = piece_of(e, rho);
  return e->a[i] + e->K[i] / (e->Gamma[i] - 1.0) * pow(rho, e->Gamma[i] - 1.0);
}

static double p_cold(const orc_eos* e, double rho) {
  int i = piece_of(e, rho);
  return e->K[i] * pow(rho, e->Gamma[i]);
}

double orc_press(const orc_eos* e, double rho, double eps) {
  return p_cold(e, rho) + (e->Gamma_th - 1.0) * rho * (eps - orc_eps_cold(e, rho));
}

/* Sound speed squared for p(rho, eps):
 *   c_s^2 = (dp/drho + p/rho^2 dp/deps) / (1 + eps + p/rho)
 * which reduces to Gamma p / h for the ideal gas (App. B). */
double orc_cs2(const orc_eos* e, double rho, double eps) {
  int i = piece_of(e, rho);
  double gth = e->Gamma_th;
  double pc = e->K[i] * pow(rho, e->Gamma[i]);
  double ec = e->a[i] + e->K[i] / (e->Gamma[i] - 1.0) * pow(rho, e->Gamma[i] - 1.0);
  double p = pc + (gth - 1.0) * rho * (eps - ec);
  /* d eps_cold / d rho = K rho^(Gamma-2) = p_cold / rho^2 */
  double dpdrho = e->Gamma[i] * pc / rho + (gth - 1.0) * (eps - ec) - (gth - 1.0) * pc / rho;
  double dpdeps = (gth - 1.0) * rho;
  double cs2 = (dpdrho + p / (rho * rho) * dpdeps) / (1.0 + eps + p / rho);
  return cs2;
}
