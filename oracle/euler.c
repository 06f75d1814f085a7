/*
 * Pointwise thermodynamics, entropy, entropy variables and fluxes of the
 * compressible Euler equations (Sec. 3.1: conserved variables, the closure
 * p = rho R T, the entropy function S = -rho s and w^T = dS/dq).
 *
 * Readings where the paper is silent:
 *  - s = ln p - gamma ln rho and S = -rho s / (gamma - 1).  The relaxation root
 *    is unchanged by any positive scaling and affine shift of S.
 *  - the entropy-conservative two-point flux is Chandrashekar's: it satisfies
 *    Tadmor's condition (w_R - w_L).f# = psi_R - psi_L with psi_m = rho v_m
 *    (checked by the tests).  beta = rho / (2 p).
 *  - the logarithmic mean (a - b)/(ln a - ln b) is evaluated as written for
 *    well separated arguments and as (a - b) / (2 atanh(f)), f = (a-b)/(a+b),
 *    otherwise: the same quantity, accurate as a -> b.
 *
 * TEST INFRASTRUCTURE ONLY (see esrk_oracle.h).
 */
#include <math.h>

#include "esrk_oracle.h"

double orc_logmean(double a, double b) {
  double f = (a - b) / (a + b);
  if (f == 0.0) return a;
  /* well separated: ln a - ln b carries no cancellation; close: the atanh form */
  if (fabs(f) > 0.5) return (a - b) / (log(a) - log(b));
  return (a - b) / (2.0 * atanh(f));
}

static void primitives(int dim, double gg, const double* u, double* rho, double* v,
                       double* p) {
  double ke = 0.0;
  *rho = u[0];
  for (int k = 0; k < dim; ++k) {
    v[k] = u[1 + k] / u[0];
    ke += v[k] * u[1 + k];
  }
  *p = (gg - 1.0) * (u[dim + 1] - 0.5 * ke);
}

double orc_entropy(int dim, double gg, const double* u) {
  double rho, v[3], p;
  primitives(dim, gg, u, &rho, v, &p);
  double s = log(p) - gg * log(rho);
  return -rho * s / (gg - 1.0);
}

void orc_entropy_vars(int dim, double gg, const double* u, double* w) {
  double rho, v[3], p, v2 = 0.0;
  primitives(dim, gg, u, &rho, v, &p);
  for (int k = 0; k < dim; ++k) v2 += v[k] * v[k];
  double s = log(p) - gg * log(rho);
  w[0] = (gg - s) / (gg - 1.0) - rho * v2 / (2.0 * p);
  for (int k = 0; k < dim; ++k) w[1 + k] = rho * v[k] / p;
  w[dim + 1] = -rho / p;
}

void orc_phys_flux(int dim, double gg, int m, const double* u, double* f) {
  double rho, v[3], p;
  primitives(dim, gg, u, &rho, v, &p);
  f[0] = rho * v[m];
  for (int k = 0; k < dim; ++k) f[1 + k] = rho * v[k] * v[m] + (k == m ? p : 0.0);
  f[dim + 1] = (u[dim + 1] + p) * v[m];
}

void orc_ec_flux(int dim, double gg, int m, const double* uL, const double* uR,
                 double* f) {
  double rL, vL[3], pL, rR, vR[3], pR;
  primitives(dim, gg, uL, &rL, vL, &pL);
  primitives(dim, gg, uR, &rR, vR, &pR);
  double bL = rL / (2.0 * pL), bR = rR / (2.0 * pR);
  double rho_ln = orc_logmean(rL, rR);
  double beta_ln = orc_logmean(bL, bR);
  double rho_avg = 0.5 * (rL + rR), beta_avg = 0.5 * (bL + bR);
  double v2_avg = 0.0, vavg[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < dim; ++k) {
    vavg[k] = 0.5 * (vL[k] + vR[k]);
    v2_avg += 0.5 * (vL[k] * vL[k] + vR[k] * vR[k]);
  }
  double p_hat = rho_avg / (2.0 * beta_avg);
  f[0] = rho_ln * vavg[m];
  double fe = f[0] * (1.0 / (2.0 * (gg - 1.0) * beta_ln) - 0.5 * v2_avg);
  for (int k = 0; k < dim; ++k) {
    f[1 + k] = f[0] * vavg[k] + (k == m ? p_hat : 0.0);
    fe += vavg[k] * f[1 + k];
  }
  f[dim + 1] = fe;
}

double orc_wave_speed(int dim, double gg, const double* u) {
  double rho, v[3], p;
  primitives(dim, gg, u, &rho, v, &p);
  double c = sqrt(gg * p / rho), s = 0.0;
  for (int k = 0; k < dim; ++k) s += fabs(v[k]) + c;
  return s;
}

/* w = dS/du as above, in extended precision from a double state (internal). */
void orc__entropy_vars_ld(int dim, double gg, const double* q, long double* w) {
  long double G = gg, rho = q[0], E = q[dim + 1], m2 = 0.0L;
  for (int d = 0; d < dim; ++d) m2 += (long double)q[1 + d] * q[1 + d];
  long double p = (G - 1.0L) * (E - 0.5L * m2 / rho);
  long double s = logl(p) - G * logl(rho);
  w[0] = (G - s) / (G - 1.0L) - 0.5L * m2 / (rho * p);
  for (int d = 0; d < dim; ++d) w[1 + d] = (long double)q[1 + d] / p;
  w[dim + 1] = -rho / p;
}
