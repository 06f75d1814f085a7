/*
 * Explicit Runge-Kutta step with the local entropy estimate (Sec. 2, the
 * Runge-Kutta example: stage equations, final update and the estimate
 * eta_new = eta(u_old) + dt sum_i b_i (eta' f)(y^i), valid for b_i >= 0),
 * and the whole locally relaxed step (local relaxation theorem: one global
 * gamma = min_k gamma_k, u_gamma = u_old + gamma (u_new - u_old),
 * t_gamma = t_old + gamma dt).
 *
 * Tableaux are written in Butcher form (c | A ; b^T):
 *   SSPRK(3,3): c = (0, 1, 1/2), a21 = 1, a31 = a32 = 1/4, b = (1/6, 1/6, 2/3);
 *   RK(4,4):    c = (0, 1/2, 1/2, 1), a21 = a32 = 1/2, a43 = 1,
 *               b = (1/6, 1/3, 1/3, 1/6).
 * Both have b_i >= 0 as the estimate requires.
 *
 * TEST INFRASTRUCTURE ONLY (see esrk_oracle.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "esrk_oracle.h"

typedef struct {
  int s;
  double A[4][4], b[4], c[4];
} tableau;

static int get_tableau(int which, tableau* T) {
  memset(T, 0, sizeof(*T));
  if (which == ORC_SSPRK33) {
    T->s = 3;
    T->A[1][0] = 1.0;
    T->A[2][0] = 0.25;
    T->A[2][1] = 0.25;
    T->b[0] = 1.0 / 6.0;
    T->b[1] = 1.0 / 6.0;
    T->b[2] = 2.0 / 3.0;
    T->c[1] = 1.0;
    T->c[2] = 0.5;
    return ORC_OK;
  }
  if (which == ORC_RK44) {
    T->s = 4;
    T->A[1][0] = 0.5;
    T->A[2][1] = 0.5;
    T->A[3][2] = 1.0;
    T->b[0] = 1.0 / 6.0;
    T->b[1] = 1.0 / 3.0;
    T->b[2] = 1.0 / 3.0;
    T->b[3] = 1.0 / 6.0;
    T->c[1] = 0.5;
    T->c[2] = 0.5;
    T->c[3] = 1.0;
    return ORC_OK;
  }
  return ORC_EINVAL;
}

int orc_tableau_stages(int which) {
  tableau T;
  return get_tableau(which, &T) ? -1 : T.s;
}

int orc_rk_step(const orc_mesh* g, int which, const double* u_old, double dt,
                double* du, double* deta, double* ystages, double* kstages,
                double* estages) {
  tableau T;
  if (get_tableau(which, &T)) return ORC_EINVAL;
  long N = orc_num_nodes(g), ne = orc_num_elems(g);
  if (N < 0) return ORC_EINVAL;
  long len = (long)(g->dim + 2) * N;
  double* K = (double*)malloc(sizeof(double) * T.s * len);
  double* E = (double*)malloc(sizeof(double) * T.s * ne);
  double* y = (double*)malloc(sizeof(double) * len);
  if (!K || !E || !y) {
    free(K);
    free(E);
    free(y);
    return ORC_EINVAL;
  }
  int rc = ORC_OK;
  for (int i = 0; i < T.s && rc == ORC_OK; ++i) {
    for (long q = 0; q < len; ++q) {
      double acc = 0.0;
      for (int j = 0; j < i; ++j) acc += T.A[i][j] * K[j * len + q];
      y[q] = u_old[q] + dt * acc;
    }
    if (ystages) memcpy(ystages + i * len, y, sizeof(double) * len);
    rc = orc_rhs(g, y, K + i * len, E + i * ne, NULL);
  }
  if (rc == ORC_OK) {
    for (long q = 0; q < len; ++q) {
      double acc = 0.0;
      for (int i = 0; i < T.s; ++i) acc += T.b[i] * K[i * len + q];
      du[q] = dt * acc;
    }
    for (long k = 0; k < ne; ++k) {
      double acc = 0.0;
      for (int i = 0; i < T.s; ++i) acc += T.b[i] * E[i * ne + k];
      deta[k] = dt * acc;
    }
    if (kstages) memcpy(kstages, K, sizeof(double) * T.s * len);
    if (estages) memcpy(estages, E, sizeof(double) * T.s * ne);
  }
  free(K);
  free(E);
  free(y);
  return rc;
}

int orc_step(const orc_mesh* g, int which, const orc_relax_opts* o, double cfl,
             double dt, double* u, double* t, double* gamma, double* gamma_k,
             double* dt_used, long* bad_elem) {
  long N = orc_num_nodes(g), ne = orc_num_elems(g);
  if (N < 0) return ORC_EINVAL;
  long len = (long)(g->dim + 2) * N;
  if (!(dt > 0.0)) dt = orc_cfl_dt(g, u, cfl);
  double* du = (double*)malloc(sizeof(double) * len);
  double* deta = (double*)malloc(sizeof(double) * ne);
  double* gk = (double*)malloc(sizeof(double) * ne);
  if (!du || !deta || !gk) {
    free(du);
    free(deta);
    free(gk);
    return ORC_EINVAL;
  }
  double gam = 1.0;
  int rc = orc_rk_step(g, which, u, dt, du, deta, NULL, NULL, NULL);
  if (rc == ORC_OK)
    rc = orc_local_relaxation_solve(g, o, u, du, deta, gk, &gam, NULL, NULL, NULL, NULL,
                                    bad_elem);
  if (rc == ORC_OK) {
    for (long q = 0; q < len; ++q) u[q] = u[q] + gam * du[q];
    *t = *t + gam * dt;
    if (gamma) *gamma = gam;
    if (gamma_k) memcpy(gamma_k, gk, sizeof(double) * ne);
  }
  if (dt_used) *dt_used = dt;
  free(du);
  free(deta);
  free(gk);
  return rc;
}
