/*
 * Explicit Runge-Kutta step with the local entropy estimate (Sec. 2, the
 * Runge-Kutta example: stage equations, final update and the estimate
 * eta_new = eta(u_old) + dt sum_i b_i (eta' f)(y^i), valid for b_i >= 0),
 * the whole locally relaxed step (local relaxation theorem: one global
 * gamma = min_k gamma_k, u_gamma = u_old + gamma (u_new - u_old),
 * t_gamma = t_old + gamma dt), and the adaptive step of the embedded pairs
 * (Sec. 4: the schemes with an embedded method run with error-controlled
 * step sizes).
 *
 * Tableaux are written in Butcher form (c | A ; b^T ; bhat^T):
 *   SSPRK(3,3): c = (0, 1, 1/2), a21 = 1, a31 = a32 = 1/4, b = (1/6, 1/6, 2/3);
 *   RK(4,4):    c = (0, 1/2, 1/2, 1), a21 = a32 = 1/2, a43 = 1,
 *               b = (1/6, 1/3, 1/3, 1/6);
 *   BSRK(4,3):  the Bogacki-Shampine 3(2) pair (1989), four stages, the
 *               fourth evaluated at the third-order solution (b4 = 0);
 *   BSRK(8,5):  the Bogacki-Shampine 5(4) pair (1996), eight stages, the last
 *               at the fifth-order solution (b8 = 0); bhat is the fourth-order
 *               companion that uses all eight stages.
 * Each b has b_i >= 0 as the estimate requires.  The coefficients are those
 * of the published methods; the tests check them against the order
 * conditions.
 *
 * TEST INFRASTRUCTURE ONLY (see esrk_oracle.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "esrk_oracle.h"

#define MAXS 8

typedef struct {
  int s, p, q; /* stages, order, embedded order (0: none) */
  double A[MAXS][MAXS], b[MAXS], bh[MAXS], c[MAXS];
} tableau;

static void fill_c(tableau* T) {
  for (int i = 0; i < T->s; ++i) {
    double acc = 0.0;
    for (int j = 0; j < i; ++j) acc += T->A[i][j];
    T->c[i] = acc;
  }
}

static int get_tableau(int which, tableau* T) {
  memset(T, 0, sizeof(*T));
  if (which == ORC_SSPRK33) {
    T->s = 3;
    T->p = 3;
    T->A[1][0] = 1.0;
    T->A[2][0] = 0.25;
    T->A[2][1] = 0.25;
    T->b[0] = 1.0 / 6.0;
    T->b[1] = 1.0 / 6.0;
    T->b[2] = 2.0 / 3.0;
    fill_c(T);
    return ORC_OK;
  }
  if (which == ORC_RK44) {
    T->s = 4;
    T->p = 4;
    T->A[1][0] = 0.5;
    T->A[2][1] = 0.5;
    T->A[3][2] = 1.0;
    T->b[0] = 1.0 / 6.0;
    T->b[1] = 1.0 / 3.0;
    T->b[2] = 1.0 / 3.0;
    T->b[3] = 1.0 / 6.0;
    fill_c(T);
    return ORC_OK;
  }
  if (which == ORC_BSRK43) {
    T->s = 4;
    T->p = 3;
    T->q = 2;
    T->A[1][0] = 1.0 / 2.0;
    T->A[2][1] = 3.0 / 4.0;
    T->A[3][0] = 2.0 / 9.0;
    T->A[3][1] = 1.0 / 3.0;
    T->A[3][2] = 4.0 / 9.0;
    for (int j = 0; j < 3; ++j) T->b[j] = T->A[3][j];
    T->bh[0] = 7.0 / 24.0;
    T->bh[1] = 1.0 / 4.0;
    T->bh[2] = 1.0 / 3.0;
    T->bh[3] = 1.0 / 8.0;
    fill_c(T);
    return ORC_OK;
  }
  if (which == ORC_BSRK85) {
    T->s = 8;
    T->p = 5;
    T->q = 4;
    static const double A[8][7] = {
        {0, 0, 0, 0, 0, 0, 0},
        {1.0 / 6.0, 0, 0, 0, 0, 0, 0},
        {2.0 / 27.0, 4.0 / 27.0, 0, 0, 0, 0, 0},
        {183.0 / 1372.0, -162.0 / 343.0, 1053.0 / 1372.0, 0, 0, 0, 0},
        {68.0 / 297.0, -4.0 / 11.0, 42.0 / 143.0, 1960.0 / 3861.0, 0, 0, 0},
        {597.0 / 22528.0, 81.0 / 352.0, 63099.0 / 585728.0, 58653.0 / 366080.0,
         4617.0 / 20480.0, 0, 0},
        {174197.0 / 959244.0, -30942.0 / 79937.0, 8152137.0 / 19744439.0,
         666106.0 / 1039181.0, -29421.0 / 29068.0, 482048.0 / 414219.0, 0},
        {587.0 / 8064.0, 0.0, 4440339.0 / 15491840.0, 24353.0 / 124800.0, 387.0 / 44800.0,
         2152.0 / 5985.0, 7267.0 / 94080.0}};
    static const double bh[8] = {2479.0 / 34992.0,      0.0,
                                 123.0 / 416.0,         612941.0 / 3411720.0,
                                 43.0 / 1440.0,         2272.0 / 6561.0,
                                 79937.0 / 1113912.0,   3293.0 / 556956.0};
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < i; ++j) T->A[i][j] = A[i][j];
    for (int j = 0; j < 7; ++j) T->b[j] = A[7][j];
    for (int j = 0; j < 8; ++j) T->bh[j] = bh[j];
    fill_c(T);
    return ORC_OK;
  }
  return ORC_EINVAL;
}

int orc_tableau(int which, double* A, double* b, double* bhat, double* c, int* s, int* p,
                int* q) {
  tableau T;
  if (get_tableau(which, &T)) return ORC_EINVAL;
  for (int i = 0; i < MAXS; ++i) {
    for (int j = 0; j < MAXS; ++j) A[i * MAXS + j] = T.A[i][j];
    b[i] = T.b[i];
    bhat[i] = T.bh[i];
    c[i] = T.c[i];
  }
  *s = T.s;
  *p = T.p;
  *q = T.q;
  return ORC_OK;
}

int orc_tableau_stages(int which) {
  tableau T;
  return get_tableau(which, &T) ? -1 : T.s;
}

/* internal helpers (euler.c, relax.c) */
void orc__entropy_vars_ld(int dim, double gg, const double* q, long double* w);
int orc__geom_mass(const orc_mesh* g, double* M);

static int rk_step_impl(const orc_mesh* g, int which, const double* u_old, double dt,
                        double* du, double* deta, double* ystages, double* kstages,
                        double* estages, double* err, double* a_out) {
  tableau T;
  if (get_tableau(which, &T)) return ORC_EINVAL;
  if (err && T.q == 0) return ORC_EINVAL;
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
    /* phi_k(0) = sum_i M w(u_old).du - deta_k written without the cancelling
     * difference: dt sum_i b_i sum_nodes M (w(u_old) - w(y^i)).k_i, with
     * the entropy variables in extended precision (an identity of the
     * estimate's definition; the y^i are recomputed from the stored slopes) */
    if (a_out) {
      int nd = 1, nv = g->dim + 2;
      for (int m = 0; m < g->dim; ++m) nd *= g->deg + 1;
      double* M = (double*)malloc(sizeof(double) * nd);
      long double* acc = (long double*)calloc(ne, sizeof(long double));
      if (!M || !acc) {
        free(M);
        free(acc);
        free(K);
        free(E);
        free(y);
        return ORC_EINVAL;
      }
      orc__geom_mass(g, M);
      for (int i = 1; i < T.s; ++i) {
        if (T.b[i] == 0.0) continue;
        for (long q = 0; q < len; ++q) {
          double a = 0.0;
          for (int j = 0; j < i; ++j) a += T.A[i][j] * K[j * len + q];
          y[q] = u_old[q] + dt * a;
        }
        for (long k = 0; k < ne; ++k) {
          long double s = 0.0L;
          for (int n = 0; n < nd; ++n) {
            long gi = k * nd + n;
            double uo[5], yi[5];
            long double w0[5], w1[5];
            for (int v = 0; v < nv; ++v) {
              uo[v] = u_old[v * N + gi];
              yi[v] = y[v * N + gi];
            }
            orc__entropy_vars_ld(g->dim, g->gas_gamma, uo, w0);
            orc__entropy_vars_ld(g->dim, g->gas_gamma, yi, w1);
            for (int v = 0; v < nv; ++v)
              s += (long double)M[n] * (w0[v] - w1[v]) * K[i * len + v * N + gi];
          }
          acc[k] += (long double)T.b[i] * s;
        }
      }
      for (long k = 0; k < ne; ++k) a_out[k] = (double)((long double)dt * acc[k]);
      free(M);
      free(acc);
    }
    /* local error estimate u_new - uhat_new = dt sum_i (b_i - bhat_i) k_i */
    if (err)
      for (long q = 0; q < len; ++q) {
        double acc = 0.0;
        for (int i = 0; i < T.s; ++i) acc += (T.b[i] - T.bh[i]) * K[i * len + q];
        err[q] = dt * acc;
      }
    if (kstages) memcpy(kstages, K, sizeof(double) * T.s * len);
    if (estages) memcpy(estages, E, sizeof(double) * T.s * ne);
  }
  free(K);
  free(E);
  free(y);
  return rc;
}

int orc_rk_step(const orc_mesh* g, int which, const double* u_old, double dt,
                double* du, double* deta, double* ystages, double* kstages,
                double* estages) {
  return rk_step_impl(g, which, u_old, dt, du, deta, ystages, kstages, estages, NULL, NULL);
}

int orc_rk_step_a(const orc_mesh* g, int which, const double* u_old, double dt, double* du,
                  double* deta, double* a_out) {
  return rk_step_impl(g, which, u_old, dt, du, deta, NULL, NULL, NULL, NULL, a_out);
}

int orc_rk_step_err(const orc_mesh* g, int which, const double* u_old, double dt,
                    double* du, double* deta, double* err) {
  return rk_step_impl(g, which, u_old, dt, du, deta, NULL, NULL, NULL, err, NULL);
}

double orc_error_norm(const orc_mesh* g, const double* u_old, const double* du,
                      const double* err, double atol, double rtol) {
  long N = orc_num_nodes(g);
  long len = (long)(g->dim + 2) * N;
  long double acc = 0.0L;
  for (long q = 0; q < len; ++q) {
    double un = u_old[q] + du[q];
    double sc = atol + rtol * fmax(fabs(u_old[q]), fabs(un));
    double e = err[q] / sc;
    acc += (long double)e * e;
  }
  return sqrt((double)(acc / (long double)len));
}

double orc_adapt_factor(double err, int q, int accepted) {
  /* elementary controller: dt_new = dt * clip(safety * err^(-1/(q+1))) */
  double safety = accepted ? 0.9 : 0.45;
  double f = (err > 0.0) ? safety * pow(err, -1.0 / (q + 1)) : 10.0;
  if (!(err == err)) f = 0.1; /* no usable estimate: shrink */
  return fmin(10.0, fmax(0.1, f));
}

int orc_adaptive_step(const orc_mesh* g, int which, const orc_relax_opts* o, int mode,
                      double atol, double rtol, double cfl, double dt, double* u, double* t,
                      double* gamma, double* err_out, int* accepted, double* dt_next,
                      double* dt_used) {
  tableau T;
  if (get_tableau(which, &T) || T.q == 0 || mode < 0 || mode > 2) return ORC_EINVAL;
  long N = orc_num_nodes(g), ne = orc_num_elems(g);
  if (N < 0) return ORC_EINVAL;
  long len = (long)(g->dim + 2) * N;
  if (!(dt > 0.0)) dt = orc_cfl_dt(g, u, cfl);
  double* du = (double*)malloc(sizeof(double) * len);
  double* er = (double*)malloc(sizeof(double) * len);
  double* deta = (double*)malloc(sizeof(double) * ne);
  double* gk = (double*)malloc(sizeof(double) * ne);
  double* a = (double*)malloc(sizeof(double) * ne);
  int rc = (du && er && deta && gk && a) ? ORC_OK : ORC_EINVAL;
  if (rc == ORC_OK) rc = rk_step_impl(g, which, u, dt, du, deta, NULL, NULL, NULL, er, a);
  double en = 0.0, gam = 1.0;
  int acc = 0;
  if (rc == ORC_OK) {
    en = orc_error_norm(g, u, du, er, atol, rtol);
    acc = en <= 1.0;
    if (acc && mode == 0)
      rc = orc_local_relaxation_solve_a(g, o, u, du, deta, a, gk, &gam, NULL, NULL, NULL, NULL,
                                        NULL);
    else if (acc && mode == 1)
      rc = orc_global_relaxation_solve_a(g, o, u, du, deta, a, &gam, NULL, NULL, NULL, NULL);
  }
  if (rc == ORC_OK && acc) {
    for (long q = 0; q < len; ++q) u[q] = u[q] + gam * du[q];
    *t = *t + gam * dt;
  }
  if (rc == ORC_OK) {
    if (gamma) *gamma = gam;
    if (err_out) *err_out = en;
    if (accepted) *accepted = acc;
    if (dt_next) *dt_next = dt * orc_adapt_factor(en, T.q, acc);
  }
  if (dt_used) *dt_used = dt;
  free(du);
  free(er);
  free(deta);
  free(gk);
  free(a);
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
  double* a = (double*)malloc(sizeof(double) * ne);
  if (!du || !deta || !gk || !a) {
    free(du);
    free(deta);
    free(gk);
    free(a);
    return ORC_EINVAL;
  }
  double gam = 1.0;
  int rc = orc_rk_step_a(g, which, u, dt, du, deta, a);
  if (rc == ORC_OK)
    rc = orc_local_relaxation_solve_a(g, o, u, du, deta, a, gk, &gam, NULL, NULL, NULL, NULL,
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
  free(a);
  return rc;
}
