/*
 * Local relaxation (Sec. 2: the local relaxation equation, its existence
 * lemma and the theorem that gamma = min_k gamma_k keeps every local entropy
 * inequality).
 *
 * For a Runge-Kutta method the old values are those of the previous step
 * (m = 1), so eta_k^old = eta_k(u_old) and only the increments
 * du = u_new - u_old and deta_k = eta_k^new - eta_k^old enter:
 *   r_k(gamma)   = eta_k(u_old + gamma du) - eta_k(u_old) - gamma deta_k,
 *   phi_k(gamma) = r_k(gamma) / gamma.
 * r_k is convex with r_k(0) = 0, so phi_k is nondecreasing and
 * phi_k(0) = r_k'(0) = sum_i M_i w(u_old,i).du_i - deta_k.  gamma_k is the
 * positive root of phi_k.
 *
 * Readings where the paper is silent (root solver, tolerance, degenerate
 * elements):
 *  - entropy differences per node are taken from ratios (log1p of dp/p and
 *    drho/rho) in extended precision, so r_k carries no cancellation of the
 *    large absolute entropy values;
 *  - an element whose curvature r_k(1) - phi_k(0) is below 64 eps times its
 *    round-off scale (sum_i M_i sum_v |w_v du_v| + |deta_k|) has no
 *    determinable root; it is inactive and gets gamma_k = +INF;
 *  - an active element with phi_k(0) >= 0 has no positive root (ENOROOT);
 *  - the root is bracketed from [0, 1], doubling the upper end up to
 *    gamma_max (an admissibility failure counts as phi = +INF), then bisected
 *    to width tol*max(1, gamma); the lower end (where phi <= 0) is returned.
 *    If phi(gamma_max) <= 0 the element returns gamma_max.  Any value in
 *    (0, gamma_k] keeps the element's inequality (theorem), so the lower end
 *    is the safe side.
 *  - gamma = min_k gamma_k, and gamma = 1 when every element is inactive.
 *
 * TEST INFRASTRUCTURE ONLY (see esrk_oracle.h).
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>

#include "esrk_oracle.h"

int orc__geom_mass(const orc_mesh* g, double* M);

/* S(u + d) - S(u) at one node, extended precision.  *ok = 0 if u + d has
 * rho <= 0 or p <= 0. */
static long double entropy_change(int dim, double gg, const double* u, const double* d,
                                  long double scale, int* ok) {
  long double G = gg;
  long double rho = u[0], E = u[dim + 1];
  long double drho = scale * (long double)d[0], dE = scale * (long double)d[dim + 1];
  long double m2 = 0.0L, mdm = 0.0L, dm2 = 0.0L;
  for (int k = 0; k < dim; ++k) {
    long double m = u[1 + k], dm = scale * (long double)d[1 + k];
    m2 += m * m;
    mdm += m * dm;
    dm2 += dm * dm;
  }
  long double rho1 = rho + drho;
  long double p = (G - 1.0L) * (E - 0.5L * m2 / rho);
  /* |m'|^2/rho' - |m|^2/rho = (rho (2 m.dm + |dm|^2) - drho |m|^2) / (rho rho') */
  long double dke = (rho * (2.0L * mdm + dm2) - drho * m2) / (rho * rho1);
  long double dp = (G - 1.0L) * (dE - 0.5L * dke);
  long double p1 = p + dp;
  if (!(rho1 > 0.0L) || !(p1 > 0.0L)) {
    *ok = 0;
    return 0.0L;
  }
  long double s0 = logl(p) - G * logl(rho);
  long double ds = log1pl(dp / p) - G * log1pl(drho / rho);
  /* S = -rho s / (G-1):  rho' s' - rho s = drho s0 + rho' ds */
  return -(drho * s0 + rho1 * ds) / (G - 1.0L);
}

typedef struct {
  const orc_mesh* g;
  long k, N;
  int nd, nv;
  const double* u;
  const double* du;
  double deta;
  const double* M;
  long double shift; /* phi(0) given - (A - deta): 0 unless phi(0) is supplied */
} elem_ctx;

static long double r_of_gamma(const elem_ctx* c, double gamma, int* ok) {
  long double sum = 0.0L;
  *ok = 1;
  for (int i = 0; i < c->nd; ++i) {
    long gi = c->k * c->nd + i;
    double ui[5], di[5];
    for (int v = 0; v < c->nv; ++v) {
      ui[v] = c->u[v * c->N + gi];
      di[v] = c->du[v * c->N + gi];
    }
    int okn = 1;
    long double dS = entropy_change(c->g->dim, c->g->gas_gamma, ui, di, gamma, &okn);
    if (!okn) {
      *ok = 0;
      return INFINITY;
    }
    sum += (long double)c->M[i] * dS;
  }
  return sum - (long double)gamma * (long double)c->deta;
}

static long double phi_elem(double gamma, void* vctx, int* ok) {
  const elem_ctx* c = (const elem_ctx*)vctx;
  long double r = r_of_gamma(c, gamma, ok);
  if (!*ok) return INFINITY;
  return r / (long double)gamma + c->shift;
}

void orc__entropy_vars_ld(int dim, double gg, const double* q, long double* w);

int orc_root_nondecreasing(orc_phi_fn phi, void* ctx, double phi0,
                           const orc_relax_opts* o, double* root, int* iters) {
  int it = 0, ok = 1;
  if (!(phi0 < 0.0)) return ORC_ENOROOT;
  double lo = 0.0, hi = 1.0;
  long double fhi = phi(hi, ctx, &ok);
  ++it;
  if (!ok) fhi = INFINITY;
  while (fhi <= 0.0L) {
    if (hi >= o->gamma_max) {
      *root = o->gamma_max;
      if (iters) *iters = it;
      return ORC_OK;
    }
    lo = hi;
    hi = fmin(2.0 * hi, o->gamma_max);
    fhi = phi(hi, ctx, &ok);
    ++it;
    if (!ok) fhi = INFINITY;
  }
  while (hi - lo > o->tol * fmax(1.0, hi) && it < o->maxit) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    long double fm = phi(mid, ctx, &ok);
    ++it;
    if (!ok) fm = INFINITY;
    if (fm <= 0.0L)
      lo = mid;
    else
      hi = mid;
  }
  *root = lo;
  if (iters) *iters = it;
  return ORC_OK;
}

long double orc_relax_r(const orc_mesh* g, long k, const double* u_old, const double* du,
                        double deta_k, double gamma, int* admissible) {
  double M[4096];
  orc__geom_mass(g, M);
  elem_ctx c;
  c.g = g;
  c.k = k;
  c.N = orc_num_nodes(g);
  c.nv = g->dim + 2;
  c.nd = 1;
  for (int m = 0; m < g->dim; ++m) c.nd *= g->deg + 1;
  c.u = u_old;
  c.du = du;
  c.deta = deta_k;
  c.M = M;
  c.shift = 0.0L;
  int ok = 1;
  long double r = r_of_gamma(&c, gamma, &ok);
  if (admissible) *admissible = ok;
  return r;
}

int orc_local_relaxation_solve(const orc_mesh* g, const orc_relax_opts* o,
                               const double* u_old, const double* du,
                               const double* deta, double* gamma_k, double* gamma,
                               double* phi0_out, double* curv_out, double* noise_out,
                               int* iters_out, long* bad_elem) {
  return orc_local_relaxation_solve_a(g, o, u_old, du, deta, NULL, gamma_k, gamma, phi0_out,
                                      curv_out, noise_out, iters_out, bad_elem);
}

int orc_local_relaxation_solve_a(const orc_mesh* g, const orc_relax_opts* o,
                                 const double* u_old, const double* du, const double* deta,
                                 const double* a_in, double* gamma_k, double* gamma,
                                 double* phi0_out, double* curv_out, double* noise_out,
                                 int* iters_out, long* bad_elem) {
  long N = orc_num_nodes(g), ne = orc_num_elems(g);
  if (N < 0) return ORC_EINVAL;
  int nd = 1, nv = g->dim + 2;
  for (int m = 0; m < g->dim; ++m) nd *= g->deg + 1;
  if (nd > 4096) return ORC_EINVAL;
  double M[4096];
  orc__geom_mass(g, M);
  double gmin = INFINITY;
  int rc = ORC_OK;
  if (bad_elem) *bad_elem = -1;
  for (long k = 0; k < ne; ++k) {
    /* phi(0) = sum_i M_i w(u_old,i).du_i - deta_k, and its round-off scale */
    long double A = 0.0L, scale = 0.0L;
    for (int i = 0; i < nd; ++i) {
      long gi = k * nd + i;
      double ui[5];
      long double wi[5];
      for (int v = 0; v < nv; ++v) ui[v] = u_old[v * N + gi];
      orc__entropy_vars_ld(g->dim, g->gas_gamma, ui, wi);
      for (int v = 0; v < nv; ++v) {
        long double t = (long double)M[i] * wi[v] * du[v * N + gi];
        A += t;
        scale += fabsl(t);
      }
    }
    scale += fabsl((long double)deta[k]);
    /* phi(0) = A - deta, or the supplied value of the same quantity */
    long double naive = A - (long double)deta[k];
    long double a = a_in ? (long double)a_in[k] : naive;
    double phi0 = (double)a;
    elem_ctx c = {g, k, N, nd, nv, u_old, du, deta[k], M, a - naive};
    int ok = 1;
    long double r1 = r_of_gamma(&c, 1.0, &ok);
    /* curvature r(1) - phi(0) = B(1), the relative entropy of u_old + du */
    double curv = ok ? (double)(r1 - naive) : INFINITY;
    double noise = (double)(64.0L * DBL_EPSILON * scale);
    if (phi0_out) phi0_out[k] = phi0;
    if (curv_out) curv_out[k] = curv;
    if (noise_out) noise_out[k] = noise;
    double gk;
    int its = 0;
    if (curv <= noise) {
      gk = INFINITY; /* inactive: no determinable root */
    } else if (phi0 > noise) {
      gk = 0.0;
      if (rc == ORC_OK) {
        rc = ORC_ENOROOT;
        if (bad_elem) *bad_elem = k;
      }
    } else if (phi0 > -0.5 * curv) {
      /* degenerate: phi(0) ~ 0 while the relative entropy is not, so the
       * root lies below about 1/2 (the existence lemma needs the element's
       * own slope at u_old to carry the curvature; an element that a wave
       * reaches only in the last stages of the step has none) */
      gk = INFINITY;
    } else {
      orc_root_nondecreasing(phi_elem, &c, phi0, o, &gk, &its);
    }
    gamma_k[k] = gk;
    if (iters_out) iters_out[k] = its;
    if (gk < gmin) gmin = gk;
  }
  if (gamma) *gamma = isinf(gmin) ? 1.0 : gmin;
  return rc;
}

/* ---- global relaxation (the relaxation idea applied to the single global
 * functional eta = sum_k eta_k, Sec. 1; remark after the local theorem) ----
 * r(gamma) = sum_k r_k(gamma) = eta(u_old + gamma du) - eta(u_old) - gamma sum_k deta_k,
 * phi = r / gamma; gamma is its positive root (entropy equality). */
typedef struct {
  const orc_mesh* g;
  long N, ne;
  int nd, nv;
  const double* u;
  const double* du;
  const double* deta;
  const double* M;
  long double shift; /* phi(0) given - (A - D): 0 unless phi(0) is supplied */
} glob_ctx;

static long double r_global(const glob_ctx* c, double gamma, int* ok) {
  long double sum = 0.0L;
  *ok = 1;
  for (long k = 0; k < c->ne; ++k) {
    elem_ctx e = {c->g, k, c->N, c->nd, c->nv, c->u, c->du, c->deta[k], c->M, 0.0L};
    int okk = 1;
    long double r = r_of_gamma(&e, gamma, &okk);
    if (!okk) {
      *ok = 0;
      return INFINITY;
    }
    sum += r;
  }
  return sum;
}

static long double phi_global(double gamma, void* vctx, int* ok) {
  const glob_ctx* c = (const glob_ctx*)vctx;
  long double r = r_global(c, gamma, ok);
  if (!*ok) return INFINITY;
  return r / (long double)gamma + c->shift;
}

int orc_global_relaxation_solve(const orc_mesh* g, const orc_relax_opts* o,
                                const double* u_old, const double* du, const double* deta,
                                double* gamma, double* phi0_out, double* curv_out,
                                double* noise_out, int* iters_out) {
  return orc_global_relaxation_solve_a(g, o, u_old, du, deta, NULL, gamma, phi0_out, curv_out,
                                       noise_out, iters_out);
}

int orc_global_relaxation_solve_a(const orc_mesh* g, const orc_relax_opts* o,
                                  const double* u_old, const double* du, const double* deta,
                                  const double* a_in, double* gamma, double* phi0_out,
                                  double* curv_out, double* noise_out, int* iters_out) {
  long N = orc_num_nodes(g), ne = orc_num_elems(g);
  if (N < 0 || !gamma) return ORC_EINVAL;
  int nd = 1, nv = g->dim + 2;
  for (int m = 0; m < g->dim; ++m) nd *= g->deg + 1;
  if (nd > 4096) return ORC_EINVAL;
  double M[4096];
  orc__geom_mass(g, M);
  /* phi(0) = sum_i M_i w(u_old,i).du_i - sum_k deta_k and its round-off scale */
  long double A = 0.0L, scale = 0.0L, D = 0.0L, asum = 0.0L;
  for (long k = 0; k < ne; ++k) {
    for (int i = 0; i < nd; ++i) {
      long gi = k * nd + i;
      double ui[5];
      long double wi[5];
      for (int v = 0; v < nv; ++v) ui[v] = u_old[v * N + gi];
      orc__entropy_vars_ld(g->dim, g->gas_gamma, ui, wi);
      for (int v = 0; v < nv; ++v) {
        long double t = (long double)M[i] * wi[v] * du[v * N + gi];
        A += t;
        scale += fabsl(t);
      }
    }
    D += deta[k];
    scale += fabsl((long double)deta[k]);
    if (a_in) asum += a_in[k];
  }
  /* phi(0) = A - D, or the sum of the supplied per-element values */
  long double naive = A - D;
  long double a = a_in ? asum : naive;
  glob_ctx c = {g, N, ne, nd, nv, u_old, du, deta, M, a - naive};
  int ok = 1;
  double phi0 = (double)a;
  long double r1 = r_global(&c, 1.0, &ok);
  double curv = ok ? (double)(r1 - naive) : INFINITY;
  double noise = (double)(64.0L * DBL_EPSILON * scale);
  if (phi0_out) *phi0_out = phi0;
  if (curv_out) *curv_out = curv;
  if (noise_out) *noise_out = noise;
  int its = 0;
  if (curv <= noise) {
    *gamma = 1.0; /* no curvature above round-off: nothing to relax */
  } else if (!(phi0 < 0.0)) {
    *gamma = 0.0;
    if (iters_out) *iters_out = 0;
    return ORC_ENOROOT;
  } else {
    orc_root_nondecreasing(phi_global, &c, phi0, o, gamma, &its);
  }
  if (iters_out) *iters_out = its;
  return ORC_OK;
}

/* r(gamma) summed over all elements (for tests). */
long double orc_global_relax_r(const orc_mesh* g, const double* u_old, const double* du,
                               const double* deta, double gamma, int* admissible) {
  double M[4096];
  orc__geom_mass(g, M);
  glob_ctx c;
  c.g = g;
  c.N = orc_num_nodes(g);
  c.ne = orc_num_elems(g);
  c.nv = g->dim + 2;
  c.nd = 1;
  for (int m = 0; m < g->dim; ++m) c.nd *= g->deg + 1;
  c.u = u_old;
  c.du = du;
  c.deta = deta;
  c.M = M;
  c.shift = 0.0L;
  int ok = 1;
  long double r = r_global(&c, gamma, &ok);
  if (admissible) *admissible = ok;
  return r;
}
