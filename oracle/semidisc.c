/*
 * Entropy-stable semidiscretization on a periodic Cartesian mesh (or a 1-D
 * mesh with Dirichlet exterior states at both ends, entering through the
 * same interface flux) of
 * tensor-product Lobatto elements (Sec. 3.1, the element equation: the
 * flux-differencing volume term 2 D o F(q,q) 1, interface SATs with added
 * interface dissipation, and the BR1-type viscous terms).
 *
 * Plain loops, no symmetry exploitation, no blocking: every node pair is
 * evaluated where the formula names it.
 *
 * Readings where the paper defers to cited work:
 *  - volume term, per node i of element k, with metric 2/h_m of the affine map:
 *      V_i = sum_m (2/h_m) sum_j 2 D[i_m][j] f#_m(u_i, u_{i with i_m <- j});
 *  - interface flux: f* = f#_m(u_L, u_R) - (lambda_scale/2) lambda (u_R - u_L),
 *    lambda = max(|v_m| + c) over both sides (local Lax-Friedrichs);
 *    SAT: node with i_m = p gets (2/h_m)(1/w_p)(f* - f_m(u_L)),
 *         node with i_m = 0 gets -(2/h_m)(1/w_0)(f* - f_m(u_R));
 *    dudt = -(V + SAT) + Visc;
 *  - viscous terms (Navier-Stokes) in BR1 form with central interface values:
 *      theta_m = (2/h_m) [D w + lift(0.5 (w_nbr - w))]  (gradient of w),
 *      g_m = viscous flux from the chain rule (constant mu, Stokes hypothesis,
 *            heat conductivity mu c_p / Pr),
 *      Visc = sum_m (2/h_m) [D g_m + lift(0.5 (g_m,nbr - g_m))],
 *    where lift puts (1/w_p) x on the i_m = p face and -(1/w_0) x on i_m = 0.
 *
 * TEST INFRASTRUCTURE ONLY (see esrk_oracle.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "esrk_oracle.h"

typedef struct {
  int dim, n, nv, nd, bc;
  long ne, N;
  int nel[3];
  double h[3];
  double x[16], w[16], D[256];
} geom;

static int setup(const orc_mesh* g, geom* G) {
  if (g->dim < 1 || g->dim > 3 || g->deg < 1 || g->deg > 15) return ORC_EINVAL;
  /* Dirichlet boundaries: 1-D Euler only */
  if (g->bc != 0 && (g->bc != 1 || g->dim != 1 || g->mu > 0.0)) return ORC_EINVAL;
  if (g->bc && (g->bckind[0] < 0 || g->bckind[0] > 1 || g->bckind[1] < 0 || g->bckind[1] > 1))
    return ORC_EINVAL;
  G->bc = g->bc;
  G->dim = g->dim;
  G->n = g->deg + 1;
  G->nv = g->dim + 2;
  G->nd = 1;
  G->ne = 1;
  for (int m = 0; m < 3; ++m) {
    G->nel[m] = (m < g->dim) ? g->nel[m] : 1;
    if (G->nel[m] < 1) return ORC_EINVAL;
    G->h[m] = (m < g->dim) ? (g->hi[m] - g->lo[m]) / g->nel[m] : 1.0;
  }
  for (int m = 0; m < g->dim; ++m) {
    G->nd *= G->n;
    G->ne *= G->nel[m];
  }
  G->N = G->ne * G->nd;
  orc_lgl(g->deg, G->x, G->w);
  orc_dmat(g->deg, G->D);
  return ORC_OK;
}

long orc_num_elems(const orc_mesh* g) {
  geom G;
  return setup(g, &G) ? -1 : G.ne;
}
long orc_num_nodes(const orc_mesh* g) {
  geom G;
  return setup(g, &G) ? -1 : G.N;
}

static void elem_index(const geom* G, long k, int* km) {
  km[0] = (int)(k % G->nel[0]);
  km[1] = (int)((k / G->nel[0]) % G->nel[1]);
  km[2] = (int)(k / ((long)G->nel[0] * G->nel[1]));
}
static long elem_flat(const geom* G, const int* km) {
  return km[0] + (long)G->nel[0] * (km[1] + (long)G->nel[1] * km[2]);
}
/* Neighbour element across the face of k in direction m (dir = -1 or +1);
 * -1 on a Dirichlet boundary. */
static long neighbour(const geom* G, long k, int m, int dir) {
  int km[3];
  elem_index(G, k, km);
  if (G->bc && (km[m] + dir < 0 || km[m] + dir >= G->nel[m])) return -1;
  km[m] = (km[m] + dir + G->nel[m]) % G->nel[m];
  return elem_flat(G, km);
}
static void node_index(const geom* G, int i, int* im) {
  im[0] = im[1] = im[2] = 0;
  for (int m = 0; m < G->dim; ++m) {
    im[m] = i % G->n;
    i /= G->n;
  }
}
static int node_flat(const geom* G, const int* im) {
  int i = 0;
  for (int m = G->dim - 1; m >= 0; --m) i = i * G->n + im[m];
  return i;
}
static int node_with(const geom* G, int i, int m, int j) {
  int im[3];
  node_index(G, i, im);
  im[m] = j;
  return node_flat(G, im);
}
static double mass(const geom* G, int i) {
  int im[3];
  node_index(G, i, im);
  double M = 1.0;
  for (int m = 0; m < G->dim; ++m) M *= 0.5 * G->h[m] * G->w[im[m]];
  return M;
}
static void gather(const geom* G, const double* a, long gi, double* out) {
  for (int v = 0; v < G->nv; ++v) out[v] = a[v * G->N + gi];
}

static void two_point(const orc_mesh* g, int m, const double* uL, const double* uR,
                      double* f) {
  if (g->volume_flux == 1) {
    double fl[5], fr[5];
    orc_phys_flux(g->dim, g->gas_gamma, m, uL, fl);
    orc_phys_flux(g->dim, g->gas_gamma, m, uR, fr);
    for (int v = 0; v < g->dim + 2; ++v) f[v] = 0.5 * (fl[v] + fr[v]);
  } else {
    orc_ec_flux(g->dim, g->gas_gamma, m, uL, uR, f);
  }
}

static double normal_speed(int dim, double gg, int m, const double* u) {
  double rho = u[0], ke = 0.0;
  for (int k = 0; k < dim; ++k) ke += u[1 + k] * u[1 + k] / rho;
  double p = (gg - 1.0) * (u[dim + 1] - 0.5 * ke);
  return fabs(u[1 + m] / rho) + sqrt(gg * p / rho);
}

/* interface flux f* between a left and a right state in direction m */
static void interface_flux(const orc_mesh* g, int m, const double* uL, const double* uR,
                           double* fs) {
  int nv = g->dim + 2;
  two_point(g, m, uL, uR, fs);
  double lam = fmax(normal_speed(g->dim, g->gas_gamma, m, uL),
                    normal_speed(g->dim, g->gas_gamma, m, uR));
  for (int v = 0; v < nv; ++v) fs[v] -= 0.5 * g->lambda_scale * lam * (uR[v] - uL[v]);
}

int orc_volume_term(const orc_mesh* g, const double* u, double* V) {
  geom G;
  if (setup(g, &G)) return ORC_EINVAL;
  for (long k = 0; k < G.ne; ++k) {
    for (int i = 0; i < G.nd; ++i) {
      long gi = k * G.nd + i;
      int im[3];
      node_index(&G, i, im);
      double ui[5], uj[5], f[5], acc[5] = {0, 0, 0, 0, 0};
      gather(&G, u, gi, ui);
      for (int m = 0; m < G.dim; ++m) {
        for (int j = 0; j < G.n; ++j) {
          gather(&G, u, k * G.nd + node_with(&G, i, m, j), uj);
          two_point(g, m, ui, uj, f);
          double c = (2.0 / G.h[m]) * 2.0 * G.D[im[m] * G.n + j];
          for (int v = 0; v < G.nv; ++v) acc[v] += c * f[v];
        }
      }
      for (int v = 0; v < G.nv; ++v) V[v * G.N + gi] = acc[v];
    }
  }
  return ORC_OK;
}

/* Surface SAT contribution (the term that is subtracted together with V). */
static void surface_term(const orc_mesh* g, const geom* G, const double* u, double* Sf) {
  const int p = G->n - 1;
  for (long k = 0; k < G->ne; ++k) {
    for (int i = 0; i < G->nd; ++i) {
      long gi = k * G->nd + i;
      int im[3];
      node_index(G, i, im);
      double ui[5], un[5], fs[5], fp[5], acc[5] = {0, 0, 0, 0, 0};
      gather(G, u, gi, ui);
      for (int m = 0; m < G->dim; ++m) {
        if (im[m] == p) { /* this node is the left state of the +m interface */
          long kn = neighbour(G, k, m, +1);
          if (kn < 0) /* right boundary: given state, or the trace itself (outflow) */
            for (int v = 0; v < G->nv; ++v) un[v] = g->bckind[1] ? ui[v] : g->ubc[1][v];
          else
            gather(G, u, kn * G->nd + node_with(G, i, m, 0), un);
          interface_flux(g, m, ui, un, fs);
          orc_phys_flux(G->dim, g->gas_gamma, m, ui, fp);
          double c = (2.0 / G->h[m]) / G->w[p];
          for (int v = 0; v < G->nv; ++v) acc[v] += c * (fs[v] - fp[v]);
        }
        if (im[m] == 0) { /* right state of the -m interface */
          long kn = neighbour(G, k, m, -1);
          if (kn < 0) /* left boundary */
            for (int v = 0; v < G->nv; ++v) un[v] = g->bckind[0] ? ui[v] : g->ubc[0][v];
          else
            gather(G, u, kn * G->nd + node_with(G, i, m, p), un);
          interface_flux(g, m, un, ui, fs);
          orc_phys_flux(G->dim, g->gas_gamma, m, ui, fp);
          double c = (2.0 / G->h[m]) / G->w[0];
          for (int v = 0; v < G->nv; ++v) acc[v] -= c * (fs[v] - fp[v]);
        }
      }
      for (int v = 0; v < G->nv; ++v) Sf[v * G->N + gi] = acc[v];
    }
  }
}

double orc_interface_dissipation(const orc_mesh* g, const double* u) {
  geom G;
  if (setup(g, &G)) return NAN;
  const int p = G.n - 1;
  double total = 0.0;
  for (long k = 0; k < G.ne; ++k) {
    for (int i = 0; i < G.nd; ++i) {
      int im[3];
      node_index(&G, i, im);
      for (int m = 0; m < G.dim; ++m) {
        if (im[m] != p) continue;
        double uL[5], uR[5], wL[5], wR[5];
        gather(&G, u, k * G.nd + i, uL);
        long kn = neighbour(&G, k, m, +1);
        if (kn < 0) continue; /* interior interfaces only */
        gather(&G, u, kn * G.nd + node_with(&G, i, m, 0), uR);
        orc_entropy_vars(G.dim, g->gas_gamma, uL, wL);
        orc_entropy_vars(G.dim, g->gas_gamma, uR, wR);
        double lam = fmax(normal_speed(G.dim, g->gas_gamma, m, uL),
                          normal_speed(G.dim, g->gas_gamma, m, uR));
        double a = 1.0; /* face quadrature weight */
        for (int q = 0; q < G.dim; ++q)
          if (q != m) a *= 0.5 * G.h[q] * G.w[im[q]];
        double dot = 0.0;
        for (int v = 0; v < G.nv; ++v) dot += (wR[v] - wL[v]) * (uR[v] - uL[v]);
        total += a * 0.5 * g->lambda_scale * lam * dot;
      }
    }
  }
  return total;
}

/* ---- BR1 viscous terms ---- */

/* lift of a central interface value onto the face nodes of element k */
static void br1_apply(const geom* G, int ncomp, long k, int i, int m,
                      const double* field_of_m, double* out) {
  /* out[c] = (2/h_m)[sum_j D[i_m][j] a_c(i[m<-j]) + lifts], for the ncomp
   * components of the field a stored at field_of_m[c * N + node]. */
  const int p = G->n - 1;
  int im[3];
  node_index(G, i, im);
  long gi = k * G->nd + i;
  for (int c = 0; c < ncomp; ++c) {
    double s = 0.0;
    for (int j = 0; j < G->n; ++j)
      s += G->D[im[m] * G->n + j] * field_of_m[c * G->N + k * G->nd + node_with(G, i, m, j)];
    double own = field_of_m[c * G->N + gi];
    if (im[m] == p) {
      long kn = neighbour(G, k, m, +1);
      double nb = field_of_m[c * G->N + kn * G->nd + node_with(G, i, m, 0)];
      s += (0.5 * (own + nb) - own) / G->w[p];
    }
    if (im[m] == 0) {
      long kn = neighbour(G, k, m, -1);
      double nb = field_of_m[c * G->N + kn * G->nd + node_with(G, i, m, p)];
      s -= (0.5 * (own + nb) - own) / G->w[0];
    }
    out[c] = (2.0 / G->h[m]) * s;
  }
}

int orc_br1_gradient(const orc_mesh* g, const double* u, double* theta) {
  geom G;
  if (setup(g, &G)) return ORC_EINVAL;
  double* W = (double*)malloc(sizeof(double) * G.nv * G.N);
  if (!W) return ORC_EINVAL;
  for (long gi = 0; gi < G.N; ++gi) {
    double ui[5], wi[5];
    gather(&G, u, gi, ui);
    orc_entropy_vars(G.dim, g->gas_gamma, ui, wi);
    for (int v = 0; v < G.nv; ++v) W[v * G.N + gi] = wi[v];
  }
  for (long k = 0; k < G.ne; ++k)
    for (int i = 0; i < G.nd; ++i)
      for (int m = 0; m < G.dim; ++m) {
        double out[5];
        br1_apply(&G, G.nv, k, i, m, W, out);
        for (int v = 0; v < G.nv; ++v) theta[(m * G.nv + v) * G.N + k * G.nd + i] = out[v];
      }
  free(W);
  return ORC_OK;
}

/* Viscous flux g_m at one node from the state and the gradients theta_m' of
 * the entropy variables, th[m' * nv + v].  Chain rule with
 * v_k = -w_{1+k}/w_E and T = -1/(R w_E). */
static void viscous_flux(const orc_mesh* g, const double* u, const double* th, int m,
                         double* out) {
  const int dim = g->dim, nv = dim + 2;
  const double gg = g->gas_gamma, R = g->gas_r, mu = g->mu;
  double rho = u[0], v[3] = {0, 0, 0}, ke = 0.0;
  for (int k = 0; k < dim; ++k) {
    v[k] = u[1 + k] / rho;
    ke += v[k] * u[1 + k];
  }
  double p = (gg - 1.0) * (u[dim + 1] - 0.5 * ke);
  double wE = -rho / p;
  double dv[3][3] = {{0}}, dT[3] = {0};
  for (int q = 0; q < dim; ++q) {
    for (int k = 0; k < dim; ++k)
      dv[k][q] = (-th[q * nv + 1 + k] - v[k] * th[q * nv + dim + 1]) / wE;
    dT[q] = th[q * nv + dim + 1] / (R * wE * wE);
  }
  double div = 0.0;
  for (int k = 0; k < dim; ++k) div += dv[k][k];
  double kappa = mu * (gg * R / (gg - 1.0)) / g->prandtl;
  out[0] = 0.0;
  double e = 0.0;
  for (int k = 0; k < dim; ++k) {
    double tau = mu * (dv[k][m] + dv[m][k] - (k == m ? 2.0 / 3.0 * div : 0.0));
    out[1 + k] = tau;
    e += tau * v[k];
  }
  out[dim + 1] = e + kappa * dT[m];
}

static int viscous_term(const orc_mesh* g, const geom* G, const double* u, double* visc,
                        double* visc_diss) {
  const int nv = G->nv, dim = G->dim;
  double* th = (double*)malloc(sizeof(double) * dim * nv * G->N);
  double* gf = (double*)malloc(sizeof(double) * dim * nv * G->N);
  if (!th || !gf) {
    free(th);
    free(gf);
    return ORC_EINVAL;
  }
  orc_br1_gradient(g, u, th);
  for (long gi = 0; gi < G->N; ++gi) {
    double ui[5], tloc[15], out[5];
    gather(G, u, gi, ui);
    for (int q = 0; q < dim; ++q)
      for (int v = 0; v < nv; ++v) tloc[q * nv + v] = th[(q * nv + v) * G->N + gi];
    for (int m = 0; m < dim; ++m) {
      viscous_flux(g, ui, tloc, m, out);
      for (int v = 0; v < nv; ++v) gf[(m * nv + v) * G->N + gi] = out[v];
    }
  }
  for (long k = 0; k < G->ne; ++k) {
    double diss = 0.0;
    for (int i = 0; i < G->nd; ++i) {
      long gi = k * G->nd + i;
      double acc[5] = {0, 0, 0, 0, 0};
      for (int m = 0; m < dim; ++m) {
        double out[5];
        br1_apply(G, nv, k, i, m, gf + (long)m * nv * G->N, out);
        for (int v = 0; v < nv; ++v) acc[v] += out[v];
        for (int v = 0; v < nv; ++v)
          diss += mass(G, i) * th[(m * nv + v) * G->N + gi] * gf[(m * nv + v) * G->N + gi];
      }
      for (int v = 0; v < nv; ++v) visc[v * G->N + gi] = acc[v];
    }
    if (visc_diss) visc_diss[k] = diss;
  }
  free(th);
  free(gf);
  return ORC_OK;
}

int orc_rhs(const orc_mesh* g, const double* u, double* dudt, double* eta_rate,
            double* visc_diss) {
  geom G;
  if (setup(g, &G)) return ORC_EINVAL;
  for (long gi = 0; gi < G.N; ++gi) {
    double ui[5];
    gather(&G, u, gi, ui);
    double rho = ui[0], ke = 0.0;
    for (int k = 0; k < G.dim; ++k) ke += ui[1 + k] * ui[1 + k] / rho;
    double p = (g->gas_gamma - 1.0) * (ui[G.dim + 1] - 0.5 * ke);
    if (!(rho > 0.0) || !(p > 0.0)) return ORC_ENONPHYS;
  }
  double* V = (double*)malloc(sizeof(double) * G.nv * G.N);
  double* Sf = (double*)malloc(sizeof(double) * G.nv * G.N);
  double* Vi = NULL;
  if (!V || !Sf) {
    free(V);
    free(Sf);
    return ORC_EINVAL;
  }
  orc_volume_term(g, u, V);
  surface_term(g, &G, u, Sf);
  for (long q = 0; q < (long)G.nv * G.N; ++q) dudt[q] = -(V[q] + Sf[q]);
  if (g->mu > 0.0) {
    Vi = (double*)malloc(sizeof(double) * G.nv * G.N);
    if (!Vi) {
      free(V);
      free(Sf);
      return ORC_EINVAL;
    }
    viscous_term(g, &G, u, Vi, visc_diss);
    for (long q = 0; q < (long)G.nv * G.N; ++q) dudt[q] += Vi[q];
  } else if (visc_diss) {
    for (long k = 0; k < G.ne; ++k) visc_diss[k] = 0.0;
  }
  if (eta_rate) {
    for (long k = 0; k < G.ne; ++k) {
      double s = 0.0;
      for (int i = 0; i < G.nd; ++i) {
        long gi = k * G.nd + i;
        double ui[5], wi[5];
        gather(&G, u, gi, ui);
        orc_entropy_vars(G.dim, g->gas_gamma, ui, wi);
        double dot = 0.0;
        for (int v = 0; v < G.nv; ++v) dot += wi[v] * dudt[v * G.N + gi];
        s += mass(&G, i) * dot;
      }
      eta_rate[k] = s;
    }
  }
  free(V);
  free(Sf);
  free(Vi);
  return ORC_OK;
}

int orc_elem_entropy(const orc_mesh* g, const double* u, double* eta) {
  geom G;
  if (setup(g, &G)) return ORC_EINVAL;
  for (long k = 0; k < G.ne; ++k) {
    double s = 0.0;
    for (int i = 0; i < G.nd; ++i) {
      double ui[5];
      gather(&G, u, k * G.nd + i, ui);
      s += mass(&G, i) * orc_entropy(G.dim, g->gas_gamma, ui);
    }
    eta[k] = s;
  }
  return ORC_OK;
}

int orc_elem_max_speed(const orc_mesh* g, const double* u, double* smax) {
  geom G;
  if (setup(g, &G)) return ORC_EINVAL;
  for (long k = 0; k < G.ne; ++k) {
    double s = 0.0;
    for (int i = 0; i < G.nd; ++i) {
      double ui[5];
      gather(&G, u, k * G.nd + i, ui);
      s = fmax(s, orc_wave_speed(G.dim, g->gas_gamma, ui));
    }
    smax[k] = s;
  }
  return ORC_OK;
}

double orc_cfl_dt(const orc_mesh* g, const double* u, double cfl) {
  geom G;
  if (setup(g, &G)) return NAN;
  double smax = 0.0, hmin = G.h[0];
  for (int m = 1; m < G.dim; ++m) hmin = fmin(hmin, G.h[m]);
  for (long gi = 0; gi < G.N; ++gi) {
    double ui[5];
    gather(&G, u, gi, ui);
    smax = fmax(smax, orc_wave_speed(G.dim, g->gas_gamma, ui));
  }
  return cfl * hmin / ((double)G.n * smax);
}

/* exported for the relaxation file */
int orc__geom_mass(const orc_mesh* g, double* M) {
  geom G;
  if (setup(g, &G)) return ORC_EINVAL;
  for (int i = 0; i < G.nd; ++i) M[i] = mass(&G, i);
  return ORC_OK;
}
