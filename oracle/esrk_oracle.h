/*
 * esrk_oracle.h -- plain, slow CPU reference of the locally entropy-stable
 * relaxation Runge-Kutta hot path (Ranocha, Dalcin, Parsani, arXiv:2003.08831).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the oracle that the GPU path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source, header, table or
 * helper with the HIP library; both sides only agree on the array layout.
 *
 * Everything is FP64 except the relaxation function r_kappa(gamma), whose
 * element sums are accumulated in x87 extended precision (long double): the
 * root of r_kappa is a small difference of large entropy sums.
 *
 * Layout of every state array (host memory, caller-owned):
 *   u[v*N + k*nd + i]   v in [0, dim+2): rho, rho*v_1..rho*v_dim, rho*E
 *                       k = element, lexicographic with x fastest
 *                       i = node, lexicographic over (deg+1)^dim, xi_1 fastest
 *   nd = (deg+1)^dim, N = (number of elements) * nd.
 *
 * Return codes: 0 ok, negative on error (see ORC_E* below).
 */
#ifndef ESRK_ORACLE_H
#define ESRK_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOROOT (-4) /* an active element has no positive relaxation root */
#define ORC_ENONPHYS (-5) /* rho <= 0 or p <= 0 in a state that must be admissible */

/* Periodic Cartesian mesh of (deg+1)^dim Lobatto-node elements and the
 * physics constants.  mu == 0 means the Euler equations. */
typedef struct {
  int dim;              /* 1, 2 or 3 */
  int deg;              /* polynomial degree p; n = p+1 nodes per direction */
  int nel[3];           /* elements per direction (entries >= dim ignored) */
  double lo[3], hi[3];  /* domain box */
  double gas_gamma;     /* ratio of specific heats */
  double gas_r;         /* gas constant R in p = rho R T */
  double mu;            /* dynamic viscosity (constant); 0 -> Euler */
  double prandtl;       /* Prandtl number */
  double lambda_scale;  /* interface dissipation scale: 1 = local Lax-Friedrichs, 0 = EC */
  int volume_flux;      /* 0 = entropy-conservative (Chandrashekar), 1 = central average */
  int bc;               /* 0 = periodic; 1 = boundaries at both ends (1-D Euler only) */
  double ubc[2][5];     /* Dirichlet exterior states (conserved), [0] left, [1] right */
  int bckind[2];        /* per end: 0 = Dirichlet (exterior state ubc), 1 = outflow
                           (exterior state = the interior trace, so the SAT vanishes) */
} orc_mesh;

/* ---- summation-by-parts operators on Lobatto nodes (Sec. 3.1) ---- */
int orc_lgl(int deg, double* x, double* w);      /* x[n], w[n] */
int orc_dmat(int deg, double* D);                /* D[i*n+j] = l_j'(x_i) */

/* ---- pointwise thermodynamics and fluxes (Sec. 3.1) ---- */
double orc_logmean(double a, double b);
double orc_entropy(int dim, double gg, const double* u);                 /* S = -rho s/(gg-1) */
void orc_entropy_vars(int dim, double gg, const double* u, double* w);   /* w = dS/du */
void orc_phys_flux(int dim, double gg, int m, const double* u, double* f);
void orc_ec_flux(int dim, double gg, int m, const double* uL, const double* uR, double* f);
double orc_wave_speed(int dim, double gg, const double* u);              /* sum_m |v_m| + c */

/* ---- semidiscretization (Sec. 3.1, the element equation) ---- */
long orc_num_elems(const orc_mesh* g);
long orc_num_nodes(const orc_mesh* g);
/* dudt = f(u).  eta_rate[k] = sum_i M_i w(u_i).dudt_i (nullable).
 * visc_diss[k] = sum_i M_i sum_m theta_m,i . g_m,i (nullable; 0 for Euler). */
int orc_rhs(const orc_mesh* g, const double* u, double* dudt, double* eta_rate,
            double* visc_diss);
/* Volume flux-differencing term alone, V_i (no sign flip), for the pins. */
int orc_volume_term(const orc_mesh* g, const double* u, double* V);
/* Sum over all interfaces and face nodes of a*(lambda/2)*(w_R-w_L).(u_R-u_L). */
double orc_interface_dissipation(const orc_mesh* g, const double* u);
/* BR1 gradient of the entropy variables theta[(m*nv + v)*N + node]. */
int orc_br1_gradient(const orc_mesh* g, const double* u, double* theta);
/* eta[k] = sum_i M_i S(u_i) */
int orc_elem_entropy(const orc_mesh* g, const double* u, double* eta);
/* dt = cfl * min_m h_m / ((deg+1) * max_i sum_m(|v_m|+c)) */
double orc_cfl_dt(const orc_mesh* g, const double* u, double cfl);

/* ---- explicit Runge-Kutta step with the entropy estimate (Sec. 2, RK example) ---- */
#define ORC_SSPRK33 0
#define ORC_RK44 1
#define ORC_BSRK43 2 /* Bogacki-Shampine 3(2), embedded pair */
#define ORC_BSRK85 3 /* Bogacki-Shampine 5(4), embedded pair */
int orc_tableau_stages(int tableau);
/* Butcher tableau, zero padded to 8 stages: A[8*8] row-major, b, bhat (zero
 * without an embedded method), c; s stages, order p, embedded order q (0: none). */
int orc_tableau(int tableau, double* A, double* b, double* bhat, double* c, int* s, int* p,
                int* q);
/* One step from u_old with step dt.  Outputs:
 *   du[nv*N]   = dt * sum_i b_i k_i          (u_new - u_old)
 *   deta[N_e]  = dt * sum_i b_i e_i,k        (eta_new - eta_old)
 *   ystages    = s stage vectors y^i (nullable, s*nv*N)
 *   kstages    = s stage slopes k_i (nullable)
 *   estages    = s per-element entropy rates e_i,k (nullable, s*N_e) */
int orc_rk_step(const orc_mesh* g, int tableau, const double* u_old, double dt,
                double* du, double* deta, double* ystages, double* kstages,
                double* estages);

/* The same step plus a[N_e]: phi_k(0) = sum_i M w(u_old).du - deta_k evaluated
 * as dt sum_i b_i sum_nodes M (w(u_old) - w(y^i)).k_i (the same quantity
 * without the cancelling difference; entropy variables in extended precision). */
int orc_rk_step_a(const orc_mesh* g, int tableau, const double* u_old, double dt,
                  double* du, double* deta, double* a);
/* The same step plus the embedded pair's error estimate
 * err[nv*N] = dt sum_i (b_i - bhat_i) k_i (ORC_EINVAL without an embedded method). */
int orc_rk_step_err(const orc_mesh* g, int tableau, const double* u_old, double dt,
                    double* du, double* deta, double* err);
/* sqrt(mean over all nv*N entries of (err / (atol + rtol max(|u_old|, |u_old+du|)))^2) */
double orc_error_norm(const orc_mesh* g, const double* u_old, const double* du,
                      const double* err, double atol, double rtol);
/* Step-size factor clip(safety err^(-1/(q+1)), 0.1, 10), safety 0.9 after an
 * accepted step and 0.45 after a rejected one. */
double orc_adapt_factor(double err, int q, int accepted);
/* ---- local relaxation (Sec. 2, local relaxation equation and theorem) ---- */
typedef struct {
  double tol;        /* bracket width at which bisection stops (relative to max(1,gamma)) */
  double gamma_max;  /* largest relaxation parameter tried */
  int maxit;         /* bisection iteration cap */
} orc_relax_opts;

/* One error-controlled step attempt: the embedded pair's step from u with dt
 * (dt <= 0: CFL rule), the error norm; accepted iff norm <= 1, then the
 * relaxation of `mode` (0 local, 1 global, 2 none; phi(0) from
 * orc_rk_step_a) and the relaxed update of u
 * and t; rejected: u and t unchanged.  dt_next = dt * orc_adapt_factor. */
int orc_adaptive_step(const orc_mesh* g, int tableau, const orc_relax_opts* o, int mode,
                      double atol, double rtol, double cfl, double dt, double* u, double* t,
                      double* gamma, double* err, int* accepted, double* dt_next,
                      double* dt_used);

/* Per element: r_k(gamma) = eta_k(u_old + gamma du) - eta_k(u_old) - gamma deta_k,
 * phi_k = r_k / gamma; gamma_k = its positive root (or +INF for an inactive
 * element, or gamma_max).  gamma = min_k gamma_k (1 if all inactive).
 * Optional outputs: phi0[k] = phi_k(0), curv[k] = r_k(1) - phi_k(0),
 * noise[k] = the round-off scale used for the activity test, iters[k]. */
int orc_local_relaxation_solve(const orc_mesh* g, const orc_relax_opts* o,
                               const double* u_old, const double* du,
                               const double* deta, double* gamma_k, double* gamma,
                               double* phi0, double* curv, double* noise,
                               int* iters, long* bad_elem);
/* The same with phi_k(0) supplied (a[N_e], e.g. from orc_rk_step_a; NULL:
 * A - deta): phi_k(gamma) = a_k + B_k(gamma)/gamma with B_k the relative
 * entropy sum; the activity test and its outputs are unchanged. */
int orc_local_relaxation_solve_a(const orc_mesh* g, const orc_relax_opts* o,
                                 const double* u_old, const double* du, const double* deta,
                                 const double* a, double* gamma_k, double* gamma,
                                 double* phi0, double* curv, double* noise, int* iters,
                                 long* bad_elem);
/* r_k(gamma) for one element (for tests). */
long double orc_relax_r(const orc_mesh* g, long k, const double* u_old,
                        const double* du, double deta_k, double gamma, int* admissible);

/* Global relaxation: one gamma with eta(u_old + gamma du) = eta(u_old) + gamma sum_k deta_k
 * (root of r = sum_k r_k; gamma = 1 if its curvature r(1) - phi(0) is at round-off level,
 * ORC_ENOROOT if phi(0) >= 0).  phi0, curv, noise, iters nullable. */
int orc_global_relaxation_solve(const orc_mesh* g, const orc_relax_opts* o,
                                const double* u_old, const double* du, const double* deta,
                                double* gamma, double* phi0, double* curv, double* noise,
                                int* iters);
/* The same with the per-element phi_k(0) supplied (summed; NULL: A - D). */
int orc_global_relaxation_solve_a(const orc_mesh* g, const orc_relax_opts* o,
                                  const double* u_old, const double* du, const double* deta,
                                  const double* a, double* gamma, double* phi0, double* curv,
                                  double* noise, int* iters);
long double orc_global_relax_r(const orc_mesh* g, const double* u_old, const double* du,
                               const double* deta, double gamma, int* admissible);

/* Generic safeguarded bracket + bisection on a nondecreasing phi with phi(0) = phi0 < 0. */
typedef long double (*orc_phi_fn)(double gamma, void* ctx, int* admissible);
int orc_root_nondecreasing(orc_phi_fn phi, void* ctx, double phi0,
                           const orc_relax_opts* o, double* root, int* iters);

/* Whole step: RK step (with phi_k(0) from orc_rk_step_a), local relaxation,
 * global gamma, relaxed update.
 * dt <= 0 takes dt from the CFL rule.  On return u holds u_gamma, *t the
 * relaxed time t_old + gamma*dt.  gamma_k (nullable, N_e). */
int orc_step(const orc_mesh* g, int tableau, const orc_relax_opts* o, double cfl,
             double dt, double* u, double* t, double* gamma, double* gamma_k,
             double* dt_used, long* bad_elem);

/* ---- network proposing initial relaxation parameters (mlp.c) ---- */
#define ORC_MLP_PARAMS 1281
/* Y[b] = network(X[b][0..5)) */
int orc_mlp_forward(const double* params, const double* X, int B, double* Y);
/* grad[ORC_MLP_PARAMS] = dL/dparams, L = mean_b (Y[b] - T[b])^2 (also returned) */
int orc_mlp_grad(const double* params, const double* X, const double* T, int B, double* grad,
                 double* loss);
/* One Adam update of params[ORC_MLP_PARAMS] (beta1 0.9, beta2 0.999, eps 1e-8). */
int orc_mlp_adam(double* params, const double* grad, double* m, double* v, int step, double lr);
/* Sample normalization; model holds ORC_MLP_MODEL entries (see mlp.c). */
#define ORC_MLP_MODEL 1298
int orc_mlp_prepare(double* model, const double* raw, const double* gamma, int B, int fit,
                    double* xn, double* tn);
/* smax[k] = max over the nodes of element k of sum_m (|v_m| + c) */
int orc_elem_max_speed(const orc_mesh* g, const double* u, double* smax);

#ifdef __cplusplus
}
#endif
#endif
