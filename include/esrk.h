/*
 * esrk.h -- C-ABI of the MI355X (gfx950) locally entropy-stable relaxation
 * Runge-Kutta hot path (Ranocha, Dalcin, Parsani, "Fully-Discrete Explicit
 * Locally Entropy-Stable Schemes for the Compressible Euler and Navier-Stokes
 * Equations", arXiv:2003.08831).
 *
 * The problem is the ODE u' = f(u) of Sec. 1, with f the entropy-stable
 * semidiscretization of Sec. 3.1 (element equation: flux-differencing volume
 * term with an entropy-conservative two-point flux on tensor-product Lobatto
 * nodes, interface SATs with local Lax-Friedrichs dissipation and, for
 * Navier-Stokes, BR1 viscous terms), advanced by an explicit Runge-Kutta
 * method (Sec. 2, Runge-Kutta example) and made locally entropy stable by the
 * local relaxation of Sec. 2 (local relaxation equation; theorem with
 * gamma = min_k gamma_k).
 *
 * Conventions for every call:
 *  - all array arguments are DEVICE pointers (HIP device memory, e.g. from
 *    torch.empty(..., device="cuda")) owned by the caller; the library never
 *    frees or retains them beyond the call;
 *  - state layout: double u[v * N + k * nd + i], v in [0, dim+2) for
 *    rho, rho*v_1..rho*v_dim, rho*E; element k lexicographic with x fastest;
 *    node i lexicographic over (deg+1)^dim with xi_1 fastest;
 *    nd = (deg+1)^dim, N = num_elems * nd;
 *  - per-element arrays have num_elems entries;
 *  - `stream` is a hipStream_t (NULL = the default stream); calls only
 *    enqueue work on it and never synchronize the host, except
 *    esrk_sync_status;
 *  - argument errors are returned synchronously; conditions detected on the
 *    device (no relaxation root, non-physical state) are latched in a device
 *    status word and reported by esrk_sync_status;
 *  - a context is not thread-safe; calls on one context must not overlap.
 *  - the mesh is a periodic Cartesian box; every element has the same
 *    polynomial degree.
 */
#ifndef ESRK_H
#define ESRK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ESRK_OK = 0,
  ESRK_EINVAL = 1,   /* bad argument or configuration */
  ESRK_EHIP = 2,     /* a HIP runtime call failed */
  ESRK_ENOMEM = 3,   /* workspace allocation failed */
  ESRK_ENOROOT = 4,  /* an active element has no positive relaxation root */
  ESRK_ENONPHYS = 5, /* rho <= 0 or p <= 0 in a state */
  ESRK_ENAN = 6,     /* a NaN was produced */
  ESRK_ENOTSUP = 7   /* configuration not compiled in */
} esrk_status;

enum { ESRK_FP64 = 0, ESRK_FP32_FLUX = 1 };
/* Runge-Kutta methods (Sec. 4 lists the ones used there): SSPRK(3,3);
 * classical RK(4,4); BSRK(4,3), the Bogacki-Shampine 3(2) embedded pair;
 * BSRK(8,5), the Bogacki-Shampine 5(4) embedded pair.  The last two evaluate
 * their last stage at the propagated solution with weight zero: without error
 * control esrk_step skips that stage. */
enum { ESRK_SSPRK33 = 0, ESRK_RK44 = 1, ESRK_BSRK43 = 2, ESRK_BSRK85 = 3 };
/* Trial-point rule of the relaxation root solves (esrk_set_root_method): all
 * keep the bracket [lo, hi] with phi(lo) <= 0 < phi(hi) and stop at the same
 * width (Alefeld also at an exact zero of phi), so they return the same root
 * to root_tol. */
enum { ESRK_ROOT_ILLINOIS = 0, ESRK_ROOT_BRENT = 1, ESRK_ROOT_BISECTION = 2, ESRK_ROOT_ALEFELD = 3 };
/* Relaxation applied by esrk_step (esrk_set_relaxation_mode). */
enum { ESRK_RELAX_LOCAL = 0, ESRK_RELAX_GLOBAL = 1, ESRK_RELAX_NONE = 2 };

typedef struct {
  int dim;             /* 1, 2 or 3 */
  int deg;             /* polynomial degree p in [1, 5]; p+1 Lobatto nodes per direction */
  int nel[3];          /* elements per direction (entries >= dim ignored) */
  double lo[3], hi[3]; /* periodic box */
  double gas_gamma;    /* ratio of specific heats */
  double gas_r;        /* gas constant in p = rho R T */
  double mu;           /* constant dynamic viscosity (0: Euler) */
  double prandtl;      /* Prandtl number */
  double lambda_scale; /* interface dissipation: 1 = local Lax-Friedrichs, 0 = EC surface */
  int precision;       /* ESRK_FP64, or ESRK_FP32_FLUX (flux differencing in FP32) */
  int tableau;         /* ESRK_SSPRK33, ESRK_RK44, ESRK_BSRK43 or ESRK_BSRK85 (all b_i >= 0) */
  double cfl;          /* dt = cfl * min h / ((deg+1) * max_i sum_m (|v_m| + c)) */
  double root_tol;     /* relaxation bracket width, relative to max(1, gamma) */
  int root_maxit;      /* iteration cap of the per-element root solve */
  double gamma_max;    /* largest relaxation parameter tried */
} esrk_config;

typedef struct esrk_ctx esrk_ctx;

/* Creates a context: validates cfg (ESRK_EINVAL also when a state array,
 * (dim+2) * elements * (deg+1)^dim values, would exceed 2^31 - 1 entries:
 * the kernels index it in 32 bits), builds the Lobatto SBP tables and
 * allocates all device workspace (the only allocation the library makes).
 * Sec. 3.1 (diagonal-norm SBP operators on Lobatto nodes). */
esrk_status esrk_create(const esrk_config* cfg, esrk_ctx** out);
void esrk_destroy(esrk_ctx* ctx);

size_t esrk_num_nodes(const esrk_ctx* ctx);
size_t esrk_num_elems(const esrk_ctx* ctx);
int esrk_num_vars(const esrk_ctx* ctx);

/* dudt = f(u) for the Euler equations (Sec. 3.1, element equation without
 * the viscous terms).  eta_rate (nullable, [num_elems]):
 * eta_rate[k] = sum_i M_i w(u_i).dudt_i, the element entropy rate that enters
 * the estimate of Sec. 2 (Runge-Kutta example).  u and dudt must not alias. */
esrk_status esrk_rhs_euler(esrk_ctx* ctx, const double* u, double* dudt,
                           double* eta_rate, void* stream);

/* dudt = f(u) for Navier-Stokes (Sec. 3.1: Euler part plus the BR1 viscous
 * terms in entropy variables; the context must have mu > 0, else
 * ESRK_EINVAL).  eta_rate as for esrk_rhs_euler (it includes the viscous
 * contribution).  visc_diss (nullable, [num_elems]):
 * sum_i M_i sum_m theta_m,i . g_m,i >= 0, the element's viscous entropy
 * dissipation rate.  u and dudt must not alias. */
esrk_status esrk_rhs_ns(esrk_ctx* ctx, const double* u, double* dudt, double* eta_rate,
                        double* visc_diss, void* stream);

/* One stage of the configured Runge-Kutta method (Sec. 2, stage equations and
 * estimate), stage in [0, s):
 *   k = f(y_in);
 *   du  = (stage == 0 ? 0 : du) + dt b_stage k          (u_new - u_old after the last stage)
 *   deta[k] = (stage == 0 ? 0 : deta[k]) + dt b_stage sum_i M_i w(y_in).k
 *   y_out = y^{stage+1} (omitted after the last stage; y_out may be NULL there).
 * For stage 0, y_in must equal u_old.  y_out must not alias y_in or u_old.
 * BSRK(4,3) and BSRK(8,5) form y_out from u_old and the slopes of earlier
 * stages, which the context stores: run the stages of one step in order, with
 * the same u_old and dt.  They also accumulate the embedded pair's error
 * estimate in the context (esrk_error_estimate).  Every stage also adds its
 * part of phi_k(0) to the context's accumulator (esrk_stage_phi0); deta may
 * be NULL, and then the entropy rate w(y_in).k is not formed (what esrk_step
 * does: its solves need only phi_k(0)). */
esrk_status esrk_rk_stage(esrk_ctx* ctx, int stage, double dt, const double* u_old,
                          const double* y_in, double* y_out, double* du, double* deta,
                          void* stream);

/* Local relaxation (Sec. 2, local relaxation equation and theorem).  With the
 * increments du = u_new - u_old and deta = eta_new - eta_old (eta_old is
 * eta_k(u_old) for Runge-Kutta), gamma_k is the positive root of
 *   phi_k(g) = (eta_k(u_old + g du) - eta_k(u_old) - g deta_k) / g,
 * solved per element to root_tol; elements whose root is not determinable in
 * FP64 (curvature r_k(1) - phi_k(0) at most
 * 64 eps (sum_i M_i sum_v |w_v du_v| + |deta_k|)) get +INF.  With precision
 * ESRK_FP32_FLUX the increments carry FP32 flux rounding: eps is then the
 * FP32 epsilon, and an element with phi_k(0) >= 0 whose entropy change r_k(1)
 * stays within that level is inactive too.  An element with
 * -B_k(1)/2 < phi_k(0) <= its round-off level (B_k(1) = r_k(1) - phi_k(0),
 * the relative entropy of the step; the root would lie below about 1/2) is
 * degenerate and inactive: the existence lemma needs the element's own slope
 * at u_old to carry the curvature, and an element that a wave reaches only
 * in the last stages of the step has none.  An element with phi_k(0) above
 * the round-off level latches ESRK_ENOROOT.  *gamma (device scalar) =
 * min_k gamma_k, or 1 if every element is inactive.  gamma_guess (nullable,
 * float [num_elems]) seeds the solve: after phi_k(1) it is the next trial
 * point if it lies in (0, gamma_max]; the result does not depend on it beyond
 * root_tol.  iters (nullable, [num_elems]) receives the number of phi
 * evaluations per element. */
esrk_status esrk_local_relaxation_solve(esrk_ctx* ctx, const double* u_old,
                                        const double* du, const double* deta,
                                        const float* gamma_guess, double* gamma_k,
                                        double* gamma, int32_t* iters, void* stream);

/* phi_k(0) = sum_i M w(u_old).du - deta_k of each element, accumulated by the
 * last run of stages (esrk_rk_stage or esrk_step) without the cancelling
 * difference: dt sum_i b_i sum_nodes M (w(u_old) - w(y^i)).k_i, with the
 * entropy-variable changes w(y^i) - w(u_old) written in the state
 * differences (an identity of the estimate's definition in Sec. 2; in
 * elements with round-off-level dynamics the difference form loses its
 * digits and such an element can set gamma = min_k gamma_k).  phi0 device
 * [num_elems].  Enqueue only. */
esrk_status esrk_stage_phi0(esrk_ctx* ctx, double* phi0, void* stream);

/* esrk_local_relaxation_solve with phi_k(0) supplied (device [num_elems],
 * e.g. from esrk_stage_phi0 after the stages that produced du and deta):
 * phi_k(g) = phi0_k + B_k(g)/g.  The activity test is unchanged.  esrk_step
 * solves this way. */
esrk_status esrk_local_relaxation_solve_phi0(esrk_ctx* ctx, const double* u_old,
                                             const double* du, const double* deta,
                                             const double* phi0, double* gamma_k,
                                             double* gamma, int32_t* iters, void* stream);

/* One whole locally relaxed step, in place on u (Sec. 2: RK step, estimate,
 * gamma = min_k gamma_k, u <- u + gamma du, t <- t + gamma dt).  t is a device
 * scalar.  dt > 0 is used as given; dt <= 0 takes dt from the CFL rule on the
 * device, or, under error control (esrk_set_adaptive) after the first
 * attempt, the controller's proposal.  gamma_k_out (nullable, [num_elems])
 * and stats_out (nullable, device double[8] = {gamma, dt, t, number of
 * inactive elements, largest and total number of phi evaluations of the root
 * solves, weighted error norm (0 without error control), 1 if the attempt was
 * accepted else 0}) are written on the device.  A rejected attempt leaves u
 * and t unchanged (gamma_k = +INF, stats gamma = 1) and only shrinks the
 * proposal.  If the device detects an error, u and t are left unchanged and the
 * status is latched.  No host synchronization, no allocation, in every
 * relaxation mode (esrk_set_relaxation_mode). */
esrk_status esrk_step(esrk_ctx* ctx, double* u, double* t, double dt, double* gamma_k_out,
                      double* stats_out, void* stream);

/* nsteps calls of esrk_step(ctx, u, t, 0 (CFL step size), NULL, stats_out)
 * recorded once into a HIP graph and replayed on `stream` (not the NULL
 * stream): the same kernels and arguments as the eager steps, so the same
 * results bit for bit, with one launch for the whole loop.  The recording is
 * kept and replayed while u, t, stats_out, nsteps, the stream and the
 * context's settings are unchanged; any setter call (relaxation mode, root
 * method, boundary states, error control, step model) makes the next call
 * record again.  ENOTSUP under error control (the controller's state lives
 * on the host); EINVAL for NULL u, t or stream or nsteps < 1.  Enqueue only;
 * device errors are latched as for esrk_step. */
esrk_status esrk_run_graph(esrk_ctx* ctx, double* u, double* t, int nsteps, double* stats_out,
                           void* stream);

/* Global relaxation (Sec. 2, the relaxation equation applied to the total
 * entropy instead of each element's): one gamma with
 *   eta(u_old + gamma du) = eta(u_old) + gamma sum_k deta_k,
 * eta being the total entropy sum_k eta_k, solved to root_tol.  The same
 * activity rule as the local solve, summed over the mesh: gamma = 1 if the
 * curvature r(1) - phi(0) is at most
 * 64 eps (sum_i M_i sum_v |w_v du_v| + sum_k |deta_k|); otherwise
 * phi(0) >= 0 returns ESRK_ENOROOT.  The root lies between the smallest and
 * the largest per-element root.  Each device pass sweeps the nodes once for
 * four trial values and a one-block kernel updates the bracket on the device
 * (up to 12 passes; a pass after convergence returns at once).  This call
 * waits for the result: *gamma (device scalar) is written before it returns,
 * *passes (nullable, host) receives the number of passes that did work.
 * ESRK_ENAN if the sums at gamma = 1 are not finite (a state that is not
 * physical, say); nothing is latched on the device. */
esrk_status esrk_global_relaxation_solve(esrk_ctx* ctx, const double* u_old,
                                         const double* du, const double* deta,
                                         double* gamma, int* passes, void* stream);

/* Relaxation used by esrk_step: ESRK_RELAX_LOCAL (default: gamma = min_k
 * gamma_k), ESRK_RELAX_GLOBAL (the root of esrk_global_relaxation_solve,
 * found on the device without host synchronization; ESRK_ENOROOT and
 * ESRK_ENAN are latched like the local solve's errors, gamma_k_out is not
 * written) or ESRK_RELAX_NONE (the unrelaxed Runge-Kutta step, gamma = 1).
 * All three are enqueue-only.  In the last two modes stats_out
 * reports zero inactive elements and zero evaluations.  EINVAL for another
 * mode. */
esrk_status esrk_set_relaxation_mode(esrk_ctx* ctx, int mode);

/* Error control of the embedded pairs (Sec. 4 runs them with error-controlled
 * steps; the controller is not given there, so this is the elementary one):
 * an attempt with step dt has the estimate err = dt sum_i (b_i - bhat_i) k_i
 * and the norm
 *   E = sqrt(mean over all nv*N entries of (err / (atol + rtol max(|u_old|, |u_old + du|)))^2);
 * it is accepted iff E <= 1, and the next proposal is
 *   dt * min(10, max(0.1, s E^(-1/(q+1)))), s = 0.9 after an accepted and 0.45
 * after a rejected attempt (0.1 for a non-finite E, 10 for E = 0), q the
 * embedded order.  atol = rtol = 0 switches the control off (default);
 * ESRK_ENOTSUP for a method without an embedded pair, EINVAL for negative or
 * non-finite tolerances.  Resets the proposal: the next esrk_step with
 * dt <= 0 starts from the CFL rule again. */
esrk_status esrk_set_adaptive(esrk_ctx* ctx, double atol, double rtol);

/* The embedded pair's estimate of the last completed run of stages
 * (esrk_rk_stage or esrk_step): err (nullable, device [nv*N]) receives
 * dt sum_i (b_i - bhat_i) k_i, *norm (nullable, device scalar) the weighted
 * norm E of esrk_set_adaptive with the tolerances in effect at the last stage
 * (EINVAL if none are set).  ESRK_ENOTSUP for a method without an embedded
 * pair.  Enqueue only. */
esrk_status esrk_error_estimate(esrk_ctx* ctx, double* err, double* norm, void* stream);

/* Dirichlet boundaries for a 1-D Euler context (Sec. 4's shock tube, sine-shock
 * and local-gamma problems are posed on intervals): u_left and u_right (host,
 * 3 conserved values each) are the exterior states that enter the first and
 * last element's outer faces through the same interface flux as interior
 * faces.  Both NULL: periodic again (default).  ENOTSUP for dim != 1 or a
 * Navier-Stokes context, ENONPHYS for a state with rho <= 0 or p <= 0,
 * EINVAL for one NULL pointer or non-finite values.  Applies to the calls
 * that follow. */
esrk_status esrk_set_dirichlet(esrk_ctx* ctx, const double* u_left, const double* u_right);

/* Boundary kinds of the two ends of a 1-D Euler context (Sec. 4, 1-D
 * problems: the ends are imposed weakly through the interface flux, as the
 * paper imposes its boundary data by penalizing against a given state).
 * ESRK_BC_DIRICHLET: the end's exterior state is u_* (3 conserved values).
 * ESRK_BC_OUTFLOW: the exterior state is the end's own interior trace, so the
 * interface flux there is the trace's physical flux (u_* is ignored and may
 * be NULL).  esrk_set_dirichlet(ctx, l, r) is esrk_set_boundaries(ctx,
 * DIRICHLET, l, DIRICHLET, r); esrk_set_dirichlet(ctx, NULL, NULL) makes the
 * mesh periodic again.  ENOTSUP for dim != 1 or a Navier-Stokes context;
 * EINVAL for another kind, a NULL or non-finite Dirichlet state; ENONPHYS for
 * a Dirichlet state with rho <= 0 or p <= 0.  Nothing changes on an error.
 * Applies to the calls that follow. */
enum { ESRK_BC_DIRICHLET = 0, ESRK_BC_OUTFLOW = 1 };
esrk_status esrk_set_boundaries(esrk_ctx* ctx, int kind_left, const double* u_left,
                                int kind_right, const double* u_right);

/* Root-solve method of the local relaxation (Sec. 4 names Brent's method and
 * the first method of Alefeld, Potra and Shi as robust, secant and Newton as
 * slightly faster): ESRK_ROOT_ILLINOIS (default: regula falsi with the
 * Illinois modification), ESRK_ROOT_BRENT (Brent's inverse quadratic
 * interpolation / secant / bisection safeguards), ESRK_ROOT_ALEFELD (the
 * first method of Alefeld, Potra and Shi's enclosing algorithm: per iteration
 * an inverse cubic or Newton-quadratic point, a double-length secant point
 * and, when the bracket has not halved, its midpoint) or ESRK_ROOT_BISECTION.
 * Brent and Alefeld do not run with a network's first trial point, which
 * keeps the Illinois rule.  Every rule stops when the bracket is narrower
 * than tol max(1, gamma) and returns its lower end.  EINVAL for another
 * value. */
esrk_status esrk_set_root_method(esrk_ctx* ctx, int method);

/* Synchronizes `ctx`'s work on the stream of its last call, returns and clears
 * the latched device status; *bad_elem (nullable) receives the smallest
 * offending element index or -1. */
esrk_status esrk_sync_status(esrk_ctx* ctx, int64_t* bad_elem);

const char* esrk_status_str(esrk_status s);

/* ---- Batches of independent simulations ----------------------------------
 * Many periodic 2-D meshes of different sizes that share degree, physics,
 * precision and Runge-Kutta method, advanced together: each stage is one
 * kernel launch over a work list covering every simulation; each simulation
 * keeps its own CFL step, its own gamma = min over its elements (Sec. 2,
 * local relaxation theorem, applied per simulation) and its own time.
 * State layout: one packed device array; simulation s occupies
 * [esrk_batch_offset(b, s), + (dim+2) * N_s) in the single-mesh layout.
 * Per-element arrays are packed the same way (esrk_batch_elem_offset). */
typedef struct esrk_batch esrk_batch;

/* cfgs[0..nsims): 2-D only (ESRK_ENOTSUP otherwise), Euler (mu = 0); dim,
 * deg, precision, tableau, gas_gamma and lambda_scale must agree (EINVAL);
 * nel, lo, hi and cfl may differ; each simulation's state must stay below
 * 2^31 entries (32-bit indexing).  Allocates all workspace. */
esrk_status esrk_batch_create(const esrk_config* cfgs, int nsims, esrk_batch** out);
void esrk_batch_destroy(esrk_batch* b);
int esrk_batch_num_sims(const esrk_batch* b);
size_t esrk_batch_state_len(const esrk_batch* b);  /* doubles of the packed state */
size_t esrk_batch_num_elems(const esrk_batch* b);
size_t esrk_batch_offset(const esrk_batch* b, int sim);
size_t esrk_batch_elem_offset(const esrk_batch* b, int sim);
int esrk_batch_tile(const esrk_batch* b);  /* elements per block of the stage kernel */

/* One locally relaxed step of every simulation, in place, with each
 * simulation's CFL step.  t: device [nsims] (inout); gamma: device [nsims]
 * (nullable, out).  No host synchronization, no allocation. */
esrk_status esrk_batch_step(esrk_batch* b, double* u, double* t, double* gamma, void* stream);

/* Times every compiled tile (elements per block) of the stage kernel on the
 * state u (read only; workspace is overwritten), keeps the fastest and
 * returns it in *tile_out (nullable).  Synchronizes the stream. */
esrk_status esrk_batch_autotune(esrk_batch* b, const double* u, int reps, int* tile_out,
                                void* stream);

/* nsteps batch steps captured once into a hipGraph (re-captured when u, t,
 * gamma, nsteps, the tile or the stream change) and replayed on `stream`,
 * which must not be the NULL stream. */
esrk_status esrk_batch_run_graph(esrk_batch* b, double* u, double* t, double* gamma, int nsteps,
                                 void* stream);

esrk_status esrk_batch_sync_status(esrk_batch* b, int64_t* bad_elem);

/* ---- Learned first trial point of the relaxation solve --------------------
 * A 5 -> 32 -> 32 -> 1 tanh network (FP32) maps element features to a trial
 * relaxation parameter; the root solve of esrk_local_relaxation_solve always
 * runs to root_tol afterwards, so the result does not depend on the network
 * beyond root_tol (Sec. 2 only prescribes solving the scalar equation).
 * Model vector (float, device, ESRK_MLP_MODEL entries):
 *   W1[32][5] @0, b1[32] @160, W2[32][32] @192, b2[32] @1216, w3[32] @1248,
 *   b3 @1280 (ESRK_MLP_TRAINED trained parameters); input normalization
 *   scale[5] @1281, mean[5] @1286, std[5] @1291; output out_mean @1296,
 *   out_std @1297.
 * Raw features of element k: r = [deta_k, eta_k(u_new) - eta_k(u_old), dt,
 *   max_i sum_m (|v_m| + c), dt * viscous dissipation rate of k];
 * network input x_j = (asinh(r_j / scale_j) - mean_j) / std_j;
 * trial point 1 + dt^2 (out_mean + out_std * y). */
#define ESRK_MLP_TRAINED 1281
#define ESRK_MLP_MODEL 1298

/* esrk_local_relaxation_solve with the learned first trial point (model,
 * nullable) and the raw features written to feats (nullable, float
 * [num_elems][5]) for training.  visc_rate (nullable, [num_elems]): the
 * element viscous dissipation rate used as the fifth feature. */
esrk_status esrk_local_relaxation_solve_ml(esrk_ctx* ctx, const double* u_old,
                                           const double* du, const double* deta, double dt,
                                           const double* visc_rate, const float* model,
                                           float* feats, double* gamma_k, double* gamma,
                                           int32_t* iters, void* stream);

/* Model used by esrk_step for the first trial point (NULL: none) and a
 * device buffer (nullable, float [num_elems][5]) that every following
 * esrk_step fills with the raw features of its elements.  Both pointers are
 * kept; the caller keeps them alive while they are set. */
esrk_status esrk_set_step_model(esrk_ctx* ctx, const float* model, float* feats_out);

/* Normalization of B logged samples for training: raw (float [B][5], raw
 * features as above), gamma (nullable, double [B], their solved relaxation
 * parameters; inactive elements must be left out).  fit != 0 first sets the
 * model's normalization entries from the samples: scale_j = mean |r_j|,
 * mean_j / std_j of asinh(r_j / scale_j), out_mean / out_std of
 * q = (gamma - 1) / dt^2.  Then x_norm[B][5] (network inputs) and, with gamma,
 * t_norm[B] = (q - out_mean) / out_std are written.  One workgroup. */
esrk_status esrk_mlp_prepare(float* model, const float* raw, const double* gamma, int B, int fit,
                             float* x_norm, float* t_norm, void* stream);

/* Network on normalized inputs: y[b] = net(x_norm[b][0..5)), B samples. */
esrk_status esrk_mlp_forward(const float* model, const float* x_norm, int B, float* y,
                             void* stream);
/* Device workspace (number of floats) that esrk_mlp_grad needs for B samples. */
size_t esrk_mlp_grad_work_size(int B);
/* grad[ESRK_MLP_TRAINED] of L = (1/B) sum_b (net(x_b) - t_b)^2 and L (loss,
 * nullable, device scalar).  work: device buffer of esrk_mlp_grad_work_size(B)
 * floats (per-block partial gradients, summed in block order afterwards, so
 * the result is deterministic). */
esrk_status esrk_mlp_grad(const float* model, const float* x_norm, const float* t_norm, int B,
                          float* grad, float* loss, float* work, void* stream);
/* One Adam update (beta1 0.9, beta2 0.999, eps 1e-8) of the trained
 * parameters; m, v: device moment vectors (zero before step 1). */
esrk_status esrk_mlp_adam(float* model, const float* grad, float* m, float* v, int step,
                          float lr, void* stream);

#ifdef __cplusplus
}
#endif
#endif
