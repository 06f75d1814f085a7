// Host side of the C-ABI (include/esrk.h): context, workspace and the
// enqueue-only entry points.  Every step of the path runs in the HIP kernels
// of rhs.hip and relax.hip; this file only validates, sizes and launches.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "internal.h"

using esrk::DevScalars;
using esrk::MeshParams;
using esrk::StageCoef;

struct esrk_ctx {
  esrk_config cfg;
  MeshParams mp;
  int stages;
  StageCoef sc[esrk::kMaxStages];
  esrk::StageRow rows[esrk::kMaxStages];
  int order_emb = 0;        // embedded order q (0: no embedded method)
  int nslots = 0;           // stored slopes of a general tableau
  bool skip_last = false;   // last stage only feeds the error estimate
  double* kst = nullptr;    // slope store (nslots x nv x N)
  double* err = nullptr;    // embedded pairs: error estimate (nv x N)
  double* errk = nullptr;   // embedded pairs: per-element squared weighted errors
  double* phi0acc = nullptr;  // phi_k(0) accumulated by the stages
  // per-stage extras of the embedded pairs in device memory:
  // [0][stage] rows and slope store only, [1][stage] with the error estimate
  esrk::StageExtra* ex_dev = nullptr;
  double atol = 0.0, rtol = 0.0;  // error control (both 0: off)
  bool have_dt_next = false;      // a proposal from the last controlled attempt exists
  size_t N, ne;
  int nv;
  double* ya = nullptr;
  double* yb = nullptr;
  double* du = nullptr;
  double* deta = nullptr;
  double* gamma_k = nullptr;
  int32_t* iters = nullptr;
  double* speed_parts = nullptr;
  void* theta = nullptr;      // Navier-Stokes: viscous fluxes g_m (dim x nv x N, T precision)
  double* visc = nullptr;     // Navier-Stokes: viscous right-hand side
  double* vdiss = nullptr;    // Navier-Stokes: per-element viscous dissipation
  esrk::RelaxPart* relax_parts = nullptr;
  int n_relax_parts = 0;
  DevScalars* scal = nullptr;
  const float* step_model = nullptr;  // network used by esrk_step for first trial points
  float* step_feats = nullptr;        // raw features written by esrk_step (nullable)
  int relax_mode = ESRK_RELAX_LOCAL;  // relaxation used by esrk_step
  int root_method = ESRK_ROOT_ILLINOIS;
  double* glob_parts = nullptr;       // global relaxation: block partials
  esrk::GlobState* glob_state = nullptr;  // global relaxation: bracket and result
  hipStream_t last = nullptr;
  // whole steps captured by esrk_run_graph, valid while the pointers, the step
  // count, the stream and the settings generation match
  unsigned gen = 0;  // bumped by every setter that changes what a step enqueues
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double *g_u = nullptr, *g_t = nullptr, *g_stats = nullptr;
  int g_steps = 0;
  unsigned g_gen = 0;
  hipStream_t g_stream = nullptr;
};

namespace {

// Embedded pairs in Butcher form (A strictly lower triangular, weights b of
// the propagated solution, bhat of the embedded one), the published
// Bogacki-Shampine 3(2) and 5(4) methods.  Both evaluate their last stage at
// the propagated solution with weight zero (b_s = 0).
struct Pair {
  int s, q;
  double A[esrk::kMaxStages][esrk::kMaxStages];
  double b[esrk::kMaxStages], bh[esrk::kMaxStages];
};

bool pair_of(int which, Pair* P) {
  std::memset(P, 0, sizeof(*P));
  if (which == ESRK_BSRK43) {
    P->s = 4;
    P->q = 2;
    const double a[4][3] = {{0, 0, 0}, {1.0 / 2, 0, 0}, {0, 3.0 / 4, 0},
                            {2.0 / 9, 1.0 / 3, 4.0 / 9}};
    const double bh[4] = {7.0 / 24, 1.0 / 4, 1.0 / 3, 1.0 / 8};
    for (int i = 0; i < 4; ++i) {
      for (int j = 0; j < i; ++j) P->A[i][j] = a[i][j];
      P->bh[i] = bh[i];
    }
    for (int j = 0; j < 3; ++j) P->b[j] = a[3][j];
    return true;
  }
  if (which == ESRK_BSRK85) {
    P->s = 8;
    P->q = 4;
    const double a[8][7] = {
        {0, 0, 0, 0, 0, 0, 0},
        {1.0 / 6, 0, 0, 0, 0, 0, 0},
        {2.0 / 27, 4.0 / 27, 0, 0, 0, 0, 0},
        {183.0 / 1372, -162.0 / 343, 1053.0 / 1372, 0, 0, 0, 0},
        {68.0 / 297, -4.0 / 11, 42.0 / 143, 1960.0 / 3861, 0, 0, 0},
        {597.0 / 22528, 81.0 / 352, 63099.0 / 585728, 58653.0 / 366080, 4617.0 / 20480, 0, 0},
        {174197.0 / 959244, -30942.0 / 79937, 8152137.0 / 19744439, 666106.0 / 1039181,
         -29421.0 / 29068, 482048.0 / 414219, 0},
        {587.0 / 8064, 0, 4440339.0 / 15491840, 24353.0 / 124800, 387.0 / 44800,
         2152.0 / 5985, 7267.0 / 94080}};
    const double bh[8] = {2479.0 / 34992,    0,
                          123.0 / 416,       612941.0 / 3411720,
                          43.0 / 1440,       2272.0 / 6561,
                          79937.0 / 1113912, 3293.0 / 556956};
    for (int i = 0; i < 8; ++i) {
      for (int j = 0; j < i; ++j) P->A[i][j] = a[i][j];
      P->bh[i] = bh[i];
    }
    for (int j = 0; j < 7; ++j) P->b[j] = a[7][j];
    return true;
  }
  return false;
}

// A Butcher tableau in the device's stage form: stage i writes
//   y_{i+1} = u_old + dt (a_{i+1,i} k_i + sum_{j<i} a_{i+1,j} k_j)
// with the k_j read back from the slope store; only slopes that a later row
// (beyond the next stage) uses are stored.  Returns the number of slots.
int pair_rows(const Pair& P, StageCoef* sc, esrk::StageRow* rows) {
  int slot_of[esrk::kMaxStages];
  int nslots = 0;
  for (int i = 0; i < P.s; ++i) {
    bool later = false;
    for (int m = i + 2; m < P.s; ++m) later = later || P.A[m][i] != 0.0;
    slot_of[i] = later ? nslots++ : -1;
  }
  for (int i = 0; i < P.s; ++i) {
    esrk::StageRow& R = rows[i];
    std::memset(&R, 0, sizeof(R));
    R.kstore = slot_of[i] + 1;
    R.ecoef = P.b[i] - P.bh[i];
    const bool has_next = i + 1 < P.s;
    sc[i] = {has_next ? 1.0 : 0.0, 0.0, has_next ? P.A[i + 1][i] : 0.0, P.b[i]};
    if (has_next)
      for (int j = 0; j < i; ++j)
        if (P.A[i + 1][j] != 0.0) {
          R.prev_slot[R.nprev] = slot_of[j];
          R.prev_a[R.nprev] = P.A[i + 1][j];
          ++R.nprev;
        }
  }
  return nslots;
}

// Runge-Kutta methods in the device's two-register form
//   y_{i+1} = alpha u_old + beta y_i + c dt k_i,  du += b dt k_i.
// SSPRK(3,3): y2 = u + dt k1, y3 = 3/4 u + 1/4 y2 + 1/4 dt k2, b = (1/6, 1/6, 2/3).
// RK(4,4): y_{i+1} = u + c_{i+1} dt k_i with c = (1/2, 1/2, 1), b = (1/6, 1/3, 1/3, 1/6).
int tableau_coefs(int which, StageCoef* sc) {
  if (which == ESRK_SSPRK33) {
    sc[0] = {1.0, 0.0, 1.0, 1.0 / 6.0};
    sc[1] = {0.75, 0.25, 0.25, 1.0 / 6.0};
    sc[2] = {0.0, 0.0, 0.0, 2.0 / 3.0};
    return 3;
  }
  if (which == ESRK_RK44) {
    sc[0] = {1.0, 0.0, 0.5, 1.0 / 6.0};
    sc[1] = {1.0, 0.0, 0.5, 1.0 / 3.0};
    sc[2] = {1.0, 0.0, 1.0, 1.0 / 3.0};
    sc[3] = {0.0, 0.0, 0.0, 1.0 / 6.0};
    return 4;
  }
  return 0;
}

esrk_status hip_status(hipError_t e) { return e == hipSuccess ? ESRK_OK : ESRK_EHIP; }

esrk::RhsArgs base_args(esrk_ctx* c) {
  esrk::RhsArgs a;
  std::memset(&a, 0, sizeof(a));
  a.scal = c->scal;
  a.dt_store = &c->scal->dt;
  a.n_speed_parts = esrk::kSpeedBlocks;
  return a;
}

// Navier-Stokes viscous right-hand side of state y into ctx->visc (no-op for Euler).
hipError_t viscous(esrk_ctx* x, const double* y, double* diss, hipStream_t s) {
  if (!(x->cfg.mu > 0.0)) return hipSuccess;
  esrk::NsArgs n;
  n.y = y;
  n.flux = x->theta;
  n.visc = x->visc;
  n.diss = diss;
  n.mu = x->cfg.mu;
  n.R = x->cfg.gas_r;
  n.kappa = x->cfg.mu * (x->cfg.gas_gamma * x->cfg.gas_r / (x->cfg.gas_gamma - 1.0)) /
            x->cfg.prandtl;
  return esrk::launch_ns(x->mp, x->cfg.precision, n, s);
}

// Uploads the per-stage extras (rows, slope store; error estimate in the
// second set, with the per-element error sums on the last stage when
// tolerances are set).  Synchronous.
hipError_t upload_extras(esrk_ctx* x) {
  if (x->order_emb == 0) return hipSuccess;
  esrk::StageExtra h[2][esrk::kMaxStages];
  std::memset(h, 0, sizeof(h));
  const bool tol = x->atol > 0.0 || x->rtol > 0.0;
  for (int v = 0; v < 2; ++v)
    for (int i = 0; i < x->stages; ++i) {
      esrk::StageExtra& E = h[v][i];
      E.row = x->rows[i];
      E.kst = x->kst;
      if (v == 1) {
        E.err = x->err;
        if (i == x->stages - 1 && tol) {
          E.errk = x->errk;
          E.atol = x->atol;
          E.rtol = x->rtol;
        }
      }
    }
  return hipMemcpy(x->ex_dev, h, sizeof(h), hipMemcpyHostToDevice);
}

// The general-tableau and error-estimate part of a stage's arguments
// (with_err: accumulate the embedded pair's estimate).
void stage_extras(const esrk_ctx* x, int stage, bool with_err, esrk::RhsArgs& a) {
  a.phi0 = x->phi0acc;
  a.ex = x->ex_dev ? x->ex_dev + (with_err ? esrk::kMaxStages : 0) + stage : nullptr;
}

// Sweeps of the device-driven global relaxation solve (a converged solve
// makes the remaining sweeps return at once).
constexpr int kGlobMaxPasses = 12;

}  // namespace

extern "C" {

const char* esrk_status_str(esrk_status s) {
  switch (s) {
    case ESRK_OK: return "ok";
    case ESRK_EINVAL: return "invalid argument";
    case ESRK_EHIP: return "HIP runtime error";
    case ESRK_ENOMEM: return "out of device memory";
    case ESRK_ENOROOT: return "no positive relaxation root in an active element";
    case ESRK_ENONPHYS: return "non-physical state (rho <= 0 or p <= 0)";
    case ESRK_ENAN: return "NaN produced";
    case ESRK_ENOTSUP: return "configuration not supported";
  }
  return "unknown status";
}

esrk_status esrk_create(const esrk_config* cfg, esrk_ctx** out) {
  if (!cfg || !out) return ESRK_EINVAL;
  *out = nullptr;
  const esrk_config& c = *cfg;
  if (c.dim < 1 || c.dim > 3 || c.deg < 1 || c.deg > esrk::kMaxN - 1) return ESRK_EINVAL;
  if (!(c.gas_gamma > 1.0) || !(c.gas_r > 0.0) || c.mu < 0.0) return ESRK_EINVAL;
  if (c.precision != ESRK_FP64 && c.precision != ESRK_FP32_FLUX) return ESRK_EINVAL;
  if (c.tableau != ESRK_SSPRK33 && c.tableau != ESRK_RK44 && c.tableau != ESRK_BSRK43 &&
      c.tableau != ESRK_BSRK85)
    return ESRK_ENOTSUP;
  if (c.mu > 0.0 && !(c.prandtl > 0.0)) return ESRK_EINVAL;
  size_t ne = 1;
  for (int m = 0; m < c.dim; ++m) {
    if (c.nel[m] < 1 || !(c.hi[m] > c.lo[m])) return ESRK_EINVAL;
    ne *= (size_t)c.nel[m];
  }
  // the kernels index a state array (nv fields of ne * (deg+1)^dim nodes) in 32 bits
  size_t nd = 1;
  for (int m = 0; m < c.dim; ++m) nd *= (size_t)(c.deg + 1);
  if (ne * nd * (size_t)(c.dim + 2) > (size_t)INT32_MAX) return ESRK_EINVAL;
  esrk_ctx* x = new (std::nothrow) esrk_ctx();
  if (!x) return ESRK_ENOMEM;
  x->cfg = c;
  if (!(x->cfg.root_tol > 0.0)) x->cfg.root_tol = 1e-12;
  if (x->cfg.root_maxit <= 0) x->cfg.root_maxit = 60;
  if (!(x->cfg.gamma_max > 1.0)) x->cfg.gamma_max = 4.0;
  if (!(x->cfg.cfl > 0.0)) x->cfg.cfl = 0.5;
  MeshParams& mp = x->mp;
  std::memset(&mp, 0, sizeof(mp));
  mp.dim = c.dim;
  mp.n = c.deg + 1;
  mp.nd = 1;
  for (int m = 0; m < c.dim; ++m) mp.nd *= mp.n;
  mp.ne = (int)ne;
  double hmin = INFINITY;
  for (int m = 0; m < 3; ++m) {
    mp.nel[m] = m < c.dim ? c.nel[m] : 1;
    const double h = m < c.dim ? (c.hi[m] - c.lo[m]) / c.nel[m] : 1.0;
    mp.two_over_h[m] = 2.0 / h;
    mp.half_h[m] = 0.5 * h;
    if (m < c.dim) hmin = std::fmin(hmin, h);
  }
  double xs[esrk::kMaxN], D[esrk::kMaxN * esrk::kMaxN];
  esrk::lobatto_tables(c.deg, xs, mp.w, D);
  for (int i = 0; i < mp.n * mp.n; ++i) mp.D2[i] = 2.0 * D[i];
  mp.inv_w_end = 1.0 / mp.w[0];
  mp.gg = c.gas_gamma;
  mp.lambda_scale = c.lambda_scale;
  mp.cfl = x->cfg.cfl;
  mp.hmin = hmin;
  for (int i = 0; i < esrk::kMaxStages; ++i) std::memset(&x->rows[i], 0, sizeof(x->rows[i]));
  Pair P;
  if (pair_of(c.tableau, &P)) {
    x->stages = P.s;
    x->order_emb = P.q;
    x->nslots = pair_rows(P, x->sc, x->rows);
    x->skip_last = P.b[P.s - 1] == 0.0;
  } else {
    x->stages = tableau_coefs(c.tableau, x->sc);
  }
  x->ne = ne;
  x->N = ne * (size_t)mp.nd;
  x->nv = c.dim + 2;
  const size_t len = x->N * (size_t)x->nv;
  bool ok = hipMalloc(&x->ya, len * sizeof(double)) == hipSuccess &&
            hipMalloc(&x->yb, len * sizeof(double)) == hipSuccess &&
            hipMalloc(&x->du, len * sizeof(double)) == hipSuccess &&
            hipMalloc(&x->deta, ne * sizeof(double)) == hipSuccess &&
            hipMalloc(&x->phi0acc, ne * sizeof(double)) == hipSuccess &&
            hipMalloc(&x->gamma_k, ne * sizeof(double)) == hipSuccess &&
            hipMalloc(&x->iters, ne * sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&x->speed_parts, esrk::kSpeedBlocks * sizeof(double)) == hipSuccess &&
            hipMalloc(&x->scal, sizeof(DevScalars)) == hipSuccess;
  if (c.mu > 0.0) {
    const size_t tsz = c.precision == ESRK_FP64 ? sizeof(double) : sizeof(float);
    ok = ok && hipMalloc(&x->theta, (size_t)c.dim * len * tsz) == hipSuccess &&
         hipMalloc(&x->visc, len * sizeof(double)) == hipSuccess &&
         hipMalloc(&x->vdiss, ne * sizeof(double)) == hipSuccess;
  }
  x->n_relax_parts = esrk::relax_blocks(mp);
  ok = ok && hipMalloc(&x->relax_parts, x->n_relax_parts * sizeof(esrk::RelaxPart)) == hipSuccess;
  ok = ok &&
       hipMalloc(&x->glob_parts, (size_t)esrk::glob_blocks(mp) * esrk::kGlobParts *
                                     sizeof(double)) == hipSuccess &&
       hipMalloc(&x->glob_state, sizeof(esrk::GlobState)) == hipSuccess;
  if (x->nslots > 0)
    ok = ok && hipMalloc(&x->kst, (size_t)x->nslots * len * sizeof(double)) == hipSuccess;
  if (x->order_emb > 0)
    ok = ok && hipMalloc(&x->err, len * sizeof(double)) == hipSuccess &&
         hipMalloc(&x->errk, ne * sizeof(double)) == hipSuccess &&
         hipMalloc(&x->ex_dev, 2 * esrk::kMaxStages * sizeof(esrk::StageExtra)) == hipSuccess;
  if (!ok) {
    esrk_destroy(x);
    return ESRK_ENOMEM;
  }
  DevScalars init;
  std::memset(&init, 0, sizeof(init));
  init.bad_elem = INT64_MAX;
  init.gamma = 1.0;
  if (hipMemcpy(x->scal, &init, sizeof(init), hipMemcpyHostToDevice) != hipSuccess ||
      upload_extras(x) != hipSuccess) {
    esrk_destroy(x);
    return ESRK_EHIP;
  }
  *out = x;
  return ESRK_OK;
}

static void drop_graph(esrk_ctx* x) {
  if (x->gexec) (void)hipGraphExecDestroy(x->gexec);
  if (x->graph) (void)hipGraphDestroy(x->graph);
  x->gexec = nullptr;
  x->graph = nullptr;
}

void esrk_destroy(esrk_ctx* x) {
  if (!x) return;
  drop_graph(x);
  (void)hipFree(x->ya);
  (void)hipFree(x->yb);
  (void)hipFree(x->du);
  (void)hipFree(x->deta);
  (void)hipFree(x->gamma_k);
  (void)hipFree(x->iters);
  (void)hipFree(x->speed_parts);
  (void)hipFree(x->theta);
  (void)hipFree(x->visc);
  (void)hipFree(x->vdiss);
  (void)hipFree(x->relax_parts);
  (void)hipFree(x->glob_parts);
  (void)hipFree(x->glob_state);
  (void)hipFree(x->kst);
  (void)hipFree(x->err);
  (void)hipFree(x->errk);
  (void)hipFree(x->phi0acc);
  (void)hipFree(x->ex_dev);
  (void)hipFree(x->scal);
  delete x;
}

size_t esrk_num_nodes(const esrk_ctx* x) { return x ? x->N : 0; }
size_t esrk_num_elems(const esrk_ctx* x) { return x ? x->ne : 0; }
int esrk_num_vars(const esrk_ctx* x) { return x ? x->nv : 0; }

esrk_status esrk_rhs_euler(esrk_ctx* x, const double* u, double* dudt, double* eta_rate,
                           void* stream) {
  if (!x || !u || !dudt || (const double*)dudt == u) return ESRK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  x->last = s;
  esrk::RhsArgs a = base_args(x);
  a.y = u;
  a.out = dudt;
  a.eta = eta_rate;
  a.stage_mode = 0;
  return hip_status(esrk::launch_rhs(x->mp, x->cfg.precision, a, s));
}

esrk_status esrk_rhs_ns(esrk_ctx* x, const double* u, double* dudt, double* eta_rate,
                        double* visc_diss, void* stream) {
  if (!x || !u || !dudt || (const double*)dudt == u) return ESRK_EINVAL;
  if (!(x->cfg.mu > 0.0)) return ESRK_EINVAL;  // Euler contexts use esrk_rhs_euler
  hipStream_t s = (hipStream_t)stream;
  x->last = s;
  hipError_t e = viscous(x, u, visc_diss, s);
  if (e != hipSuccess) return ESRK_EHIP;
  esrk::RhsArgs a = base_args(x);
  a.y = u;
  a.out = dudt;
  a.eta = eta_rate;
  a.visc = x->visc;
  a.stage_mode = 0;
  return hip_status(esrk::launch_rhs(x->mp, x->cfg.precision, a, s));
}

esrk_status esrk_rk_stage(esrk_ctx* x, int stage, double dt, const double* u_old,
                          const double* y_in, double* y_out, double* du, double* deta,
                          void* stream) {
  if (!x || stage < 0 || stage >= x->stages || !u_old || !y_in || !du || !(dt > 0.0))
    return ESRK_EINVAL;
  const bool last = stage == x->stages - 1;
  if (!last && !y_out) return ESRK_EINVAL;
  if (y_out && ((const double*)y_out == y_in || (const double*)y_out == u_old))
    return ESRK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  x->last = s;
  if (viscous(x, y_in, nullptr, s) != hipSuccess) return ESRK_EHIP;
  esrk::RhsArgs a = base_args(x);
  a.visc = x->cfg.mu > 0.0 ? x->visc : nullptr;
  a.y = y_in;
  a.u_old = u_old;
  a.out = last ? nullptr : y_out;
  a.du = du;
  a.eta = deta;
  a.dt_dev = nullptr;
  a.dt_host = dt;
  a.sc = x->sc[stage];
  a.stage_mode = 1;
  a.first = stage == 0;
  stage_extras(x, stage, true, a);
  return hip_status(esrk::launch_rhs(x->mp, x->cfg.precision, a, s));
}

static esrk::RelaxArgs relax_args(esrk_ctx* x, const double* u_old, const double* du,
                                  const double* deta, const float* guess, double* gk,
                                  int32_t* iters) {
  esrk::RelaxArgs r;
  std::memset(&r, 0, sizeof(r));
  r.u_old = u_old;
  r.du = du;
  r.deta = deta;
  r.guess = guess;
  r.gamma_k = gk;
  r.iters = iters;
  r.parts = x->relax_parts;
  r.scal = x->scal;
  r.tol = x->cfg.root_tol;
  r.gamma_max = x->cfg.gamma_max;
  r.maxit = x->cfg.root_maxit;
  r.method = x->root_method;
  r.fp32_increments = x->cfg.precision == ESRK_FP32_FLUX;
  return r;
}

esrk_status esrk_local_relaxation_solve(esrk_ctx* x, const double* u_old, const double* du,
                                        const double* deta, const float* gamma_guess,
                                        double* gamma_k, double* gamma, int32_t* iters,
                                        void* stream) {
  if (!x || !u_old || !du || !deta || !gamma_k || !gamma) return ESRK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  x->last = s;
  hipError_t e = esrk::launch_relax(
      x->mp, relax_args(x, u_old, du, deta, gamma_guess, gamma_k, iters), s);
  if (e == hipSuccess)
    e = esrk::launch_relax_finish(x->relax_parts, x->n_relax_parts, x->scal, gamma, s);
  return hip_status(e);
}

esrk_status esrk_local_relaxation_solve_phi0(esrk_ctx* x, const double* u_old,
                                             const double* du, const double* deta,
                                             const double* phi0, double* gamma_k,
                                             double* gamma, int32_t* iters, void* stream) {
  if (!x || !u_old || !du || !deta || !phi0 || !gamma_k || !gamma) return ESRK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  x->last = s;
  esrk::RelaxArgs r = relax_args(x, u_old, du, deta, nullptr, gamma_k, iters);
  r.phi0_in = phi0;
  hipError_t e = esrk::launch_relax(x->mp, r, s);
  if (e == hipSuccess)
    e = esrk::launch_relax_finish(x->relax_parts, x->n_relax_parts, x->scal, gamma, s);
  return hip_status(e);
}

esrk_status esrk_stage_phi0(esrk_ctx* x, double* phi0, void* stream) {
  if (!x || !phi0) return ESRK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  x->last = s;
  return hip_status(
      hipMemcpyAsync(phi0, x->phi0acc, x->ne * sizeof(double), hipMemcpyDeviceToDevice, s));
}

esrk_status esrk_step(esrk_ctx* x, double* u, double* t, double dt, double* gamma_k_out,
                      double* stats_out, void* stream) {
  if (!x || !u || !t) return ESRK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  x->last = s;
  const bool adaptive = x->order_emb > 0 && (x->atol > 0.0 || x->rtol > 0.0);
  // the controller's proposal replaces the CFL rule once there is one
  const bool proposal = adaptive && !(dt > 0.0) && x->have_dt_next;
  const bool cfl = !(dt > 0.0) && !proposal;
  hipError_t e = hipSuccess;
  if (cfl) e = esrk::launch_speed(x->mp, u, x->speed_parts, s);
  const double* yin = u;
  double* bufs[2] = {x->ya, x->yb};
  // without error control a last stage of weight zero feeds nothing
  const int nst = (!adaptive && x->skip_last) ? x->stages - 1 : x->stages;
  for (int i = 0; i < nst && e == hipSuccess; ++i) {
    const bool last = i == nst - 1;
    e = viscous(x, yin, x->vdiss, s);
    if (e != hipSuccess) break;
    esrk::RhsArgs a = base_args(x);
    a.visc = x->cfg.mu > 0.0 ? x->visc : nullptr;
    a.y = yin;
    a.u_old = u;
    a.out = last ? nullptr : bufs[i & 1];
    a.du = x->du;
    // the solves take phi_k(0) from the stages, so the estimate's increment
    // itself is needed only for the network's features
    a.eta = x->step_model ? x->deta : nullptr;
    if (i == 0) {
      a.speed_parts = cfl ? x->speed_parts : nullptr;
      a.dt_dev = proposal ? &x->scal->dt_next : nullptr;
      a.dt_host = dt;
    } else {
      a.dt_dev = &x->scal->dt;
    }
    a.sc = x->sc[i];
    a.stage_mode = 1;
    a.first = i == 0;
    stage_extras(x, i, adaptive, a);
    if (x->relax_mode == ESRK_RELAX_NONE) a.phi0 = nullptr;  // nothing to solve
    e = esrk::launch_rhs(x->mp, x->cfg.precision, a, s);
    yin = bufs[i & 1];
  }
  if (e == hipSuccess && adaptive) {
    e = esrk::launch_adapt(x->errk, (int)x->ne, (double)(x->N * x->nv), x->order_emb, 1,
                           x->scal, nullptr, s);
    x->have_dt_next = true;
  }
  if (e != hipSuccess) return hip_status(e);
  int nparts = x->n_relax_parts;
  if (x->relax_mode == ESRK_RELAX_LOCAL) {
    double* gk = gamma_k_out ? gamma_k_out : x->gamma_k;
    esrk::RelaxArgs r =
        relax_args(x, u, x->du, x->step_model ? x->deta : nullptr, nullptr, gk, x->iters);
    r.model = x->step_model;
    r.feats = x->step_feats;
    r.dt_dev = &x->scal->dt;
    r.vfeat = x->cfg.mu > 0.0 ? x->vdiss : nullptr;
    r.check_reject = adaptive ? 1 : 0;
    r.phi0_in = x->phi0acc;
    e = esrk::launch_relax(x->mp, r, s);
  } else if (x->relax_mode == ESRK_RELAX_GLOBAL) {
    e = esrk::launch_glob_solve(x->mp, u, x->du, nullptr, x->phi0acc, x->glob_state,
                                x->glob_parts, x->relax_parts, x->scal, 1, adaptive ? 1 : 0,
                                x->cfg.root_tol, x->cfg.gamma_max, kGlobMaxPasses, s);
    nparts = 1;
  } else {
    e = esrk::launch_set_part(x->relax_parts, INFINITY, s);  // the update takes gamma = 1
    nparts = 1;
  }
  if (e == hipSuccess)
    e = esrk::launch_apply(x->mp, u, x->du, t, x->relax_parts, nparts, x->scal, &x->scal->dt,
                           stats_out, adaptive ? 1 : 0, s);
  return hip_status(e);
}

esrk_status esrk_run_graph(esrk_ctx* x, double* u, double* t, int nsteps, double* stats_out,
                           void* stream) {
  if (!x || !u || !t || nsteps < 1 || !stream) return ESRK_EINVAL;
  // an error-controlled step takes its step size from host-side controller
  // state, which a recorded graph cannot follow
  if (x->order_emb > 0 && (x->atol > 0.0 || x->rtol > 0.0)) return ESRK_ENOTSUP;
  hipStream_t s = (hipStream_t)stream;
  if (!(x->gexec && x->g_u == u && x->g_t == t && x->g_stats == stats_out &&
        x->g_steps == nsteps && x->g_stream == s && x->g_gen == x->gen)) {
    drop_graph(x);
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return ESRK_EHIP;
    esrk_status st = ESRK_OK;
    for (int i = 0; i < nsteps && st == ESRK_OK; ++i)
      st = esrk_step(x, u, t, 0.0, nullptr, stats_out, stream);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &g);
    if (st != ESRK_OK || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return st != ESRK_OK ? st : ESRK_EHIP;
    }
    if (hipGraphInstantiate(&x->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      x->gexec = nullptr;
      return ESRK_EHIP;
    }
    x->graph = g;
    x->g_u = u;
    x->g_t = t;
    x->g_stats = stats_out;
    x->g_steps = nsteps;
    x->g_stream = s;
    x->g_gen = x->gen;
  }
  x->last = s;
  return hipGraphLaunch(x->gexec, s) == hipSuccess ? ESRK_OK : ESRK_EHIP;
}

esrk_status esrk_set_adaptive(esrk_ctx* x, double atol, double rtol) {
  if (!x || !(atol >= 0.0) || !(rtol >= 0.0) || std::isinf(atol) || std::isinf(rtol))
    return ESRK_EINVAL;
  if ((atol > 0.0 || rtol > 0.0) && x->order_emb == 0) return ESRK_ENOTSUP;
  x->atol = atol;
  x->rtol = rtol;
  x->have_dt_next = false;
  ++x->gen;
  return hip_status(upload_extras(x));
}

esrk_status esrk_error_estimate(esrk_ctx* x, double* err, double* norm, void* stream) {
  if (!x) return ESRK_EINVAL;
  if (x->order_emb == 0) return ESRK_ENOTSUP;
  if (norm && !(x->atol > 0.0 || x->rtol > 0.0)) return ESRK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  x->last = s;
  hipError_t e = hipSuccess;
  if (err)
    e = hipMemcpyAsync(err, x->err, x->N * x->nv * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && norm)
    e = esrk::launch_adapt(x->errk, (int)x->ne, (double)(x->N * x->nv), x->order_emb, 0,
                           x->scal, norm, s);
  return hip_status(e);
}

esrk_status esrk_set_boundaries(esrk_ctx* x, int kind_left, const double* u_left,
                                int kind_right, const double* u_right) {
  if (!x) return ESRK_EINVAL;
  if (x->cfg.dim != 1 || x->cfg.mu > 0.0) return ESRK_ENOTSUP;
  const int kind[2] = {kind_left, kind_right};
  const double* ext[2] = {u_left, u_right};
  double ubc[2][5] = {};
  const double g1 = x->cfg.gas_gamma - 1.0;
  // validate both ends before changing anything
  for (int s = 0; s < 2; ++s) {
    if (kind[s] == ESRK_BC_OUTFLOW) continue;
    if (kind[s] != ESRK_BC_DIRICHLET || !ext[s]) return ESRK_EINVAL;
    for (int v = 0; v < 3; ++v) {
      if (!std::isfinite(ext[s][v])) return ESRK_EINVAL;
      ubc[s][v] = ext[s][v];
    }
    const double* q = ubc[s];
    if (!(q[0] > 0.0) || !(g1 * (q[2] - 0.5 * q[1] * q[1] / q[0]) > 0.0)) return ESRK_ENONPHYS;
  }
  for (int s = 0; s < 2; ++s) {
    for (int v = 0; v < 5; ++v) x->mp.ubc[s][v] = ubc[s][v];
    x->mp.bckind[s] = kind[s] == ESRK_BC_OUTFLOW ? 1 : 0;
  }
  x->mp.bc = 1;
  ++x->gen;
  return ESRK_OK;
}

esrk_status esrk_set_dirichlet(esrk_ctx* x, const double* u_left, const double* u_right) {
  if (!x || (!u_left) != (!u_right)) return ESRK_EINVAL;
  if (!u_left) {
    x->mp.bc = 0;
    ++x->gen;
    return ESRK_OK;
  }
  return esrk_set_boundaries(x, ESRK_BC_DIRICHLET, u_left, ESRK_BC_DIRICHLET, u_right);
}

esrk_status esrk_set_root_method(esrk_ctx* x, int method) {
  if (!x || (method != ESRK_ROOT_ILLINOIS && method != ESRK_ROOT_BRENT &&
             method != ESRK_ROOT_BISECTION && method != ESRK_ROOT_ALEFELD))
    return ESRK_EINVAL;
  x->root_method = method;
  ++x->gen;
  return ESRK_OK;
}

esrk_status esrk_set_relaxation_mode(esrk_ctx* x, int mode) {
  if (!x || (mode != ESRK_RELAX_LOCAL && mode != ESRK_RELAX_GLOBAL && mode != ESRK_RELAX_NONE))
    return ESRK_EINVAL;
  x->relax_mode = mode;
  ++x->gen;
  return ESRK_OK;
}

esrk_status esrk_global_relaxation_solve(esrk_ctx* x, const double* u_old, const double* du,
                                         const double* deta, double* gamma, int* passes,
                                         void* stream) {
  if (!x || !u_old || !du || !deta || !gamma) return ESRK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  x->last = s;
  esrk::GlobState h;
  hipError_t e = esrk::launch_glob_solve(x->mp, u_old, du, deta, nullptr, x->glob_state,
                                         x->glob_parts, x->relax_parts, x->scal, 0, 0,
                                         x->cfg.root_tol, x->cfg.gamma_max, kGlobMaxPasses, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(gamma, &x->glob_state->gamma, sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&h, x->glob_state, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return ESRK_EHIP;
  if (passes) *passes = h.passes;
  return (esrk_status)h.status;
}

esrk_status esrk_local_relaxation_solve_ml(esrk_ctx* x, const double* u_old, const double* du,
                                           const double* deta, double dt,
                                           const double* visc_rate, const float* model,
                                           float* feats, double* gamma_k, double* gamma,
                                           int32_t* iters, void* stream) {
  if (!x || !u_old || !du || !deta || !gamma_k || !gamma || !(dt > 0.0)) return ESRK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  x->last = s;
  esrk::RelaxArgs r = relax_args(x, u_old, du, deta, nullptr, gamma_k, iters);
  r.model = model;
  r.feats = feats;
  r.vfeat = visc_rate;
  r.dt_host = dt;
  hipError_t e = esrk::launch_relax(x->mp, r, s);
  if (e == hipSuccess)
    e = esrk::launch_relax_finish(x->relax_parts, x->n_relax_parts, x->scal, gamma, s);
  return hip_status(e);
}

esrk_status esrk_set_step_model(esrk_ctx* x, const float* model, float* feats_out) {
  if (!x) return ESRK_EINVAL;
  x->step_model = model;
  x->step_feats = feats_out;
  ++x->gen;
  return ESRK_OK;
}

esrk_status esrk_mlp_prepare(float* model, const float* raw, const double* gamma, int B, int fit,
                             float* x_norm, float* t_norm, void* stream) {
  if (!model || B < 0 || (B > 0 && (!raw || !x_norm))) return ESRK_EINVAL;
  if (gamma && !t_norm) return ESRK_EINVAL;
  return hip_status(esrk::launch_mlp_prepare(model, raw, gamma, B, fit, x_norm, t_norm,
                                             (hipStream_t)stream));
}

esrk_status esrk_mlp_forward(const float* model, const float* x_norm, int B, float* y,
                             void* stream) {
  if (!model || B < 0 || (B > 0 && (!x_norm || !y))) return ESRK_EINVAL;
  return hip_status(esrk::launch_mlp_forward(model, x_norm, B, y, (hipStream_t)stream));
}

size_t esrk_mlp_grad_work_size(int B) {
  if (B < 1) return 0;
  return (size_t)esrk::mlp_grad_blocks(B) * (size_t)(ESRK_MLP_TRAINED + 1);
}

esrk_status esrk_mlp_grad(const float* model, const float* x_norm, const float* t_norm, int B,
                          float* grad, float* loss, float* work, void* stream) {
  if (!model || !x_norm || !t_norm || B < 1 || !grad || !work) return ESRK_EINVAL;
  return hip_status(esrk::launch_mlp_grad(model, x_norm, t_norm, B, grad, loss, work,
                                          (hipStream_t)stream));
}

esrk_status esrk_mlp_adam(float* model, const float* grad, float* m, float* v, int step,
                          float lr, void* stream) {
  if (!model || !grad || !m || !v || step < 1 || !(lr > 0.f)) return ESRK_EINVAL;
  return hip_status(esrk::launch_mlp_adam(model, grad, m, v, step, lr, (hipStream_t)stream));
}

esrk_status esrk_sync_status(esrk_ctx* x, int64_t* bad_elem) {
  if (!x) return ESRK_EINVAL;
  if (hipStreamSynchronize(x->last) != hipSuccess) return ESRK_EHIP;
  DevScalars h;
  if (hipMemcpy(&h, x->scal, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return ESRK_EHIP;
  if (bad_elem) *bad_elem = (h.bad_elem == INT64_MAX) ? -1 : (int64_t)h.bad_elem;
  const esrk_status st = (esrk_status)h.status;
  if (h.status != 0) {
    h.status = 0;
    h.bad_elem = INT64_MAX;
    if (hipMemcpy(x->scal, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) return ESRK_EHIP;
  }
  return st;
}

}  // extern "C"
