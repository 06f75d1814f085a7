// Batches of independent simulations (C-ABI in include/esrk.h): many 2-D
// meshes of different sizes that share degree, physics, precision and
// Runge-Kutta method are advanced together.  Each stage is one kernel launch
// over a work list of (simulation, element tile) items covering all
// simulations; the relaxation, the per-simulation gamma = min over that
// simulation's elements, the per-simulation CFL step and the update are one
// launch each.  A whole multi-step sequence can be captured once into a
// hipGraph and replayed.  The tile (elements per block) of the stage kernel is
// chosen by timing the compiled candidates on the caller's state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using esrk::DevScalars;
using esrk::MeshParams;
using esrk::RelaxPart;
using esrk::SimParams;
using esrk::StageCoef;

struct esrk_batch {
  esrk_config cfg0;
  MeshParams mp;  // shared operator tables and constants
  int nsims = 0;
  int stages = 0;
  StageCoef sc[4];
  std::vector<SimParams> hsims;
  SimParams* sims = nullptr;
  long long len = 0;     // doubles in the packed state
  long long nelems = 0;  // elements of all simulations
  int ntiles = 0, tiles[3] = {0, 0, 0}, tile = 0;
  int2* rhs_items[3] = {nullptr, nullptr, nullptr};
  int n_rhs_items[3] = {0, 0, 0};
  int2* relax_items = nullptr;
  int n_relax_items = 0;
  int2* node_items = nullptr;  // 256-node chunks (wave speed, update)
  int n_node_items = 0;
  double *ya = nullptr, *yb = nullptr, *du = nullptr, *deta = nullptr, *gamma_k = nullptr;
  double* phi0acc = nullptr;  // phi_k(0) accumulated by the stages
  int32_t* iters = nullptr;
  double* speed_parts = nullptr;
  RelaxPart* relax_parts = nullptr;
  double* dt_sims = nullptr;
  DevScalars* scal = nullptr;
  hipStream_t last = nullptr;
  // captured multi-step graph
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  double* g_u = nullptr;
  double* g_t = nullptr;
  double* g_gamma = nullptr;
  int g_steps = 0;
  int g_tile = -1;
  hipStream_t g_stream = nullptr;
};

namespace {

constexpr int kGrid = 2048;  // blocks of the work-list kernels (they stride over items)

int batch_tableau(int which, StageCoef* sc) {
  // same two-register forms as the single-mesh path
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

template <typename X>
bool upload(X** dst, const std::vector<X>& v) {
  if (v.empty()) return true;
  if (hipMalloc(dst, v.size() * sizeof(X)) != hipSuccess) return false;
  return hipMemcpy(*dst, v.data(), v.size() * sizeof(X), hipMemcpyHostToDevice) == hipSuccess;
}

int grid_for(int nitems) { return std::max(1, std::min(nitems, kGrid)); }

hipError_t enqueue_step(esrk_batch* b, double* u, double* t, double* gamma, int tile_idx,
                        hipStream_t s) {
  hipError_t e = esrk::launch_speed_batch(b->mp, u, b->sims, b->node_items, b->n_node_items,
                                          grid_for(b->n_node_items), b->speed_parts, s);
  const double* yin = u;
  double* bufs[2] = {b->ya, b->yb};
  for (int i = 0; i < b->stages && e == hipSuccess; ++i) {
    const bool last = i == b->stages - 1;
    esrk::RhsArgs a;
    std::memset(&a, 0, sizeof(a));
    a.y = yin;
    a.u_old = u;
    a.out = last ? nullptr : bufs[i & 1];
    a.du = b->du;
    a.eta = nullptr;  // the solve takes phi_k(0) from the stages
    a.phi0 = b->phi0acc;
    a.speed_parts = i == 0 ? b->speed_parts : nullptr;
    a.sc = b->sc[i];
    a.stage_mode = 1;
    a.first = i == 0;
    a.scal = b->scal;
    e = esrk::launch_rhs_batch(b->mp, b->cfg0.precision, b->tiles[tile_idx], a, b->sims,
                               b->rhs_items[tile_idx], b->n_rhs_items[tile_idx], b->dt_sims,
                               i == 0 ? nullptr : b->dt_sims,
                               grid_for(b->n_rhs_items[tile_idx]), s);
    yin = bufs[i & 1];
  }
  if (e == hipSuccess) {
    esrk::RelaxArgs r{};
    r.u_old = u;
    r.du = b->du;
    r.deta = nullptr;
    r.phi0_in = b->phi0acc;
    r.guess = nullptr;
    r.gamma_k = b->gamma_k;
    r.iters = b->iters;
    r.parts = b->relax_parts;
    r.scal = b->scal;
    r.tol = b->cfg0.root_tol;
    r.gamma_max = b->cfg0.gamma_max;
    r.maxit = b->cfg0.root_maxit;
    r.fp32_increments = b->cfg0.precision == ESRK_FP32_FLUX;
    e = esrk::launch_relax_batch(b->mp, r, b->sims, b->relax_items, b->n_relax_items,
                                 grid_for(b->n_relax_items), s);
  }
  if (e == hipSuccess)
    e = esrk::launch_apply_batch(b->mp, u, b->du, b->sims, b->node_items, b->n_node_items,
                                 grid_for(b->n_node_items), b->relax_parts, b->scal, b->dt_sims,
                                 t, gamma, s);
  return e;
}

void drop_graph(esrk_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->g_steps = 0;
}

}  // namespace

extern "C" {

esrk_status esrk_batch_create(const esrk_config* cfgs, int nsims, esrk_batch** out) {
  if (!cfgs || nsims < 1 || !out) return ESRK_EINVAL;
  *out = nullptr;
  const esrk_config& c0 = cfgs[0];
  if (c0.dim != 2) return ESRK_ENOTSUP;
  if (c0.deg < 1 || c0.deg > esrk::kMaxN - 1 || !(c0.gas_gamma > 1.0)) return ESRK_EINVAL;
  if (c0.precision != ESRK_FP64 && c0.precision != ESRK_FP32_FLUX) return ESRK_EINVAL;
  if (c0.tableau != ESRK_SSPRK33 && c0.tableau != ESRK_RK44) return ESRK_ENOTSUP;
  if (c0.mu != 0.0) return ESRK_ENOTSUP;
  for (int s = 0; s < nsims; ++s) {
    const esrk_config& c = cfgs[s];
    if (c.dim != c0.dim || c.deg != c0.deg || c.precision != c0.precision ||
        c.tableau != c0.tableau || c.gas_gamma != c0.gas_gamma ||
        c.lambda_scale != c0.lambda_scale || c.mu != c0.mu)
      return ESRK_EINVAL;
    for (int m = 0; m < 2; ++m)
      if (c.nel[m] < 1 || !(c.hi[m] > c.lo[m])) return ESRK_EINVAL;
    // each simulation's state is indexed in 32 bits by the kernels
    const size_t nd = (size_t)(c0.deg + 1) * (size_t)(c0.deg + 1);
    if ((size_t)c.nel[0] * (size_t)c.nel[1] * nd * 4 > (size_t)INT32_MAX) return ESRK_EINVAL;
  }
  esrk_batch* b = new (std::nothrow) esrk_batch();
  if (!b) return ESRK_ENOMEM;
  b->cfg0 = c0;
  if (!(b->cfg0.root_tol > 0.0)) b->cfg0.root_tol = 1e-12;
  if (b->cfg0.root_maxit <= 0) b->cfg0.root_maxit = 60;
  if (!(b->cfg0.gamma_max > 1.0)) b->cfg0.gamma_max = 4.0;
  b->nsims = nsims;
  b->stages = batch_tableau(c0.tableau, b->sc);
  MeshParams& mp = b->mp;
  std::memset(&mp, 0, sizeof(mp));
  mp.dim = 2;
  mp.n = c0.deg + 1;
  mp.nd = mp.n * mp.n;
  double xs[esrk::kMaxN], D[esrk::kMaxN * esrk::kMaxN];
  esrk::lobatto_tables(c0.deg, xs, mp.w, D);
  for (int i = 0; i < mp.n * mp.n; ++i) mp.D2[i] = 2.0 * D[i];
  mp.inv_w_end = 1.0 / mp.w[0];
  mp.gg = c0.gas_gamma;
  mp.lambda_scale = c0.lambda_scale;
  b->ntiles = esrk::rhs_batch_tiles(mp, c0.precision, b->tiles);
  b->tile = 1;  // the default (middle) candidate
  const int nv = 4;
  const int epb_relax = esrk::relax_batch_epb(mp);
  std::vector<std::vector<int2>> per_sim[3];
  for (int t = 0; t < 3; ++t) per_sim[t].resize(nsims);
  std::vector<int2> items[3], ritems, nitems;
  int speed_count = 0, relax_count = 0;
  for (int s = 0; s < nsims; ++s) {
    const esrk_config& c = cfgs[s];
    SimParams P;
    std::memset(&P, 0, sizeof(P));
    P.md.ne = c.nel[0] * c.nel[1];
    P.md.nel[0] = c.nel[0];
    P.md.nel[1] = c.nel[1];
    P.md.nel[2] = 1;
    double hmin = INFINITY;
    for (int m = 0; m < 3; ++m) {
      const double h = m < 2 ? (c.hi[m] - c.lo[m]) / c.nel[m] : 1.0;
      P.md.two_over_h[m] = 2.0 / h;
      P.md.half_h[m] = 0.5 * h;
      if (m < 2) hmin = std::fmin(hmin, h);
    }
    P.md.hmin = hmin;
    P.md.cfl = c.cfl > 0.0 ? c.cfl : 0.5;
    P.base = b->len;
    P.elem_base = b->nelems;
    const long long N = (long long)P.md.ne * mp.nd;
    P.speed_p0 = speed_count;
    for (long long i0 = 0; i0 < N; i0 += 256) nitems.push_back(make_int2(s, (int)i0));
    speed_count = (int)nitems.size();
    P.speed_p1 = speed_count;
    P.relax_p0 = relax_count;
    for (int k0 = 0; k0 < P.md.ne; k0 += epb_relax) ritems.push_back(make_int2(s, k0));
    relax_count = (int)ritems.size();
    P.relax_p1 = relax_count;
    for (int t = 0; t < b->ntiles; ++t)
      for (int k0 = 0; k0 < P.md.ne; k0 += b->tiles[t]) per_sim[t][s].push_back(make_int2(s, k0));
    b->hsims.push_back(P);
    b->len += (long long)nv * N;
    b->nelems += P.md.ne;
  }
  // larger simulations first, so that the blocks striding over the items end together
  std::vector<int> order(nsims);
  for (int s = 0; s < nsims; ++s) order[s] = s;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return b->hsims[a].md.ne > b->hsims[c].md.ne; });
  for (int t = 0; t < b->ntiles; ++t)
    for (int s : order) items[t].insert(items[t].end(), per_sim[t][s].begin(), per_sim[t][s].end());
  bool ok = upload(&b->sims, b->hsims) && upload(&b->relax_items, ritems) &&
            upload(&b->node_items, nitems);
  for (int t = 0; t < b->ntiles && ok; ++t) {
    ok = upload(&b->rhs_items[t], items[t]);
    b->n_rhs_items[t] = (int)items[t].size();
  }
  b->n_relax_items = (int)ritems.size();
  b->n_node_items = (int)nitems.size();
  ok = ok && hipMalloc(&b->ya, b->len * sizeof(double)) == hipSuccess &&
       hipMalloc(&b->yb, b->len * sizeof(double)) == hipSuccess &&
       hipMalloc(&b->du, b->len * sizeof(double)) == hipSuccess &&
       hipMalloc(&b->deta, b->nelems * sizeof(double)) == hipSuccess &&
       hipMalloc(&b->phi0acc, b->nelems * sizeof(double)) == hipSuccess &&
       hipMalloc(&b->gamma_k, b->nelems * sizeof(double)) == hipSuccess &&
       hipMalloc(&b->iters, b->nelems * sizeof(int32_t)) == hipSuccess &&
       hipMalloc(&b->speed_parts, std::max(1, b->n_node_items) * sizeof(double)) == hipSuccess &&
       hipMalloc(&b->relax_parts, std::max(1, b->n_relax_items) * sizeof(RelaxPart)) ==
           hipSuccess &&
       hipMalloc(&b->dt_sims, nsims * sizeof(double)) == hipSuccess &&
       hipMalloc(&b->scal, sizeof(DevScalars)) == hipSuccess;
  if (ok) {
    DevScalars init;
    std::memset(&init, 0, sizeof(init));
    init.bad_elem = INT64_MAX;
    init.gamma = 1.0;
    ok = hipMemcpy(b->scal, &init, sizeof(init), hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!ok || b->ntiles == 0) {
    esrk_batch_destroy(b);
    return ok ? ESRK_ENOTSUP : ESRK_ENOMEM;
  }
  *out = b;
  return ESRK_OK;
}

void esrk_batch_destroy(esrk_batch* b) {
  if (!b) return;
  drop_graph(b);
  (void)hipFree(b->sims);
  for (int t = 0; t < 3; ++t) (void)hipFree(b->rhs_items[t]);
  (void)hipFree(b->relax_items);
  (void)hipFree(b->node_items);
  (void)hipFree(b->ya);
  (void)hipFree(b->yb);
  (void)hipFree(b->du);
  (void)hipFree(b->deta);
  (void)hipFree(b->phi0acc);
  (void)hipFree(b->gamma_k);
  (void)hipFree(b->iters);
  (void)hipFree(b->speed_parts);
  (void)hipFree(b->relax_parts);
  (void)hipFree(b->dt_sims);
  (void)hipFree(b->scal);
  delete b;
}

int esrk_batch_num_sims(const esrk_batch* b) { return b ? b->nsims : 0; }
size_t esrk_batch_state_len(const esrk_batch* b) { return b ? (size_t)b->len : 0; }
size_t esrk_batch_num_elems(const esrk_batch* b) { return b ? (size_t)b->nelems : 0; }
size_t esrk_batch_offset(const esrk_batch* b, int sim) {
  return (b && sim >= 0 && sim < b->nsims) ? (size_t)b->hsims[sim].base : 0;
}
size_t esrk_batch_elem_offset(const esrk_batch* b, int sim) {
  return (b && sim >= 0 && sim < b->nsims) ? (size_t)b->hsims[sim].elem_base : 0;
}
int esrk_batch_tile(const esrk_batch* b) { return b ? b->tiles[b->tile] : 0; }

esrk_status esrk_batch_step(esrk_batch* b, double* u, double* t, double* gamma, void* stream) {
  if (!b || !u || !t) return ESRK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  b->last = s;
  return enqueue_step(b, u, t, gamma, b->tile, s) == hipSuccess ? ESRK_OK : ESRK_EHIP;
}

esrk_status esrk_batch_autotune(esrk_batch* b, const double* u, int reps, int* tile_out,
                                void* stream) {
  if (!b || !u) return ESRK_EINVAL;
  if (reps < 1) reps = 10;
  hipStream_t s = (hipStream_t)stream;
  b->last = s;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return ESRK_EHIP;
  float best = INFINITY;
  int best_t = b->tile;
  esrk_status st = ESRK_OK;
  // time the middle stage of the method on u for every candidate tile
  esrk::RhsArgs a;
  std::memset(&a, 0, sizeof(a));
  a.y = u;
  a.u_old = u;
  a.out = b->ya;
  a.du = b->du;
  a.phi0 = b->phi0acc;  // as in the steps: phi_k(0), no entropy rate
  a.sc = b->sc[1];
  a.stage_mode = 1;
  a.first = 1;
  a.scal = b->scal;
  // a fixed positive step for timing: dt_sims is written by the first launch
  a.dt_host = 1e-6;
  for (int t = 0; t < b->ntiles && st == ESRK_OK; ++t) {
    const int g = grid_for(b->n_rhs_items[t]);
    hipError_t e = hipSuccess;
    for (int r = 0; r < 2 && e == hipSuccess; ++r)
      e = esrk::launch_rhs_batch(b->mp, b->cfg0.precision, b->tiles[t], a, b->sims,
                                 b->rhs_items[t], b->n_rhs_items[t], b->dt_sims, nullptr, g, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r)
      e = esrk::launch_rhs_batch(b->mp, b->cfg0.precision, b->tiles[t], a, b->sims,
                                 b->rhs_items[t], b->n_rhs_items[t], b->dt_sims, nullptr, g, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      st = ESRK_EHIP;
      break;
    }
    if (ms < best) {
      best = ms;
      best_t = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == ESRK_OK) {
    b->tile = best_t;
    if (tile_out) *tile_out = b->tiles[best_t];
  }
  return st;
}

esrk_status esrk_batch_run_graph(esrk_batch* b, double* u, double* t, double* gamma, int nsteps,
                                 void* stream) {
  if (!b || !u || !t || nsteps < 1 || !stream) return ESRK_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  b->last = s;
  if (!(b->gexec && b->g_u == u && b->g_t == t && b->g_gamma == gamma && b->g_steps == nsteps &&
        b->g_tile == b->tile && b->g_stream == s)) {
    drop_graph(b);
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return ESRK_EHIP;
    hipError_t e = hipSuccess;
    for (int i = 0; i < nsteps && e == hipSuccess; ++i) e = enqueue_step(b, u, t, gamma, b->tile, s);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return ESRK_EHIP;
    }
    if (hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return ESRK_EHIP;
    }
    b->graph = g;
    b->g_u = u;
    b->g_t = t;
    b->g_gamma = gamma;
    b->g_steps = nsteps;
    b->g_tile = b->tile;
    b->g_stream = s;
  }
  return hipGraphLaunch(b->gexec, s) == hipSuccess ? ESRK_OK : ESRK_EHIP;
}

esrk_status esrk_batch_sync_status(esrk_batch* b, int64_t* bad_elem) {
  if (!b) return ESRK_EINVAL;
  if (hipStreamSynchronize(b->last) != hipSuccess) return ESRK_EHIP;
  DevScalars h;
  if (hipMemcpy(&h, b->scal, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return ESRK_EHIP;
  if (bad_elem) *bad_elem = (h.bad_elem == INT64_MAX) ? -1 : (int64_t)h.bad_elem;
  const esrk_status st = (esrk_status)h.status;
  if (h.status != 0) {
    h.status = 0;
    h.bad_elem = INT64_MAX;
    if (hipMemcpy(b->scal, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) return ESRK_EHIP;
  }
  return st;
}

}  // extern "C"
