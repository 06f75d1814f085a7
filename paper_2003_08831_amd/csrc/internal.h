// Internal declarations shared by the HIP sources of libesrk (not part of the
// C-ABI).  Nothing here is shared with the CPU oracle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/esrk.h"

namespace esrk {

constexpr int kMaxN = 6;  // degree <= 5

// Network proposing relaxation parameters (mlp.hip): layout of the model vector.
constexpr int kMlpIn = 5, kMlpH = 32;
constexpr int kOffW1 = 0, kOffB1 = 160, kOffW2 = 192, kOffB2 = 1216, kOffW3 = 1248, kOffB3 = 1280;
constexpr int kMlpTrained = 1281;
constexpr int kOffScale = 1281, kOffMean = 1286, kOffStd = 1291, kOffOutMean = 1296,
              kOffOutStd = 1297;
constexpr int kMlpModel = 1298;

// Device-resident scalars of one context.
struct DevScalars {
  double dt;           // step size of the current step
  double gamma;        // global relaxation parameter of the last solve
  int status;          // latched esrk_status (0 = ok)
  int rejected;        // error-controlled step: the last attempt was rejected
  long long bad_elem;  // smallest offending element, or INT64_MAX
  double err;          // error-controlled step: weighted norm of the estimate
  double dt_next;      // error-controlled step: proposed next step size
};

// Per-block partial results (no same-address atomics on the hot path; the
// consumer kernel reduces the partials in a fixed order).
constexpr int kSpeedBlocks = 256;  // blocks of the wave-speed pass
struct RelaxPart {
  double gmin;      // min over the block's elements of gamma_k (+INF if none)
  int n_inactive;   // elements with gamma_k = +INF
  int max_iters;    // largest number of phi evaluations
  int sum_iters;    // phi evaluations summed over the block's elements
};

// Mesh + operator tables passed by value to kernels.
struct MeshParams {
  int dim, n, nd, ne;
  int nel[3];
  double two_over_h[3];  // metric of the affine element map, 2/h_m
  double half_h[3];      // h_m / 2
  double D2[kMaxN * kMaxN];  // 2 D_ab, D = Lobatto differentiation matrix
  double w[kMaxN];           // Lobatto weights
  double inv_w_end;          // 1 / w_0 = 1 / w_p
  double gg;                 // ratio of specific heats
  double lambda_scale;
  double cfl, hmin;
  int bc;             // 0 periodic, 1 boundaries at both ends (1-D Euler)
  double ubc[2][5];   // Dirichlet exterior states (conserved): [0] left, [1] right
  int bckind[2];      // per end: 0 Dirichlet (ubc), 1 outflow (exterior = interior trace)
};

// The per-mesh part of MeshParams (differs between the simulations of a batch).
struct MeshDims {
  int ne;
  int nel[3];
  double two_over_h[3];
  double half_h[3];
  double hmin, cfl;
  int bc;  // 0 periodic, 1 boundaries at both ends of direction 0 (1-D)
};
// Work item of block b of nb.  The hardware hands consecutive blocks of a
// launch to the 8 XCDs in turn; this remap gives the blocks one XCD receives
// consecutive items, so elements that share faces are mostly handled on the
// same XCD and read each other's traces from its L2.  A bijection on [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  constexpr int X = 8;
  const int q = nb / X, rem = nb - q * X;
  const int x = b % X, i = b / X;
  return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + i;
}

__host__ __device__ inline MeshDims dims_of(const MeshParams& mp) {
  MeshDims d;
  d.ne = mp.ne;
  for (int m = 0; m < 3; ++m) {
    d.nel[m] = mp.nel[m];
    d.two_over_h[m] = mp.two_over_h[m];
    d.half_h[m] = mp.half_h[m];
  }
  d.hmin = mp.hmin;
  d.cfl = mp.cfl;
  d.bc = mp.bc;
  return d;
}

// One simulation of a batch: its mesh, where its arrays start in the packed
// batch arrays, and its ranges in the per-block partial arrays.
struct SimParams {
  MeshDims md;
  long long base;       // first double of the sim's state in packed [v][k][i] arrays
  long long elem_base;  // first element of the sim in packed per-element arrays
  int speed_p0, speed_p1;
  int relax_p0, relax_p1;
};

// Runge-Kutta stage coefficients in the two-register form used on the device:
//   y_{i+1} = alpha_i u_old + beta_i y_i + c_i dt k_i,   du += b_i dt k_i.
struct StageCoef {
  double alpha, beta, c, b;
};

// Rows of a general explicit tableau: y_{i+1} additionally takes
// dt a_{i+1,j} k_j for the stored slopes of earlier stages j < i.
constexpr int kMaxPrev = 6;
constexpr int kMaxStages = 8;
struct StageRow {
  int nprev;
  int prev_slot[kMaxPrev];  // slot of k_j in the slope store
  double prev_a[kMaxPrev];  // a_{i+1,j}
  int kstore;               // 1 + slot this stage's slope is stored in (0: not
                            // stored, so zero-initialized arguments store nothing)
  double ecoef;             // b_i - bhat_i (embedded pairs)
};

// The part of a stage's arguments that only general tableaux and embedded
// pairs use.
struct StageExtra {
  StageRow row;
  double* kst;   // slope store, slot j at kst + j nv N
  double* err;   // nullable: err (+)= ecoef dt k, stage 0 overwrites
  // nullable (last stage): per element, sum over nodes and variables of
  // (err / (atol + rtol max(|u_old|, |u_old + du|)))^2
  double* errk;
  double atol, rtol;
};

struct RhsArgs {
  const double* y;      // state the right-hand side is evaluated at
  const double* u_old;  // stage mode: step start state
  double* out;          // plain mode: dudt; stage mode: y_{i+1} (nullable on last stage)
  double* du;           // stage mode: increment accumulator
  double* eta;          // plain: eta_rate (nullable); stage: deta accumulator
  const double* dt_dev; // stage mode: device dt (nullable -> dt_host or speed_parts)
  const double* speed_parts;  // stage 0 with CFL step: wave-speed maxima per block
  int n_speed_parts;
  double* dt_store;     // first stage: where the step size is published (nullable)
  long long elem_base;  // added to element indices in error reports
  const double* visc;   // nullable: viscous right-hand side added to k (Navier-Stokes)
  double dt_host;
  StageCoef sc;
  int stage_mode;       // 0: plain right-hand side, 1: RK stage
  int first;            // stage 0 overwrites du/deta
  DevScalars* scal;
  // stage mode (nullable): general tableau rows and error estimate, in device
  // memory (read in the epilogue only, so they hold no scalar registers
  // through the flux phases)
  const StageExtra* ex;
  // stage mode (nullable): phi_k(0) accumulated without cancellation,
  // phi (+)= b dt sum_nodes M (w(u_old) - w(y)).k  (stage 0 writes 0)
  double* phi0;
};

// Host tables (Lobatto nodes/weights/derivative matrix), built in extended
// precision from the closed forms.
void lobatto_tables(int deg, double* x, double* w, double* D);

// Launchers (return hipError_t).
hipError_t launch_rhs(const MeshParams& mp, int precision, const RhsArgs& a,
                      hipStream_t s);

// BR1 viscous terms: theta (T precision, [dim][nv][N]) and Visc (FP64, [nv][N]).
struct NsArgs {
  const double* y;
  void* flux;  // viscous fluxes g_m, [m][v][node], T precision
  double* visc;
  double* diss;  // nullable, [ne]
  double mu, kappa, R;
};
hipError_t launch_ns(const MeshParams& mp, int precision, const NsArgs& a, hipStream_t s);

struct RelaxArgs {
  const double* u_old;
  const double* du;
  const double* deta;
  const float* guess;  // nullable: external first trial points
  const float* model;  // nullable: network proposing the first trial point
  float* feats;        // nullable: raw network features per element [ne][5]
  const double* vfeat; // nullable: per-element viscous dissipation rate
  const double* dt_dev;  // step size for the features (nullable -> dt_host)
  double dt_host;
  double* gamma_k;
  int32_t* iters;      // nullable
  RelaxPart* parts;    // one per block
  DevScalars* scal;
  double tol, gamma_max;
  int maxit;
  int method;  // ESRK_ROOT_*: trial-point rule inside the bracket
  // FP32-flux increments: an element whose phi(0) >= 0 while its entropy
  // change r(1) stays within the FP32 rounding level is inactive, not ENOROOT
  int fp32_increments;
  // error-controlled steps: nothing to solve when scal->rejected is set
  int check_reject;
  // nullable: phi_k(0) per element from the stages (else A_k - deta_k)
  const double* phi0_in;
};
int relax_blocks(const MeshParams& mp);

// global relaxation: trial values per pass and the partial layout
// [A, scale, sum deta, sum |deta|, B(g_0) .. B(g_{T-1})]
constexpr int kGlobTrials = 4;
constexpr int kGlobParts = 4 + kGlobTrials;
struct GlobTrials {
  double g[kGlobTrials];
};
int glob_blocks(const MeshParams& mp);
// Device state of the global relaxation solve (bracket, trial values, result).
struct GlobState {
  double lo, flo, hi, fhi, s_prev, gamma, phi0, noise;
  double g[kGlobTrials];
  int stage;   // 0 first pass, 1 expanding the bracket, 2 refining, 3 done
  int halved;  // the last refining pass halved the bracket
  int passes;  // device passes that did work
  int status;  // ESRK_OK, ESRK_ENOROOT or ESRK_ENAN
};
// Global relaxation on the device: max_passes sweeps of four trial values
// (a sweep after convergence returns at once), the bracket logic in a
// one-block kernel between sweeps, no host synchronization.  phi0_in
// (nullable): per-element phi_k(0), summed in place of A - sum deta.  The
// result goes to st->gamma and to rparts[0] for the update; with latch, an
// error is latched in scal like the local solve's; with check_reject, a
// rejected error-controlled attempt is skipped.
hipError_t launch_glob_solve(const MeshParams& mp, const double* u_old, const double* du,
                             const double* deta, const double* phi0_in, GlobState* st,
                             double* parts, RelaxPart* rparts, DevScalars* scal, int latch,
                             int check_reject, double tol, double gmax, int max_passes,
                             hipStream_t s);
hipError_t launch_set_part(RelaxPart* parts, double g, hipStream_t s);
hipError_t launch_relax(const MeshParams& mp, const RelaxArgs& a, hipStream_t s);
// gamma = min over partials (1 if all inactive) -> *gamma and scal->gamma
hipError_t launch_relax_finish(const RelaxPart* parts, int nparts, DevScalars* scal,
                               double* gamma, hipStream_t s);
// wave-speed maxima per block of the state u -> parts[kSpeedBlocks]
hipError_t launch_speed(const MeshParams& mp, const double* u, double* parts, hipStream_t s);
// u <- u + gamma du with gamma reduced from the relaxation partials (skipped
// when an error is latched); t <- t + gamma dt; optional stats.
hipError_t launch_apply(const MeshParams& mp, double* u, const double* du, double* t,
                        const RelaxPart* parts, int nparts, DevScalars* scal,
                        const double* dt_dev, double* stats_out, int adaptive, hipStream_t s);
// Error control: err = sqrt(sum_k errk[k] / count) -> scal->err,
// scal->rejected = !(err <= 1), scal->dt_next = scal->dt * factor(err, q)
// (the factor clip(safety err^(-1/(q+1)), 0.1, 10), safety 0.9 after an
// accepted and 0.45 after a rejected attempt; 0.1 for a non-finite err).
// With decide = 0 only *norm_out (device scalar) receives err.
hipError_t launch_adapt(const double* errk, int ne, double count, int q, int decide,
                        DevScalars* scal, double* norm_out, hipStream_t s);

// ---- network kernels ----
hipError_t launch_mlp_forward(const float* p, const float* X, int B, float* Y, hipStream_t s);
hipError_t launch_mlp_prepare(float* p, const float* raw, const double* gamma, int B, int fit,
                              float* xn, float* tn, hipStream_t s);
int mlp_grad_blocks(int B);
// part: mlp_grad_blocks(B) * (kMlpTrained + 1) floats of workspace
hipError_t launch_mlp_grad(const float* p, const float* X, const float* T, int B, float* grad,
                           float* loss, float* part, hipStream_t s);
hipError_t launch_mlp_adam(float* p, const float* g, float* m, float* v, int step, float lr,
                           hipStream_t s);

// ---- batches of simulations (2-D meshes) ----
int rhs_batch_tiles(const MeshParams& mp, int precision, int* out);
hipError_t launch_rhs_batch(const MeshParams& mp, int precision, int tile, const RhsArgs& a,
                            const SimParams* sims, const int2* items, int nitems,
                            double* dt_sims, const double* dt_in, int grid, hipStream_t s);
int relax_batch_epb(const MeshParams& mp);
hipError_t launch_relax_batch(const MeshParams& mp, const RelaxArgs& a, const SimParams* sims,
                              const int2* items, int nitems, int grid, hipStream_t s);
hipError_t launch_speed_batch(const MeshParams& mp, const double* u, const SimParams* sims,
                              const int2* items, int nitems, int grid, double* parts,
                              hipStream_t s);
hipError_t launch_apply_batch(const MeshParams& mp, double* u, const double* du,
                              const SimParams* sims, const int2* items, int nitems, int grid,
                              const RelaxPart* parts, DevScalars* scal, const double* dt_sims,
                              double* t, double* gamma_out, hipStream_t s);

}  // namespace esrk
