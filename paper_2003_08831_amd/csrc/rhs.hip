// Fused entropy-stable right-hand side / Runge-Kutta stage kernel (gfx950).
//
// What it computes (Sec. 3.1, element equation, inviscid part): for every node
// i of element k,
//   dudt_i = -sum_m (2/h_m) [ sum_{j != i_m} 2 D[i_m][j] f#_m(u_i, u_{i, i_m <- j})
//                             + (1/w_p) f*_{+m}  (node on the +m face)
//                             - (1/w_0) f*_{-m}  (node on the -m face) ],
// with f# the entropy-conservative two-point flux and
// f* = f#(u_L, u_R) - (lambda_scale/2) lambda (u_R - u_L) the local
// Lax-Friedrichs interface flux.  This is the SBP-SAT form with the physical
// flux terms of the SAT and of the flux-differencing diagonal cancelled
// analytically (2 D_pp = 1/w_p on Lobatto nodes, D_ii = 0 for inner nodes).
// The epilogue forms the element entropy rate sum_i M_i w(u_i).dudt_i in FP64
// and, in stage mode, the Runge-Kutta update (Sec. 2, Runge-Kutta example).
//
// Mapping: one block holds E elements.  Phase 0: one thread per node stages the
// node primitives (rho, v, beta = rho/2p, |v|^2) in LDS with coalesced SoA
// loads.  Phase 1a: one thread per (element, direction, line) evaluates every
// unordered node pair of its line once (symmetric flux, scattered to both
// nodes with 2 D_ab and 2 D_ba) and writes the line's contribution to a
// per-direction LDS accumulator.  Phase 1b: one thread per (line, end) adds
// the interface flux at that end.  Phase 2: one thread per node sums the
// directions, writes the outputs and the per-element entropy-rate partials.
// Splitting 1a and 1b keeps the register peak at the larger of the two
// phases (3-D p=3 FP64: about 120 VGPRs instead of about 250 for both in one).
#include "device_math.h"
#include "internal.h"

// Tuning knobs (compile-time): the number of line tasks a block is sized for
// (elements per block = max(1, target / tasks per element)), capped by an LDS
// budget in KiB, and the minimum waves per SIMD requested from the register
// allocator (0 = compiler's choice).  One wavefront of tasks per block measured
// fastest: a single-wave block needs no cross-wave barrier waits and many
// small blocks overlap each other's memory latency.
#ifndef ESRK_RHS_TARGET_TASKS
#define ESRK_RHS_TARGET_TASKS 64
#endif
#ifndef ESRK_RHS_LDS_KB
#define ESRK_RHS_LDS_KB 64
#endif
#ifndef ESRK_RHS_WAVES_PER_EU
#define ESRK_RHS_WAVES_PER_EU 0
#endif

namespace esrk {

template <int DIM, int N>
struct Geo {
  static constexpr int ND = (DIM == 1) ? N : (DIM == 2) ? N * N : N * N * N;
  static constexpr int NL = ND / N;  // lines per direction
  static constexpr int NV = DIM + 2;
  static constexpr int TASKS = DIM * NL;
};

template <int DIM, int N, typename T>
struct RhsCfg {
  using G = Geo<DIM, N>;
  static constexpr int NP = DIM + 3;  // rho, v[DIM], beta, |v|^2
  // LDS slot of node i: i + i/N, so that lines along any direction spread
  // over the banks (element stride NDP)
  static constexpr int NDP = G::ND + G::ND / N;
  // the direction accumulators reuse the primitives' slots (phase 1a reads
  // the primitives into registers before any accumulator is written)
  static constexpr int SLOTS = NP > DIM * G::NV ? NP : DIM * G::NV;
  static constexpr int LDS_PER_ELEM =
      NDP * SLOTS * (int)sizeof(T) + G::ND * (int)sizeof(double);
  static constexpr int BUDGET = ESRK_RHS_LDS_KB * 1024;
  static constexpr int E_TASK =
      (ESRK_RHS_TARGET_TASKS / G::TASKS) > 0 ? ESRK_RHS_TARGET_TASKS / G::TASKS : 1;
  static constexpr int E_LDS = (BUDGET / LDS_PER_ELEM) > 0 ? BUDGET / LDS_PER_ELEM : 1;
  static constexpr int E = E_TASK < E_LDS ? E_TASK : E_LDS;
};

// Block shape for E elements per block.
template <int DIM, int N, typename T, int E>
struct RhsShape {
  using G = Geo<DIM, N>;
  using C = RhsCfg<DIM, N, T>;
  static constexpr int NP = C::NP, NDP = C::NDP;
  static constexpr int IR = 0, IV = 1, IB = DIM + 1, IV2 = DIM + 2;
  static constexpr int EN = E * G::ND, ENP = E * NDP;
  static constexpr int RAW = E * G::TASKS;
  static constexpr int THREADS = ((RAW < 64 ? 64 : RAW) + 63) / 64 * 64;
  static constexpr int SP = NP * ENP, SACC = DIM * G::NV * ENP;
  static constexpr int SBUF = SP > SACC ? SP : SACC;  // primitives, then accumulators
  static_assert(THREADS >= RAW, "one line task per thread");
};

__device__ __forceinline__ void latch(DevScalars* s, int code, long long elem) {
  atomicCAS(&s->status, 0, code);
  atomicMin((unsigned long long*)&s->bad_elem, (unsigned long long)elem);
}

template <int DIM>
__device__ __forceinline__ int neighbour(const MeshDims& md, int k, int m, int dir) {
  int c[3];
  c[0] = k % md.nel[0];
  c[1] = (k / md.nel[0]) % md.nel[1];
  c[2] = k / (md.nel[0] * md.nel[1]);
  int cm = (m == 0) ? c[0] : (m == 1) ? c[1] : c[2];
  const int nm = (m == 0) ? md.nel[0] : (m == 1) ? md.nel[1] : md.nel[2];
  cm += dir;
  if (md.bc && (cm < 0 || cm >= nm)) return -1;  // boundary face
  cm = (cm < 0) ? cm + nm : (cm >= nm ? cm - nm : cm);
  if (m == 0) c[0] = cm;
  if (m == 1) c[1] = cm;
  if (m == 2) c[2] = cm;
  return c[0] + md.nel[0] * (c[1] + md.nel[1] * c[2]);
}

// First node of line l along direction m (lines of a direction numbered
// lexicographically over the other directions); divisions by the compile-time
// N only.
template <int DIM, int N>
__device__ __forceinline__ int line_base(int m, int l) {
  if (DIM == 1) return 0;
  if (DIM == 2) return m == 0 ? l * N : l;
  const int b0 = l * N;                       // m = 0: l = i1 + N i2
  const int b1 = (l % N) + (l / N) * N * N;   // m = 1: l = i0 + N i2
  return m == 0 ? b0 : (m == 1 ? b1 : l);     // m = 2: l = i0 + N i1
}

// Interface flux f* in direction m between a left and a right node, given
// both primitive sets and conserved states.
template <typename T, int DIM>
__device__ __forceinline__ void interface_flux(int m, const Prim<T, DIM>& A, const T* qL,
                                               const Prim<T, DIM>& B, const T* qR, T gg,
                                               T half_inv_gm1, T lam_scale, T* F) {
  const PairMeans<T> mn = pair_means(A.rho, B.rho, A.beta, B.beta);
  ec_flux_from_means<T, DIM>(m, A, B, mn, half_inv_gm1, F);
  T vA = A.v[0], vB = B.v[0];
#pragma unroll
  for (int k = 1; k < DIM; ++k) {
    vA = (m == k) ? A.v[k] : vA;
    vB = (m == k) ? B.v[k] : vB;
  }
  // c^2 = gamma p / rho = gamma / (2 beta)
  const T cA = sqrt(T(0.5) * gg * rcp(A.beta)), cB = sqrt(T(0.5) * gg * rcp(B.beta));
  const T sA = fabs(vA) + cA, sB = fabs(vB) + cB;
  const T lam = sA > sB ? sA : sB;
  const T hl = T(0.5) * lam_scale * lam;
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) F[v] -= hl * (qR[v] - qL[v]);
}

// One block's work: E elements starting at element k0 of the mesh md.
template <int DIM, int N, typename T, int E>
__device__ __forceinline__ void rhs_block(const MeshParams& mp, const MeshDims& md,
                                          const RhsArgs& a, const int k0, T* sp, T* sacc,
                                          double* sred, double* s_dt, int* snbr) {
  using S = RhsShape<DIM, N, T, E>;
  using C = S;
  using G = Geo<DIM, N>;
  constexpr int ND = G::ND, NV = G::NV, NDP = S::NDP;
  constexpr int EN = S::EN;    // nodes per block
  constexpr int ENP = S::ENP;  // padded LDS slots per field
  constexpr int TH = S::THREADS;

  const int tid = threadIdx.x;
  // 32-bit node indices: the library rejects meshes with nv * nodes >= 2^31
  const int Ntot = md.ne * ND;
  const T gg = T(mp.gg);
  const T half_inv_gm1 = T(0.5) / (gg - T(1));

  // CFL step size of the first stage, from the wave-speed partials of the step
  // start state (max is exact, so every block derives the same dt).
  if (a.stage_mode && a.speed_parts && tid < 64) {
    double mx = 0.0;
    for (int q = tid; q < a.n_speed_parts; q += 64) mx = fmax(mx, a.speed_parts[q]);
#pragma unroll
    for (int off = 32; off >= 1; off /= 2) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (tid == 0) *s_dt = md.cfl * md.hmin / (double(mp.n) * mx);
  }

  // face neighbours of the block's elements (runtime divisions once per element)
  for (int t = tid; t < E * 2 * DIM; t += TH) {
    const int e = t / (2 * DIM);
    const int md_ = (t - e * 2 * DIM) >> 1;
    const int k = k0 + e < md.ne ? k0 + e : 0;
    snbr[t] = neighbour<DIM>(md, k, md_, (t & 1) ? +1 : -1);
  }

  // ---- phase 0: node primitives into LDS ----
  for (int idx = tid; idx < EN; idx += TH) {
    const int e = idx / ND;
    const int i = idx - e * ND;
    const int slot = e * NDP + i + i / N;
    const int k = k0 + e;
    T q[NV];
    if (k < md.ne) {
      const int gi = k0 * ND + idx;
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v] = T(a.y[v * Ntot + gi]);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v] = T(0);
      q[0] = T(1);
      q[NV - 1] = T(1);
    }
    Prim<T, DIM> P;
    T p;
    prim_from_cons<T, DIM>(q, gg, P, p);
    if (!(P.rho > T(0)) || !(p > T(0))) {
      if (k < md.ne) latch(a.scal, ESRK_ENONPHYS, a.elem_base + k);
      P.rho = T(1);
      P.beta = T(0.5);
    }
    sp[C::IR * ENP + slot] = P.rho;
#pragma unroll
    for (int d = 0; d < DIM; ++d) sp[(C::IV + d) * ENP + slot] = P.v[d];
    sp[C::IB * ENP + slot] = P.beta;
    sp[C::IV2 * ENP + slot] = P.v2;
  }
  __syncthreads();

  // ---- phase 1a: line tasks (volume pairs) ----
  // One task per thread.  The primitives of the line go to registers, then a
  // barrier: the accumulators written below overwrite the primitives' slots.
  {
    const int task = tid;
    const int e = task / G::TASKS;
    const int r = task - e * G::TASKS;
    const int m = r / G::NL;
    const int l = r - m * G::NL;
    const int k = k0 + e;
    const bool has = task < E * G::TASKS && k < md.ne;
    const int stride = (m == 0) ? 1 : (m == 1) ? N : N * N;
    const int base = line_base<DIM, N>(m, l);
    // velocity components in the line's frame: component 0 is the line
    // direction m, then m+1, m+2 (cyclic), so the flux code below is the
    // direction-0 flux with no per-lane component selection
    int comp[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) comp[c] = (m + c) % DIM;

    Prim<T, DIM> P[N];
    if (has) {
#pragma unroll
      for (int q = 0; q < N; ++q) {
        const int node = base + q * stride;
        const int slot = e * NDP + node + node / N;
        P[q].rho = sp[C::IR * ENP + slot];
#pragma unroll
        for (int d = 0; d < DIM; ++d) P[q].v[d] = sp[(C::IV + comp[d]) * ENP + slot];
        P[q].beta = sp[C::IB * ENP + slot];
        P[q].v2 = sp[C::IV2 * ENP + slot];
      }
    }
    __syncthreads();
    if (has) {
      T acc[N][NV];
#pragma unroll
      for (int q = 0; q < N; ++q)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[q][v] = T(0);

#pragma unroll
      for (int p0 = 0; p0 < N; ++p0) {
#pragma unroll
        for (int p1 = p0 + 1; p1 < N; ++p1) {
          const PairMeans<T> mn =
              pair_means<T, true>(P[p0].rho, P[p1].rho, P[p0].beta, P[p1].beta);
          T F[NV];
          ec_flux_from_means<T, DIM>(0, P[p0], P[p1], mn, half_inv_gm1, F);
          const T d01 = T(mp.D2[p0 * N + p1]), d10 = T(mp.D2[p1 * N + p0]);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            acc[p0][v] += d01 * F[v];
            acc[p1][v] += d10 * F[v];
          }
        }
      }

      const T metric_m = (m == 0) ? T(md.two_over_h[0])
                                  : (m == 1) ? T(md.two_over_h[1]) : T(md.two_over_h[2]);
#pragma unroll
      for (int q = 0; q < N; ++q) {
        const int node = base + q * stride;
        const int slot = e * NDP + node + node / N;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int f = (v == 0 || v == NV - 1) ? v : 1 + comp[v - 1];
          sacc[(m * NV + f) * ENP + slot] = metric_m * acc[q][v];
        }
      }
    }
  }
  __syncthreads();

  // ---- phase 1b: face tasks (one interface flux each) ----
  // Task (line, side): side 0 is the line's -m face (the -m neighbour's last
  // node | own first node), side 1 its +m face (own last node | the +m
  // neighbour's first node).  Every face goes through this one loop body (not
  // unrolled) with the same operand order on both elements that share it, so
  // both compute a bit-identical f* and the scheme stays conservative to
  // round-off of the sums.  Kept apart from the volume pairs, neither phase
  // holds the other's registers.
  {
    const T lam_scale = T(mp.lambda_scale);
    const T iw = T(mp.inv_w_end);
#pragma unroll 1
    for (int ft = tid; ft < E * 2 * G::TASKS; ft += TH) {
      // all -m faces first, then all +m faces: neighbouring lanes take
      // neighbouring lines (coalesced trace loads)
      const int side = ft >= E * G::TASKS;
      const int task = side ? ft - E * G::TASKS : ft;
      const int e = task / G::TASKS;
      const int r = task - e * G::TASKS;
      const int m = r / G::NL;
      const int l = r - m * G::NL;
      const int k = k0 + e;
      if (k >= md.ne) continue;
      const int stride = (m == 0) ? 1 : (m == 1) ? N : N * N;
      const int base = line_base<DIM, N>(m, l);
      int comp[DIM];
#pragma unroll
      for (int c = 0; c < DIM; ++c) comp[c] = (m + c) % DIM;
      const int kn = snbr[e * 2 * DIM + 2 * m + side];
      const int own = base + (side ? (N - 1) * stride : 0);
      const int nbr = base + (side ? 0 : (N - 1) * stride);
      // a boundary face (1-D) takes the exterior state from mp.ubc (Dirichlet)
      // or from the own trace (outflow: f* is then the trace's physical flux)
      const bool bnd = kn < 0;
      const int gL = side ? k * ND + own : (bnd ? 0 : kn * ND + nbr);
      const int gR = side ? (bnd ? 0 : kn * ND + nbr) : k * ND + own;
      T ql[NV], qr[NV], F[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int f = (v == 0 || v == NV - 1) ? v : 1 + comp[v - 1];
        ql[v] = T(a.y[f * Ntot + gL]);
        qr[v] = T(a.y[f * Ntot + gR]);
      }
      if constexpr (DIM == 1) {
        if (bnd) {
          const bool outflow = (side ? mp.bckind[1] : mp.bckind[0]) != 0;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            if (side) qr[v] = outflow ? ql[v] : T(mp.ubc[1][v]);
            else ql[v] = outflow ? qr[v] : T(mp.ubc[0][v]);
          }
        }
      }
      Prim<T, DIM> Pl, Pr;
      T pl, pr;
      prim_from_cons<T, DIM>(ql, gg, Pl, pl);
      prim_from_cons<T, DIM>(qr, gg, Pr, pr);
      interface_flux<T, DIM>(0, Pl, ql, Pr, qr, gg, half_inv_gm1, lam_scale, F);
      const T metric_m = (m == 0) ? T(md.two_over_h[0])
                                  : (m == 1) ? T(md.two_over_h[1]) : T(md.two_over_h[2]);
      const T sg = metric_m * (side ? iw : -iw);
      const int slot = e * NDP + own + own / N;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int f = (v == 0 || v == NV - 1) ? v : 1 + comp[v - 1];
        sacc[(m * NV + f) * ENP + slot] += sg * F[v];
      }
    }
  }
  __syncthreads();

  // ---- phase 2: node epilogue ----
  const double ggd = mp.gg;
  const double inv_gm1d = 1.0 / (ggd - 1.0);
  double dt = 0.0;
  if (a.stage_mode) {
    dt = a.speed_parts ? *s_dt : (a.dt_dev ? *a.dt_dev : a.dt_host);
    // the first stage publishes the step size for the later stages and the update
    if (a.first && k0 == 0 && tid == 0 && a.dt_store) *a.dt_store = dt;
  }
  const bool want_y = a.stage_mode && a.out && a.sc.beta != 0.0;
  const StageExtra* ex = a.stage_mode ? a.ex : nullptr;
  double* const errk = ex ? ex->errk : nullptr;
  double* const errv = ex ? ex->err : nullptr;
  const bool want_uold = a.stage_mode && (a.out || errk || a.phi0);
  const bool want_psi = a.stage_mode && a.phi0 && !a.first;
  const bool want_du = a.stage_mode && !a.first;
  // Per node of this thread: the entropy-rate term, the phi_k(0) term and the
  // weighted squared error (last stage of an error-controlled step), each
  // summed per element after the loop.  When an element's nodes are a
  // power-of-two segment of a wave the sums are butterfly shuffles within the
  // segment; otherwise they go through LDS.
  constexpr int ITER = (EN + TH - 1) / TH;
  constexpr bool kWaveRed = (ND & (ND - 1)) == 0 && ND <= 64 && TH % 64 == 0;
  // one element per block otherwise (3-D, p >= 4): block-wide sums
  constexpr bool kBlockRed = !kWaveRed && E == 1 && TH % 64 == 0;
  double wdv[ITER], esq[ITER], psi[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) wdv[it] = esq[it] = psi[it] = 0.0;
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int idx = tid + it * TH;
    if (idx >= EN) break;
    const int e = idx / ND;
    const int k = k0 + e;
    if (k >= md.ne) {
      if (!kWaveRed && !kBlockRed) sred[idx] = 0.0;
      continue;
    }
    const int i = idx - e * ND;
    const int slot = e * NDP + i + i / N;
    const int gi = k0 * ND + idx;
    // global operands of the update first (latency hidden by the work below)
    double uo[NV], yv[NV], dp[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      uo[v] = want_uold ? a.u_old[v * Ntot + gi] : 0.0;
      yv[v] = a.y[v * Ntot + gi];
      dp[v] = want_du ? a.du[v * Ntot + gi] : 0.0;
    }
    double kv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T s = T(0);
#pragma unroll
      for (int m = 0; m < DIM; ++m) s += sacc[(m * NV + v) * ENP + slot];
      kv[v] = -double(s);
      if (a.visc) kv[v] += a.visc[v * Ntot + gi];
    }
    // entropy rate w(y).k in FP64, w = [(g - s)/(g-1) - beta |v|^2, 2 beta v,
    // -2 beta] (primitives recomputed from y: their LDS slots now hold the
    // accumulators); not formed when nobody reads it (a step that solves
    // with phi_k(0) from the stages)
    double wdot = 0.0;
    if (a.eta) {
      Prim<double, DIM> P;
      double p;
      prim_from_cons<double, DIM>(yv, ggd, P, p);
      const double lnr = log_d(P.rho), lnb = log_d(P.beta);
      const double s_phys = (1.0 - ggd) * lnr - 0.6931471805599453 - lnb;  // ln p - g ln rho
      wdot = ((ggd - s_phys) * inv_gm1d - P.beta * P.v2) * kv[0];
#pragma unroll
      for (int d = 0; d < DIM; ++d) wdot += 2.0 * P.beta * P.v[d] * kv[1 + d];
      wdot += -2.0 * P.beta * kv[NV - 1];
    }
    double M = 1.0;
    {
      int ii = i;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int im = ii % N;
        ii /= N;
        // select chain: a runtime index into the kernel-argument array would
        // copy the array to scratch memory
        double wq = mp.w[0];
#pragma unroll
        for (int t = 1; t < N; ++t) wq = (im == t) ? mp.w[t] : wq;
        M *= md.half_h[d] * wq;
      }
    }
    wdv[it] = M * wdot;
    if (!kWaveRed && !kBlockRed) sred[idx] = wdv[it];

    if (a.stage_mode) {
      const double cdt = a.sc.c * dt, bdt = a.sc.b * dt;
      const size_t slot_len = (size_t)NV * Ntot;
      if (a.out) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double y = a.sc.alpha * uo[v] + cdt * kv[v];
          if (want_y) y += a.sc.beta * yv[v];
          // general tableaux: the earlier stored slopes of this row
#pragma unroll
          for (int j = 0; j < kMaxPrev; ++j)
            if (ex && j < ex->row.nprev)
              y += (ex->row.prev_a[j] * dt) *
                   ex->kst[ex->row.prev_slot[j] * slot_len + (size_t)v * Ntot + gi];
          a.out[v * Ntot + gi] = y;
        }
      }
      if (ex && ex->row.kstore > 0) {
        double* ks = ex->kst + (size_t)(ex->row.kstore - 1) * slot_len;
#pragma unroll
        for (int v = 0; v < NV; ++v) ks[(size_t)v * Ntot + gi] = kv[v];
      }
      double dn[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        dn[v] = dp[v] + bdt * kv[v];
        a.du[v * Ntot + gi] = dn[v];
      }
      if (want_psi) {
        // this node's part of phi_k(0): M (w(u_old) - w(y)).k
        double dw[NV];
        entropy_var_change<DIM>(uo, yv, ggd, inv_gm1d, dw);
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) s += dw[v] * kv[v];
        psi[it] = -M * s;
      }
      if (errv) {
        const double edt = ex->row.ecoef * dt;
        const double atol = ex->atol, rtol = ex->rtol;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double ev = (a.first ? 0.0 : errv[v * Ntot + gi]) + edt * kv[v];
          errv[v * Ntot + gi] = ev;
          if (errk) {
            const double sc = atol + rtol * fmax(fabs(uo[v]), fabs(uo[v] + dn[v]));
            const double q = ev / sc;
            esq[it] += q * q;
          }
        }
      }
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) a.out[v * Ntot + gi] = kv[v];
    }
  }
  if constexpr (kWaveRed) {
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      double s = wdv[it], sp = psi[it], se = esq[it];
#pragma unroll
      for (int off = ND / 2; off >= 1; off /= 2) {
        s += __shfl_xor(s, off, 64);
        if (a.stage_mode && a.phi0) sp += __shfl_xor(sp, off, 64);
        if (errk) se += __shfl_xor(se, off, 64);
      }
      const int idx = tid + it * TH;
      const int k = k0 + idx / ND;
      if (idx < EN && idx % ND == 0 && k < md.ne) {
        if (a.eta) {
          if (a.stage_mode)
            a.eta[k] = (a.first ? 0.0 : a.eta[k]) + a.sc.b * dt * s;
          else
            a.eta[k] = s;
        }
        if (a.stage_mode && a.phi0) a.phi0[k] = (a.first ? 0.0 : a.phi0[k]) + a.sc.b * dt * sp;
        if (errk) errk[k] = se;
      }
    }
    return;
  }
  if constexpr (kBlockRed) {
    // per thread in a fixed order, then butterfly shuffles within each wave,
    // then the waves' partials in LDS summed by thread 0 in wave order
    double s = 0.0, sp = 0.0, se = 0.0;
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      s += wdv[it];
      sp += psi[it];
      se += esq[it];
    }
#pragma unroll
    for (int off = 32; off >= 1; off /= 2) {
      s += __shfl_xor(s, off, 64);
      sp += __shfl_xor(sp, off, 64);
      se += __shfl_xor(se, off, 64);
    }
    constexpr int NW = TH / 64;
    static_assert(3 * NW <= EN, "wave partials fit the reduction buffer");
    const int wave = tid >> 6;
    if ((tid & 63) == 0) {
      sred[3 * wave] = s;
      sred[3 * wave + 1] = sp;
      sred[3 * wave + 2] = se;
    }
    __syncthreads();
    if (tid == 0 && k0 < md.ne) {
      double ts = 0.0, tp = 0.0, te = 0.0;
      for (int w = 0; w < NW; ++w) {
        ts += sred[3 * w];
        tp += sred[3 * w + 1];
        te += sred[3 * w + 2];
      }
      const int k = k0;
      if (a.eta) {
        if (a.stage_mode)
          a.eta[k] = (a.first ? 0.0 : a.eta[k]) + a.sc.b * dt * ts;
        else
          a.eta[k] = ts;
      }
      if (a.stage_mode && a.phi0) a.phi0[k] = (a.first ? 0.0 : a.phi0[k]) + a.sc.b * dt * tp;
      if (errk) errk[k] = te;
    }
    return;
  }
  __syncthreads();
  if (tid < E) {
    const int k = k0 + tid;
    if (k < md.ne && a.eta) {
      double s = 0.0;
      for (int i = 0; i < ND; ++i) s += sred[tid * ND + i];
      if (a.stage_mode) {
        const double prev = a.first ? 0.0 : a.eta[k];
        a.eta[k] = prev + a.sc.b * dt * s;
      } else {
        a.eta[k] = s;
      }
    }
  }
  if (a.stage_mode && a.phi0) {
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int idx = tid + it * TH;
      if (idx < EN) sred[idx] = psi[it];
    }
    __syncthreads();
    if (tid < E) {
      const int k = k0 + tid;
      if (k < md.ne) {
        double s = 0.0;
#pragma unroll 8
        for (int i = 0; i < ND; ++i) s += sred[tid * ND + i];
        a.phi0[k] = (a.first ? 0.0 : a.phi0[k]) + a.sc.b * dt * s;
      }
    }
  }
  if (errk) {
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int idx = tid + it * TH;
      if (idx < EN) sred[idx] = esq[it];
    }
    __syncthreads();
    if (tid < E) {
      const int k = k0 + tid;
      if (k < md.ne) {
        double s = 0.0;
#pragma unroll 8
        for (int i = 0; i < ND; ++i) s += sred[tid * ND + i];
        errk[k] = s;
      }
    }
  }
}


template <int DIM, int N, typename T>
__global__ void __launch_bounds__((RhsShape<DIM, N, T, RhsCfg<DIM, N, T>::E>::THREADS))
#if ESRK_RHS_WAVES_PER_EU > 0
    __attribute__((amdgpu_waves_per_eu(ESRK_RHS_WAVES_PER_EU)))
#endif
    rhs_kernel(const MeshParams mp, const RhsArgs a) {
  constexpr int E = RhsCfg<DIM, N, T>::E;
  using S = RhsShape<DIM, N, T, E>;
  __shared__ T sbuf[S::SBUF];
  __shared__ double sred[S::EN];
  __shared__ int snbr[E * 2 * DIM];
  __shared__ double s_dt;
  // mesh sizes in LDS: the direction-dependent lookups (metric, elements per
  // direction) become LDS reads instead of a private copy in scratch memory
  __shared__ MeshDims smd;
  if (threadIdx.x == 0) smd = dims_of(mp);
  __syncthreads();
  // FP32 flux: XCD-contiguous elements (measured 1.5 % faster on 16^3 p3 and
  // 6 % on 32^3 p3); FP64: launch order (the remap measured 1-2 % slower)
  const int blk = sizeof(T) == 4 ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  rhs_block<DIM, N, T, E>(mp, smd, a, blk * E, sbuf, sbuf, sred, &s_dt, snbr);
}

// Batched form: the blocks walk a work list of (simulation, first element)
// items of many simulations sharing degree and physics but not mesh size.
// Pointers in a0 point at the packed batch arrays; per-simulation offsets
// come from sims[].
template <int DIM, int N, typename T, int E>
__global__ void __launch_bounds__((RhsShape<DIM, N, T, E>::THREADS))
    rhs_batch_kernel(const MeshParams mp, const RhsArgs a0, const SimParams* __restrict__ sims,
                     const int2* __restrict__ items, int nitems, double* dt_sims,
                     const double* dt_sims_in) {
  using S = RhsShape<DIM, N, T, E>;
  __shared__ T sbuf[S::SBUF];
  __shared__ double sred[S::EN];
  __shared__ int snbr[E * 2 * DIM];
  __shared__ double s_dt;
  __shared__ MeshDims smd;
  // One work item per block, no loop over items: a block-stride loop here let
  // the compiler hoist the FP64 series constants and argument pointers into
  // vector registers for the whole loop (+80 VGPRs, half the occupancy).  The
  // items are sorted large-first, so the dispatcher still balances the
  // uneven simulations.
  {
    const int it = blockIdx.x;
    if (it >= nitems) return;
    // the item is the same for the whole block: keep it (and everything
    // derived from it: offsets, pointers, mesh sizes) in scalar registers
    int2 w = items[it];
    w.x = __builtin_amdgcn_readfirstlane(w.x);
    w.y = __builtin_amdgcn_readfirstlane(w.y);
    const SimParams& P = sims[w.x];
    if (threadIdx.x == 0) smd = P.md;
    __syncthreads();
    RhsArgs a = a0;
    a.y = a0.y + P.base;
    a.u_old = a0.u_old ? a0.u_old + P.base : nullptr;
    a.out = a0.out ? a0.out + P.base : nullptr;
    a.du = a0.du ? a0.du + P.base : nullptr;
    a.eta = a0.eta ? a0.eta + P.elem_base : nullptr;
    a.phi0 = a0.phi0 ? a0.phi0 + P.elem_base : nullptr;
    a.speed_parts = a0.speed_parts ? a0.speed_parts + P.speed_p0 : nullptr;
    a.n_speed_parts = P.speed_p1 - P.speed_p0;
    a.dt_dev = dt_sims_in ? dt_sims_in + w.x : nullptr;
    a.dt_store = dt_sims ? dt_sims + w.x : nullptr;
    a.elem_base = P.elem_base;
    rhs_block<DIM, N, T, E>(mp, smd, a, w.y, sbuf, sbuf, sred, &s_dt, snbr);
    __syncthreads();
  }
}

template <int DIM, int N, typename T>
static hipError_t launch_one(const MeshParams& mp, const RhsArgs& a, hipStream_t s) {
  constexpr int E = RhsCfg<DIM, N, T>::E;
  const int blocks = (mp.ne + E - 1) / E;
  hipLaunchKernelGGL((rhs_kernel<DIM, N, T>), dim3(blocks), dim3(RhsShape<DIM, N, T, E>::THREADS),
                     0, s, mp, a);
  return hipGetLastError();
}

template <int DIM, typename T>
static hipError_t launch_dim(const MeshParams& mp, const RhsArgs& a, hipStream_t s) {
  switch (mp.n) {
    case 2: return launch_one<DIM, 2, T>(mp, a, s);
    case 3: return launch_one<DIM, 3, T>(mp, a, s);
    case 4: return launch_one<DIM, 4, T>(mp, a, s);
    case 5: return launch_one<DIM, 5, T>(mp, a, s);
    case 6: return launch_one<DIM, 6, T>(mp, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rhs(const MeshParams& mp, int precision, const RhsArgs& a, hipStream_t s) {
  if (precision == ESRK_FP64) {
    if (mp.dim == 1) return launch_dim<1, double>(mp, a, s);
    if (mp.dim == 2) return launch_dim<2, double>(mp, a, s);
    if (mp.dim == 3) return launch_dim<3, double>(mp, a, s);
  } else {
    if (mp.dim == 1) return launch_dim<1, float>(mp, a, s);
    if (mp.dim == 2) return launch_dim<2, float>(mp, a, s);
    if (mp.dim == 3) return launch_dim<3, float>(mp, a, s);
  }
  return hipErrorInvalidValue;
}

// ---- batched launch: tile = elements per block (0 = the default for (DIM, N)) ----
template <int DIM, int N, typename T, int E>
static hipError_t batch_one(const MeshParams& mp, const RhsArgs& a, const SimParams* sims,
                            const int2* items, int nitems, double* dt_sims,
                            const double* dt_in, int grid, hipStream_t s) {
  (void)grid;  // one block per item
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL((rhs_batch_kernel<DIM, N, T, E>), dim3(nitems),
                     dim3(RhsShape<DIM, N, T, E>::THREADS), 0, s, mp, a, sims, items, nitems,
                     dt_sims, dt_in);
  return hipGetLastError();
}

template <int DIM, int N, typename T>
static hipError_t batch_tile(const MeshParams& mp, int tile, const RhsArgs& a,
                             const SimParams* sims, const int2* items, int nitems,
                             double* dt_sims, const double* dt_in, int grid, hipStream_t s) {
  constexpr int E0 = RhsCfg<DIM, N, T>::E;
  constexpr int EH = E0 / 2 > 0 ? E0 / 2 : 1;
  constexpr int ED = (RhsCfg<DIM, N, T>::LDS_PER_ELEM * 2 * E0 <= 64 * 1024) ? 2 * E0 : E0;
  if (tile == 0 || tile == E0)
    return batch_one<DIM, N, T, E0>(mp, a, sims, items, nitems, dt_sims, dt_in, grid, s);
  if (tile == EH)
    return batch_one<DIM, N, T, EH>(mp, a, sims, items, nitems, dt_sims, dt_in, grid, s);
  if (tile == ED)
    return batch_one<DIM, N, T, ED>(mp, a, sims, items, nitems, dt_sims, dt_in, grid, s);
  return hipErrorInvalidValue;
}

template <int DIM, int N, typename T>
static void tiles_of(int* out) {
  constexpr int E0 = RhsCfg<DIM, N, T>::E;
  out[0] = E0 / 2 > 0 ? E0 / 2 : 1;
  out[1] = E0;
  out[2] = (RhsCfg<DIM, N, T>::LDS_PER_ELEM * 2 * E0 <= 64 * 1024) ? 2 * E0 : E0;
}

// Candidate tiles (elements per block) of the batched stage kernel; the
// middle one is the default.  Batching is compiled for 2-D meshes.
int rhs_batch_tiles(const MeshParams& mp, int precision, int* out) {
  if (mp.dim != 2) return 0;
#define ESRK_TILES(T)                              \
  switch (mp.n) {                                  \
    case 2: tiles_of<2, 2, T>(out); return 3;      \
    case 3: tiles_of<2, 3, T>(out); return 3;      \
    case 4: tiles_of<2, 4, T>(out); return 3;      \
    case 5: tiles_of<2, 5, T>(out); return 3;      \
    case 6: tiles_of<2, 6, T>(out); return 3;      \
  }
  if (precision == ESRK_FP64) { ESRK_TILES(double) } else { ESRK_TILES(float) }
#undef ESRK_TILES
  return 0;
}

hipError_t launch_rhs_batch(const MeshParams& mp, int precision, int tile, const RhsArgs& a,
                            const SimParams* sims, const int2* items, int nitems,
                            double* dt_sims, const double* dt_in, int grid, hipStream_t s) {
  if (mp.dim != 2) return hipErrorInvalidValue;
#define ESRK_BT(T)                                                                               \
  switch (mp.n) {                                                                                \
    case 2: return batch_tile<2, 2, T>(mp, tile, a, sims, items, nitems, dt_sims, dt_in, grid, s); \
    case 3: return batch_tile<2, 3, T>(mp, tile, a, sims, items, nitems, dt_sims, dt_in, grid, s); \
    case 4: return batch_tile<2, 4, T>(mp, tile, a, sims, items, nitems, dt_sims, dt_in, grid, s); \
    case 5: return batch_tile<2, 5, T>(mp, tile, a, sims, items, nitems, dt_sims, dt_in, grid, s); \
    case 6: return batch_tile<2, 6, T>(mp, tile, a, sims, items, nitems, dt_sims, dt_in, grid, s); \
  }
  if (precision == ESRK_FP64) { ESRK_BT(double) } else { ESRK_BT(float) }
#undef ESRK_BT
  return hipErrorInvalidValue;
}

}  // namespace esrk
