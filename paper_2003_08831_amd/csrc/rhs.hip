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
// node primitives (rho, v, beta = rho/2p, ln rho, ln beta, |v|^2, c) in LDS
// with coalesced SoA loads.  Phase 1: one thread per (element, direction,
// line) evaluates every unordered node pair of its line once (symmetric flux,
// scattered to both nodes with 2 D_ab and 2 D_ba) plus the two interface fluxes
// at the line ends, and writes the line's contribution to a per-direction LDS
// accumulator.  Phase 2: one thread per node sums the directions, writes the
// outputs and the per-element entropy-rate partials.
#include "device_math.h"
#include "internal.h"

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
  static constexpr int NP = DIM + 6;
  static constexpr int IR = 0, IV = 1, IB = DIM + 1, ILR = DIM + 2, ILB = DIM + 3,
                       IV2 = DIM + 4, IC = DIM + 5;
  static constexpr int LDS_PER_ELEM =
      G::ND * (int)((NP + DIM * G::NV) * sizeof(T) + sizeof(double));
  static constexpr int BUDGET = 64 * 1024;
  static constexpr int E_TASK = (256 / G::TASKS) > 0 ? 256 / G::TASKS : 1;
  static constexpr int E_LDS = (BUDGET / LDS_PER_ELEM) > 0 ? BUDGET / LDS_PER_ELEM : 1;
  static constexpr int E = E_TASK < E_LDS ? E_TASK : E_LDS;
  static constexpr int RAW = E * G::TASKS;
  static constexpr int THREADS = ((RAW < 64 ? 64 : RAW) + 63) / 64 * 64;
};

__device__ __forceinline__ void latch(DevScalars* s, int code, long long elem) {
  atomicCAS(&s->status, 0, code);
  atomicMin((unsigned long long*)&s->bad_elem, (unsigned long long)elem);
}

template <int DIM>
__device__ __forceinline__ int neighbour(const MeshParams& mp, int k, int m, int dir) {
  int c[3];
  c[0] = k % mp.nel[0];
  c[1] = (k / mp.nel[0]) % mp.nel[1];
  c[2] = k / (mp.nel[0] * mp.nel[1]);
  int cm = (m == 0) ? c[0] : (m == 1) ? c[1] : c[2];
  const int nm = (m == 0) ? mp.nel[0] : (m == 1) ? mp.nel[1] : mp.nel[2];
  cm += dir;
  cm = (cm < 0) ? cm + nm : (cm >= nm ? cm - nm : cm);
  if (m == 0) c[0] = cm;
  if (m == 1) c[1] = cm;
  if (m == 2) c[2] = cm;
  return c[0] + mp.nel[0] * (c[1] + mp.nel[1] * c[2]);
}

// Interface flux f* in direction m between left state qL and right state qR.
template <typename T, int DIM>
__device__ __forceinline__ void interface_flux(int m, const T* qL, const T* qR, T gg,
                                               T half_inv_gm1, T lam_scale, T* F) {
  Prim<T, DIM> A, B;
  T pA, pB;
  prim_from_cons<T, DIM>(qL, gg, A, pA);
  prim_from_cons<T, DIM>(qR, gg, B, pB);
  const T rho_ln = logmean_direct(A.rho, B.rho);
  const T ibl = inv_logmean_direct(A.beta, B.beta);
  ec_flux_from_means<T, DIM>(m, A, B, rho_ln, ibl, half_inv_gm1, F);
  T vA = A.v[0], vB = B.v[0];
#pragma unroll
  for (int k = 1; k < DIM; ++k) {
    vA = (m == k) ? A.v[k] : vA;
    vB = (m == k) ? B.v[k] : vB;
  }
  const T cA = sqrt(gg * pA / A.rho), cB = sqrt(gg * pB / B.rho);
  const T sA = fabs(vA) + cA, sB = fabs(vB) + cB;
  const T lam = sA > sB ? sA : sB;
  const T hl = T(0.5) * lam_scale * lam;
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) F[v] -= hl * (qR[v] - qL[v]);
}

template <int DIM, int N, typename T>
__global__ void __launch_bounds__((RhsCfg<DIM, N, T>::THREADS))
    rhs_kernel(const MeshParams mp, const RhsArgs a) {
  using C = RhsCfg<DIM, N, T>;
  using G = Geo<DIM, N>;
  constexpr int ND = G::ND, NV = G::NV, NP = C::NP, E = C::E, EN = E * ND;
  constexpr int TH = C::THREADS;
  __shared__ T sp[NP * EN];
  __shared__ T sacc[DIM * NV * EN];
  __shared__ double sred[EN];

  const int tid = threadIdx.x;
  const int k0 = blockIdx.x * E;
  const long long Ntot = (long long)mp.ne * ND;
  const T gg = T(mp.gg);
  const T half_inv_gm1 = T(0.5) / (gg - T(1));

  // CFL step size of the first stage, from the wave-speed partials of the step
  // start state (max is exact, so every block derives the same dt).
  __shared__ double s_dt;
  if (a.stage_mode && a.speed_parts && tid < 64) {
    double mx = 0.0;
    for (int q = tid; q < kSpeedBlocks; q += 64) mx = fmax(mx, a.speed_parts[q]);
#pragma unroll
    for (int off = 32; off >= 1; off /= 2) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (tid == 0) s_dt = mp.cfl * mp.hmin / (double(mp.n) * mx);
  }

  // ---- phase 0: node primitives into LDS ----
  for (int idx = tid; idx < EN; idx += TH) {
    const int e = idx / ND;
    const int k = k0 + e;
    T q[NV];
    if (k < mp.ne) {
      const long long gi = (long long)k0 * ND + idx;
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
      if (k < mp.ne) latch(a.scal, ESRK_ENONPHYS, k);
      P.rho = T(1);
      p = T(1);
      P.beta = T(0.5);
    }
    sp[C::IR * EN + idx] = P.rho;
#pragma unroll
    for (int d = 0; d < DIM; ++d) sp[(C::IV + d) * EN + idx] = P.v[d];
    sp[C::IB * EN + idx] = P.beta;
    sp[C::ILR * EN + idx] = log(P.rho);
    sp[C::ILB * EN + idx] = log(P.beta);
    sp[C::IV2 * EN + idx] = P.v2;
    sp[C::IC * EN + idx] = sqrt(gg * p / P.rho);
  }
  __syncthreads();

  // ---- phase 1: line tasks (volume pairs + the two interface fluxes) ----
  for (int task = tid; task < E * G::TASKS; task += TH) {
    const int e = task / G::TASKS;
    const int r = task - e * G::TASKS;
    const int m = r / G::NL;
    const int l = r - m * G::NL;
    const int k = k0 + e;
    if (k >= mp.ne) continue;
    const int stride = (m == 0) ? 1 : (m == 1) ? N : N * N;
    const int base = (l % stride) + (l / stride) * stride * N;
    const int eo = e * ND;

    Prim<T, DIM> P[N];
    T lr[N], lb[N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const int idx = eo + base + q * stride;
      P[q].rho = sp[C::IR * EN + idx];
#pragma unroll
      for (int d = 0; d < DIM; ++d) P[q].v[d] = sp[(C::IV + d) * EN + idx];
      P[q].beta = sp[C::IB * EN + idx];
      P[q].v2 = sp[C::IV2 * EN + idx];
      lr[q] = sp[C::ILR * EN + idx];
      lb[q] = sp[C::ILB * EN + idx];
    }
    T acc[N][NV];
#pragma unroll
    for (int q = 0; q < N; ++q)
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[q][v] = T(0);

#pragma unroll
    for (int p0 = 0; p0 < N; ++p0) {
#pragma unroll
      for (int p1 = p0 + 1; p1 < N; ++p1) {
        const T rho_ln = logmean(P[p0].rho, P[p1].rho, lr[p0] - lr[p1]);
        const T ibl = inv_logmean(P[p0].beta, P[p1].beta, lb[p0] - lb[p1]);
        T F[NV];
        ec_flux_from_means<T, DIM>(m, P[p0], P[p1], rho_ln, ibl, half_inv_gm1, F);
        const T d01 = T(mp.D2[p0 * N + p1]), d10 = T(mp.D2[p1 * N + p0]);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          acc[p0][v] += d01 * F[v];
          acc[p1][v] += d10 * F[v];
        }
      }
    }

    // interface fluxes at both ends of the line
    const T lam_scale = T(mp.lambda_scale);
    const T iw = T(mp.inv_w_end);
    {
      const int kn = neighbour<DIM>(mp, k, m, -1);
      const long long gin = (long long)kn * ND + base + (N - 1) * stride;
      const long long gio = (long long)k * ND + base;
      T qL[NV], qR[NV], F[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        qL[v] = T(a.y[v * Ntot + gin]);
        qR[v] = T(a.y[v * Ntot + gio]);
      }
      interface_flux<T, DIM>(m, qL, qR, gg, half_inv_gm1, lam_scale, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[0][v] -= iw * F[v];
    }
    {
      const int kn = neighbour<DIM>(mp, k, m, +1);
      const long long gin = (long long)kn * ND + base;
      const long long gio = (long long)k * ND + base + (N - 1) * stride;
      T qL[NV], qR[NV], F[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        qL[v] = T(a.y[v * Ntot + gio]);
        qR[v] = T(a.y[v * Ntot + gin]);
      }
      interface_flux<T, DIM>(m, qL, qR, gg, half_inv_gm1, lam_scale, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[N - 1][v] += iw * F[v];
    }

    const T metric = T(mp.two_over_h[0]);
    const T metric_m = (m == 0) ? metric
                                : (m == 1) ? T(mp.two_over_h[1]) : T(mp.two_over_h[2]);
#pragma unroll
    for (int q = 0; q < N; ++q) {
      const int idx = eo + base + q * stride;
#pragma unroll
      for (int v = 0; v < NV; ++v) sacc[(m * NV + v) * EN + idx] = metric_m * acc[q][v];
    }
  }
  __syncthreads();

  // ---- phase 2: node epilogue ----
  const double ggd = mp.gg;
  double dt = 0.0;
  if (a.stage_mode) {
    dt = a.speed_parts ? s_dt : (a.dt_dev ? *a.dt_dev : a.dt_host);
    // the first stage publishes the step size for the later stages and the update
    if (a.first && blockIdx.x == 0 && tid == 0) a.scal->dt = dt;
  }
  for (int idx = tid; idx < EN; idx += TH) {
    const int e = idx / ND;
    const int k = k0 + e;
    if (k >= mp.ne) {
      sred[idx] = 0.0;
      continue;
    }
    const int i = idx - e * ND;
    const long long gi = (long long)k0 * ND + idx;
    double kv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T s = T(0);
#pragma unroll
      for (int m = 0; m < DIM; ++m) s += sacc[(m * NV + v) * EN + idx];
      kv[v] = -double(s);
    }
    // entropy variables in FP64: w = [(g - s)/(g-1) - beta |v|^2, 2 beta v, -2 beta]
    double rho, beta, v2, lnr, lnb, vel[DIM];
    if constexpr (sizeof(T) == sizeof(double)) {
      rho = sp[C::IR * EN + idx];
      beta = sp[C::IB * EN + idx];
      v2 = sp[C::IV2 * EN + idx];
      lnr = sp[C::ILR * EN + idx];
      lnb = sp[C::ILB * EN + idx];
#pragma unroll
      for (int d = 0; d < DIM; ++d) vel[d] = sp[(C::IV + d) * EN + idx];
    } else {
      double q[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v] = a.y[v * Ntot + gi];
      Prim<double, DIM> P;
      double p;
      prim_from_cons<double, DIM>(q, ggd, P, p);
      rho = P.rho;
      beta = P.beta;
      v2 = P.v2;
      lnr = log(rho);
      lnb = log(beta);
#pragma unroll
      for (int d = 0; d < DIM; ++d) vel[d] = P.v[d];
    }
    (void)rho;
    const double s_phys = (1.0 - ggd) * lnr - 0.6931471805599453 - lnb;  // ln p - g ln rho
    double wdot = ((ggd - s_phys) / (ggd - 1.0) - beta * v2) * kv[0];
#pragma unroll
    for (int d = 0; d < DIM; ++d) wdot += 2.0 * beta * vel[d] * kv[1 + d];
    wdot += -2.0 * beta * kv[NV - 1];
    double M = 1.0;
    {
      int ii = i;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int im = ii % N;
        ii /= N;
        M *= mp.half_h[d] * mp.w[im];
      }
    }
    sred[idx] = M * wdot;

    if (a.stage_mode) {
      const double cdt = a.sc.c * dt, bdt = a.sc.b * dt;
      if (a.out) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double y = a.sc.alpha * a.u_old[v * Ntot + gi] + cdt * kv[v];
          if (a.sc.beta != 0.0) y += a.sc.beta * a.y[v * Ntot + gi];
          a.out[v * Ntot + gi] = y;
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double prev = a.first ? 0.0 : a.du[v * Ntot + gi];
        a.du[v * Ntot + gi] = prev + bdt * kv[v];
      }
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) a.out[v * Ntot + gi] = kv[v];
    }
  }
  __syncthreads();
  if (tid < E) {
    const int k = k0 + tid;
    if (k < mp.ne && a.eta) {
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
}

template <int DIM, int N, typename T>
static hipError_t launch_one(const MeshParams& mp, const RhsArgs& a, hipStream_t s) {
  using C = RhsCfg<DIM, N, T>;
  const int blocks = (mp.ne + C::E - 1) / C::E;
  hipLaunchKernelGGL((rhs_kernel<DIM, N, T>), dim3(blocks), dim3(C::THREADS), 0, s, mp, a);
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

}  // namespace esrk
