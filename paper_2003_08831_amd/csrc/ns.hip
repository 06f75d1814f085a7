// BR1 viscous terms of the Navier-Stokes right-hand side (Sec. 3.1, the
// element equation: the viscous volume term built from the entropy-variable
// gradients theta_j and the viscous SAT; BR1 form with central interface values).
//
//   theta_m = (2/h_m) [ D w along m + (1/w_p) (w+ - w)/2 on the +m face
//                                   - (1/w_0) (w- - w)/2 on the -m face ]
//   g_m     = viscous flux from u and theta (chain rule: v_k = -w_{1+k}/w_E,
//             T = -1/(R w_E); constant mu, Stokes hypothesis, kappa = mu c_p / Pr)
//   Visc    = sum_m (2/h_m) [ D g_m along m + the same central lifts of g_m ]
//   diss_k  = sum_i M_i sum_m theta_m,i . g_m,i   (>= 0)
//
// Two kernels, one element per block and one thread per node:
//   grad_kernel : w at the element's nodes into LDS, w of the face neighbours in
//                 registers, theta for every node -> theta buffer (T precision);
//   visc_kernel : g_m at the element's nodes into LDS (from u and theta), g_m of
//                 the face neighbours in registers, Visc -> visc buffer (FP64) and
//                 the element's viscous entropy dissipation.
// The fused stage kernel adds the visc buffer to the inviscid right-hand side.
#include "device_math.h"
#include "internal.h"

namespace esrk {

template <int DIM, int N>
struct NsGeo {
  static constexpr int ND = (DIM == 1) ? N : (DIM == 2) ? N * N : N * N * N;
  static constexpr int NV = DIM + 2;
  // elements per block: fill about one wavefront with nodes
  static constexpr int E = (64 / ND) > 0 ? 64 / ND : 1;
  static constexpr int RAW = E * ND;
  static constexpr int THREADS = ((RAW + 63) / 64) * 64;
};

template <int DIM>
__device__ __forceinline__ int ns_neighbour(const MeshParams& mp, int k, int m, int dir) {
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

// entropy variables w(u) = [(g - s)/(g-1) - rho|v|^2/(2p), rho v/p, -rho/p],
// s = ln p - g ln rho
template <typename T, int DIM>
__device__ __forceinline__ void entropy_vars(const T* q, T gg, T* w) {
  const T rho = q[0];
  const T inv = rcp(rho);
  T v2 = T(0), vel[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    vel[k] = q[1 + k] * inv;
    v2 += vel[k] * vel[k];
  }
  const T p = (gg - T(1)) * (q[DIM + 1] - T(0.5) * rho * v2);
  const T rp = rho * rcp(p);  // rho / p = 2 beta
  const T s = log(p) - gg * log(rho);
  w[0] = (gg - s) * rcp(gg - T(1)) - T(0.5) * rp * v2;
#pragma unroll
  for (int k = 0; k < DIM; ++k) w[1 + k] = rp * vel[k];
  w[DIM + 1] = -rp;
}

// Viscous flux g_m at one node from its state q and gradients th[m'][v].
template <typename T, int DIM>
__device__ __forceinline__ void viscous_flux(const T* q, const T (*th)[DIM + 2], int m, T gg,
                                             T R, T mu, T kappa, T* g) {
  constexpr int NV = DIM + 2;
  const T rho = q[0];
  const T inv = rcp(rho);
  T vel[DIM], v2 = T(0);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    vel[k] = q[1 + k] * inv;
    v2 += vel[k] * vel[k];
  }
  const T p = (gg - T(1)) * (q[NV - 1] - T(0.5) * rho * v2);
  const T wE = -rho * rcp(p);
  const T iwE = rcp(wE);
  // dv[k][q] = d v_k / d x_q,  dT[q] = d T / d x_q
  T dv[DIM][DIM], dT[DIM];
#pragma unroll
  for (int qd = 0; qd < DIM; ++qd) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) dv[k][qd] = (-th[qd][1 + k] - vel[k] * th[qd][NV - 1]) * iwE;
    dT[qd] = th[qd][NV - 1] * iwE * iwE / R;
  }
  T div = T(0);
#pragma unroll
  for (int k = 0; k < DIM; ++k) div += dv[k][k];
  g[0] = T(0);
  T e = T(0);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    T dkm = dv[k][0], dmk = dv[0][k];
#pragma unroll
    for (int qd = 1; qd < DIM; ++qd) {
      dkm = (m == qd) ? dv[k][qd] : dkm;
      dmk = (m == qd) ? dv[qd][k] : dmk;
    }
    const T tau = mu * (dkm + dmk - ((m == k) ? T(2.0 / 3.0) * div : T(0)));
    g[1 + k] = tau;
    e += tau * vel[k];
  }
  T dTm = dT[0];
#pragma unroll
  for (int qd = 1; qd < DIM; ++qd) dTm = (m == qd) ? dT[qd] : dTm;
  g[NV - 1] = e + kappa * dTm;
}

template <int DIM, int N, typename T>
__global__ void __launch_bounds__((NsGeo<DIM, N>::THREADS))
    grad_kernel(const MeshParams mp, const double* __restrict__ y, T* __restrict__ theta) {
  using G = NsGeo<DIM, N>;
  constexpr int ND = G::ND, NV = G::NV, E = G::E;
  __shared__ T sw[NV * E * ND];
  const int tid = threadIdx.x;
  const int e = tid / ND;
  const int i = tid - e * ND;
  const int k = blockIdx.x * E + e;
  const bool valid = e < E && k < mp.ne;
  const long long Ntot = (long long)mp.ne * ND;
  const T gg = T(mp.gg);
  int im[3] = {0, 0, 0};
  {
    int ii = i;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      im[d] = ii % N;
      ii /= N;
    }
  }
  // own node
  T wo[NV];
  if (valid) {
    T q[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = T(y[v * Ntot + (long long)k * ND + i]);
    entropy_vars<T, DIM>(q, gg, wo);
#pragma unroll
    for (int v = 0; v < NV; ++v) sw[v * E * ND + e * ND + i] = wo[v];
  }
  // face neighbours (central interface value (w_nbr - w)/2 lifted onto the face)
  T lift[DIM][NV];
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int v = 0; v < NV; ++v) lift[d][v] = T(0);
  if (valid) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const bool lo_face = im[d] == 0, hi_face = im[d] == N - 1;
      if (!lo_face && !hi_face) continue;
      const int kn = ns_neighbour<DIM>(mp, k, d, hi_face ? +1 : -1);
      int stride = 1;
#pragma unroll
      for (int q2 = 0; q2 < d; ++q2) stride *= N;
      const int inb = i + (hi_face ? -(N - 1) : (N - 1)) * stride;
      T q[NV], wn[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v] = T(y[v * Ntot + (long long)kn * ND + inb]);
      entropy_vars<T, DIM>(q, gg, wn);
      const T sg = hi_face ? T(mp.inv_w_end) : -T(mp.inv_w_end);
#pragma unroll
      for (int v = 0; v < NV; ++v) lift[d][v] = sg * T(0.5) * (wn[v] - wo[v]);
    }
  }
  __syncthreads();
  if (!valid) return;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    int stride = 1;
#pragma unroll
    for (int q2 = 0; q2 < d; ++q2) stride *= N;
    const int base = i - im[d] * stride;
    const T metric = T(mp.two_over_h[d]);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T s = lift[d][v];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        // D[i_m][j] = half of the stored 2 D table
        const T Dij = T(0.5 * mp.D2[im[d] * N + j]);
        s += Dij * sw[v * E * ND + e * ND + base + j * stride];
      }
      theta[((long long)d * NV + v) * Ntot + (long long)k * ND + i] = metric * s;
    }
  }
}

template <int DIM, int N, typename T>
__global__ void __launch_bounds__((NsGeo<DIM, N>::THREADS))
    visc_kernel(const MeshParams mp, double mu, double kappa, double R,
                const double* __restrict__ y, const T* __restrict__ theta,
                double* __restrict__ visc, double* __restrict__ diss) {
  using G = NsGeo<DIM, N>;
  constexpr int ND = G::ND, NV = G::NV, E = G::E;
  __shared__ T sg[DIM * NV * E * ND];
  __shared__ double sd[E * ND];
  const int tid = threadIdx.x;
  const int e = tid / ND;
  const int i = tid - e * ND;
  const int k = blockIdx.x * E + e;
  const bool valid = e < E && k < mp.ne;
  const long long Ntot = (long long)mp.ne * ND;
  const T gg = T(mp.gg), Tmu = T(mu), Tk = T(kappa), TR = T(R);
  int im[3] = {0, 0, 0};
  {
    int ii = i;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      im[d] = ii % N;
      ii /= N;
    }
  }
  T go[DIM][NV];
  double dsum = 0.0;
  if (valid) {
    T q[NV], th[DIM][NV];
    const long long gi = (long long)k * ND + i;
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = T(y[v * Ntot + gi]);
#pragma unroll
    for (int d = 0; d < DIM; ++d)
#pragma unroll
      for (int v = 0; v < NV; ++v) th[d][v] = theta[((long long)d * NV + v) * Ntot + gi];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      viscous_flux<T, DIM>(q, th, d, gg, TR, Tmu, Tk, go[d]);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        sg[(d * NV + v) * E * ND + e * ND + i] = go[d][v];
        dsum += double(th[d][v]) * double(go[d][v]);
      }
    }
    double M = 1.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) M *= mp.half_h[d] * mp.w[im[d]];
    dsum *= M;
  }
  if (tid < E * ND) sd[tid] = valid ? dsum : 0.0;
  // face neighbours' g_d across face d
  T lift[DIM][NV];
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int v = 0; v < NV; ++v) lift[d][v] = T(0);
  if (valid) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const bool lo_face = im[d] == 0, hi_face = im[d] == N - 1;
      if (!lo_face && !hi_face) continue;
      const int kn = ns_neighbour<DIM>(mp, k, d, hi_face ? +1 : -1);
      int stride = 1;
#pragma unroll
      for (int q2 = 0; q2 < d; ++q2) stride *= N;
      const int inb = i + (hi_face ? -(N - 1) : (N - 1)) * stride;
      const long long gn = (long long)kn * ND + inb;
      T q[NV], th[DIM][NV], gn_d[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v] = T(y[v * Ntot + gn]);
#pragma unroll
      for (int d2 = 0; d2 < DIM; ++d2)
#pragma unroll
        for (int v = 0; v < NV; ++v) th[d2][v] = theta[((long long)d2 * NV + v) * Ntot + gn];
      viscous_flux<T, DIM>(q, th, d, gg, TR, Tmu, Tk, gn_d);
      const T sgn = hi_face ? T(mp.inv_w_end) : -T(mp.inv_w_end);
#pragma unroll
      for (int v = 0; v < NV; ++v) lift[d][v] = sgn * T(0.5) * (gn_d[v] - go[d][v]);
    }
  }
  __syncthreads();
  if (valid) {
    const long long gi = (long long)k * ND + i;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double acc = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        int stride = 1;
#pragma unroll
        for (int q2 = 0; q2 < d; ++q2) stride *= N;
        const int base = i - im[d] * stride;
        T s = lift[d][v];
#pragma unroll
        for (int j = 0; j < N; ++j) {
          const T Dij = T(0.5 * mp.D2[im[d] * N + j]);
          s += Dij * sg[(d * NV + v) * E * ND + e * ND + base + j * stride];
        }
        acc += mp.two_over_h[d] * double(s);
      }
      visc[v * Ntot + gi] = acc;
    }
  }
  if (diss && valid && i == 0) {
    double s = 0.0;
    for (int q2 = 0; q2 < ND; ++q2) s += sd[e * ND + q2];
    diss[k] = s;
  }
}

template <int DIM, int N, typename T>
static hipError_t ns_one(const MeshParams& mp, const NsArgs& a, hipStream_t s) {
  using G = NsGeo<DIM, N>;
  const int blocks = (mp.ne + G::E - 1) / G::E;
  hipLaunchKernelGGL((grad_kernel<DIM, N, T>), dim3(blocks), dim3(G::THREADS), 0, s, mp, a.y,
                     (T*)a.theta);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((visc_kernel<DIM, N, T>), dim3(blocks), dim3(G::THREADS), 0, s, mp, a.mu,
                     a.kappa, a.R, a.y, (const T*)a.theta, a.visc, a.diss);
  return hipGetLastError();
}

template <int DIM, typename T>
static hipError_t ns_dim(const MeshParams& mp, const NsArgs& a, hipStream_t s) {
  switch (mp.n) {
    case 2: return ns_one<DIM, 2, T>(mp, a, s);
    case 3: return ns_one<DIM, 3, T>(mp, a, s);
    case 4: return ns_one<DIM, 4, T>(mp, a, s);
    case 5: return ns_one<DIM, 5, T>(mp, a, s);
    case 6: return ns_one<DIM, 6, T>(mp, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ns(const MeshParams& mp, int precision, const NsArgs& a, hipStream_t s) {
  if (precision == ESRK_FP64) {
    if (mp.dim == 1) return ns_dim<1, double>(mp, a, s);
    if (mp.dim == 2) return ns_dim<2, double>(mp, a, s);
    if (mp.dim == 3) return ns_dim<3, double>(mp, a, s);
  } else {
    if (mp.dim == 1) return ns_dim<1, float>(mp, a, s);
    if (mp.dim == 2) return ns_dim<2, float>(mp, a, s);
    if (mp.dim == 3) return ns_dim<3, float>(mp, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace esrk
