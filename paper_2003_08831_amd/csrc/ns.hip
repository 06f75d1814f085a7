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
//                 registers, theta at every node, then g_m from (u, theta) and
//                 the element's dissipation; g -> flux buffer (T precision);
//   visc_kernel : g_m of the element's nodes into LDS, g_m of the face
//                 neighbours from the buffer, Visc -> visc buffer (FP64); in
//                 FP32 mode the applies D g_m run as one small GEMM per block on
//                 the MFMA units.
// The flux buffer holds g rather than theta: the divergence then reads 5
// values per neighbour face node instead of recomputing g there from u and
// all of theta (20 values).
// The fused stage kernel adds the visc buffer to the inviscid right-hand side.
#include <type_traits>

#include "device_math.h"
#include "internal.h"

// 1: in FP32 mode the derivative applies of the viscous divergence (D g_m
// along each direction m) run on the matrix cores (v_mfma_f32_4x4x1f32, 16
// blocks); 0: VALU loops as in FP64.  The gradient kernel keeps VALU applies:
// with the extra LDS round trip and barrier its MFMA form measured 12-20%
// slower (one apply per field instead of one per field and direction).
#ifndef ESRK_NS_MFMA
#define ESRK_NS_MFMA 1
#endif

namespace esrk {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Derivative applies of one block on the matrix cores (FP32):
//   out[(d NV + v) E ND + e ND + node(d, l, i)]
//       = sum_j D[i][j] in[d * in_dstride + v E ND + e ND + node(d, l, j)]
// for every direction d, field v, element e of the block and line l along d.
// Rows r = ((d NV + v) E + e) NL + l are the GEMM's M dimension, the node j
// along the line its K dimension (one MFMA per j) and the output node i its N
// dimension (groups of 4).  v_mfma_f32_4x4x1f32 with 16 blocks: lane 4b + t
// supplies A = row 64 g + 4b + t and B = D[4 c0 + t][j]; it receives rows
// 64 g + 4b + (0..3) of output column 4 c0 + t.  Every lane of a wave takes
// part (out-of-range rows and columns are zero-padded).  out may equal in
// (with in_dstride = NV E ND the layouts agree): each row is read by its own
// lane before the results of that row are written, and rows are disjoint.
// Value of lane Q of this lane's quad (all four lanes of the quad active).
template <int Q>
__device__ __forceinline__ int quad_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, Q * 0x55, 0xF, 0xF, false);
}

template <int DIM, int N, int E, int NV>
__device__ __forceinline__ void dapply_mfma(const float* in, int in_dstride, float* out,
                                            const double* D2, int nthreads) {
  constexpr int ND = (DIM == 1) ? N : (DIM == 2) ? N * N : N * N * N;
  constexpr int NL = ND / N;
  constexpr int R = DIM * NV * E * NL;
  constexpr int G = (R + 63) / 64;
  constexpr int CG = (N + 3) / 4;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = nthreads >> 6;
  const int t = lane & 3;
  float B[CG][N];
#pragma unroll
  for (int c = 0; c < CG; ++c)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int i = 4 * c + t;
      B[c][j] = i < N ? float(0.5 * D2[i * N + j]) : 0.f;
    }
  for (int g = wave; g < G; g += nw) {
    // this lane's A row: its input line and, for the output, the offset of
    // the line's first node and the node stride (-1: row beyond R)
    const int row = 64 * g + lane;
    float x[N];
    int obase, ostride;
    {
      const bool ok = row < R;
      const int rr = ok ? row : 0;
      const int l = rr % NL;
      const int ev = rr / NL;  // (d NV + v) E + e
      const int e = ev % E;
      const int dv = ev / E;
      const int d = dv / NV, v = dv - d * NV;
      const int stride = (d == 0) ? 1 : (d == 1) ? N : N * N;
      const int base = (l % stride) + (l / stride) * stride * N;
      const float* src = in + d * in_dstride + (v * E + e) * ND + base;
#pragma unroll
      for (int j = 0; j < N; ++j) x[j] = ok ? src[j * stride] : 0.f;
      obase = ok ? ev * ND + base : -1;
      ostride = stride;
    }
    // output row 64 g + (lane & ~3) + q is the A row of quad lane q: its
    // offsets come from that lane by a quad broadcast (DPP quad_perm)
    const int ob[4] = {quad_bcast<0>(obase), quad_bcast<1>(obase), quad_bcast<2>(obase),
                       quad_bcast<3>(obase)};
    const int os[4] = {quad_bcast<0>(ostride), quad_bcast<1>(ostride), quad_bcast<2>(ostride),
                       quad_bcast<3>(ostride)};
#pragma unroll
    for (int c = 0; c < CG; ++c) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < N; ++j) acc = __builtin_amdgcn_mfma_f32_4x4x1f32(x[j], B[c][j], acc, 0, 0, 0);
      const int i = 4 * c + t;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (i < N && ob[q] >= 0) out[ob[q] + i * os[q]] = acc[q];
    }
  }
}

template <int DIM, int N>
struct NsGeo {
  static constexpr int ND = (DIM == 1) ? N : (DIM == 2) ? N * N : N * N * N;
  static constexpr int NV = DIM + 2;
  // elements per block: fill about one wavefront with nodes
  static constexpr int E = (64 / ND) > 0 ? 64 / ND : 1;
  static constexpr int RAW = E * ND;
  static constexpr int THREADS = ((RAW + 63) / 64) * 64;
};

template <typename T>
constexpr bool kUseMfma = ESRK_NS_MFMA && std::is_same<T, float>::value;

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
  const T s = log_d(p) - gg * log_d(rho);
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
    grad_kernel(const MeshParams mp, double mu, double kappa, double R,
                const double* __restrict__ y, T* __restrict__ gflux,
                double* __restrict__ diss) {
  using G = NsGeo<DIM, N>;
  constexpr int ND = G::ND, NV = G::NV, E = G::E;
  __shared__ T sw[NV * E * ND];
  __shared__ double sd[E * ND];
  const int tid = threadIdx.x;
  const int e = tid / ND;
  const int i = tid - e * ND;
  const int k = xcd_block(blockIdx.x, gridDim.x) * E + e;
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
  // own node
  T q[NV], wo[NV];
  if (valid) {
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
      T qn[NV], wn[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) qn[v] = T(y[v * Ntot + (long long)kn * ND + inb]);
      entropy_vars<T, DIM>(qn, gg, wn);
      const T sg = hi_face ? T(mp.inv_w_end) : -T(mp.inv_w_end);
#pragma unroll
      for (int v = 0; v < NV; ++v) lift[d][v] = sg * T(0.5) * (wn[v] - wo[v]);
    }
  }
  __syncthreads();
  double dsum = 0.0;
  if (valid) {
    T th[DIM][NV];
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
        th[d][v] = metric * s;
      }
    }
    const long long gi = (long long)k * ND + i;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      T g[NV];
      viscous_flux<T, DIM>(q, th, d, gg, TR, Tmu, Tk, g);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        gflux[((long long)d * NV + v) * Ntot + gi] = g[v];
        dsum += double(th[d][v]) * double(g[v]);
      }
    }
    double M = 1.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) M *= mp.half_h[d] * mp.w[im[d]];
    dsum *= M;
  }
  if (diss) {
    if constexpr (E == 1) {
      // one element per block: butterfly sums within each wave, then the
      // waves' partials in wave order
      double s = valid ? dsum : 0.0;
#pragma unroll
      for (int off = 32; off >= 1; off /= 2) s += __shfl_xor(s, off, 64);
      if ((tid & 63) == 0) sd[tid >> 6] = s;
      __syncthreads();
      if (tid == 0 && k < mp.ne) {
        double t = 0.0;
        for (int w = 0; w < G::THREADS / 64; ++w) t += sd[w];
        diss[k] = t;
      }
    } else {
      if (tid < E * ND) sd[tid] = valid ? dsum : 0.0;
      __syncthreads();
      if (valid && i == 0) {
        double s = 0.0;
        for (int q2 = 0; q2 < ND; ++q2) s += sd[e * ND + q2];
        diss[k] = s;
      }
    }
  }
}

template <int DIM, int N, typename T>
__global__ void __launch_bounds__((NsGeo<DIM, N>::THREADS))
    visc_kernel(const MeshParams mp, const T* __restrict__ gflux, double* __restrict__ visc) {
  using G = NsGeo<DIM, N>;
  constexpr int ND = G::ND, NV = G::NV, E = G::E;
  __shared__ T sg[DIM * NV * E * ND];
  const int tid = threadIdx.x;
  const int e = tid / ND;
  const int i = tid - e * ND;
  const int k = xcd_block(blockIdx.x, gridDim.x) * E + e;
  const bool valid = e < E && k < mp.ne;
  const long long Ntot = (long long)mp.ne * ND;
  int im[3] = {0, 0, 0};
  {
    int ii = i;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      im[d] = ii % N;
      ii /= N;
    }
  }
  // own g_d into LDS; neighbour g_d across face d: the central lift
  T lift[DIM][NV];
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int v = 0; v < NV; ++v) lift[d][v] = T(0);
  if (valid) {
    const long long gi = (long long)k * ND + i;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      T go[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        go[v] = gflux[((long long)d * NV + v) * Ntot + gi];
        sg[(d * NV + v) * E * ND + e * ND + i] = go[v];
      }
      const bool lo_face = im[d] == 0, hi_face = im[d] == N - 1;
      if (!lo_face && !hi_face) continue;
      const int kn = ns_neighbour<DIM>(mp, k, d, hi_face ? +1 : -1);
      int stride = 1;
#pragma unroll
      for (int q2 = 0; q2 < d; ++q2) stride *= N;
      const int inb = i + (hi_face ? -(N - 1) : (N - 1)) * stride;
      const long long gn = (long long)kn * ND + inb;
      const T sgn = hi_face ? T(mp.inv_w_end) : -T(mp.inv_w_end);
#pragma unroll
      for (int v = 0; v < NV; ++v)
        lift[d][v] = sgn * T(0.5) * (gflux[((long long)d * NV + v) * Ntot + gn] - go[v]);
    }
  }
  __syncthreads();
  if constexpr (kUseMfma<T>) {
    // in place: a row's line values are read (by the lane that owns the row)
    // before its results overwrite them, and rows cover disjoint LDS slots,
    // so the block needs no second LDS buffer (more resident blocks)
    dapply_mfma<DIM, N, E, NV>(sg, NV * E * ND, sg, mp.D2, G::THREADS);
    __syncthreads();
    if (valid) {
      const long long gi = (long long)k * ND + i;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
          acc += mp.two_over_h[d] *
                 double(sg[(d * NV + v) * E * ND + e * ND + i] + lift[d][v]);
        visc[v * Ntot + gi] = acc;
      }
    }
  } else if (valid) {
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
}

template <int DIM, int N, typename T>
static hipError_t ns_one(const MeshParams& mp, const NsArgs& a, hipStream_t s) {
  using G = NsGeo<DIM, N>;
  const int blocks = (mp.ne + G::E - 1) / G::E;
  hipLaunchKernelGGL((grad_kernel<DIM, N, T>), dim3(blocks), dim3(G::THREADS), 0, s, mp, a.mu,
                     a.kappa, a.R, a.y, (T*)a.flux, a.diss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((visc_kernel<DIM, N, T>), dim3(blocks), dim3(G::THREADS), 0, s, mp,
                     (const T*)a.flux, a.visc);
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
