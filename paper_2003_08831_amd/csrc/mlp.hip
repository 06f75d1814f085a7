// Small network proposing each element's relaxation parameter (the learned
// extension of the relaxation solve of Sec. 2; the root solve always runs to
// the same tolerance, so the network only picks a trial point).
//
// Network 5 -> 32 -> 32 -> 1 with tanh hidden layers, FP32.  Model vector:
//   W1[32][5] @0, b1[32] @160, W2[32][32] @192, b2[32] @1216, w3[32] @1248,
//   b3 @1280  (1281 trained parameters), then the fixed normalization
//   scale[5] @1281, mean[5] @1286, std[5] @1291, out_mean @1296, out_std @1297.
// Features of an element (raw): r = [deta, eta(u_new) - eta(u_old), dt,
//   max wave speed, dt * viscous dissipation]; network input
//   x_j = (asinh(r_j / scale_j) - mean_j) / std_j; output y gives
//   gamma_guess = 1 + dt^2 (out_mean + out_std y).
//
// Kernels: inference (thread per sample), gradient of the mean squared error
// (blocks of 64 samples staged in LDS write partial gradients, a second kernel
// sums them in block order: deterministic), Adam, and the sample normalization.
#include "internal.h"

namespace esrk {

__global__ void __launch_bounds__(256) mlp_forward_kernel(const float* __restrict__ p,
                                                          const float* __restrict__ X, int B,
                                                          float* __restrict__ Y) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float x[kMlpIn], h1[kMlpH];
#pragma unroll
  for (int i = 0; i < kMlpIn; ++i) x[i] = X[b * kMlpIn + i];
#pragma unroll
  for (int j = 0; j < kMlpH; ++j) {
    float s = p[kOffB1 + j];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) s += p[kOffW1 + j * kMlpIn + i] * x[i];
    h1[j] = tanhf(s);
  }
  float y = p[kOffB3];
  for (int j = 0; j < kMlpH; ++j) {
    float s = p[kOffB2 + j];
#pragma unroll
    for (int i = 0; i < kMlpH; ++i) s += p[kOffW2 + j * kMlpH + i] * h1[i];
    y += p[kOffW3 + j] * tanhf(s);
  }
  Y[b] = y;
}

constexpr int kChunk = 64;    // samples per gradient block
constexpr int kGradThreads = 256;

// Gradient of the mean squared error, stage 1: block c takes samples
// [64 c, 64 c + 64), runs forward and backward with one thread per sample and
// writes its partial gradient (and partial loss) to part[c][0..1282).
__global__ void __launch_bounds__(kGradThreads) mlp_grad_part_kernel(
    const float* __restrict__ p, const float* __restrict__ X, const float* __restrict__ T,
    int B, float* __restrict__ part) {
  __shared__ float sx[kChunk][kMlpIn];
  __shared__ float sh1[kChunk][kMlpH + 1], sh2[kChunk][kMlpH + 1];
  __shared__ float sz1[kChunk][kMlpH + 1], sz2[kChunk][kMlpH + 1];
  __shared__ float sdy[kChunk], sres[kChunk];
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * kChunk;
  const int nb = min(kChunk, B - c0);
  if (tid < nb) {
    const int b = c0 + tid;
    float x[kMlpIn];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) {
      x[i] = X[b * kMlpIn + i];
      sx[tid][i] = x[i];
    }
    float h1[kMlpH], h2[kMlpH];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
      float s = p[kOffB1 + j];
#pragma unroll
      for (int i = 0; i < kMlpIn; ++i) s += p[kOffW1 + j * kMlpIn + i] * x[i];
      h1[j] = tanhf(s);
      sh1[tid][j] = h1[j];
    }
    float y = p[kOffB3];
    for (int j = 0; j < kMlpH; ++j) {
      float s = p[kOffB2 + j];
#pragma unroll
      for (int i = 0; i < kMlpH; ++i) s += p[kOffW2 + j * kMlpH + i] * h1[i];
      h2[j] = tanhf(s);
      sh2[tid][j] = h2[j];
      y += p[kOffW3 + j] * h2[j];
    }
    const float r = y - T[b];
    sres[tid] = r * r;
    const float dy = 2.f * r / float(B);
    sdy[tid] = dy;
    float z2[kMlpH];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
      z2[j] = dy * p[kOffW3 + j] * (1.f - h2[j] * h2[j]);
      sz2[tid][j] = z2[j];
    }
    for (int i = 0; i < kMlpH; ++i) {
      float s = 0.f;
#pragma unroll
      for (int j = 0; j < kMlpH; ++j) s += p[kOffW2 + j * kMlpH + i] * z2[j];
      sz1[tid][i] = s * (1.f - h1[i] * h1[i]);
    }
  }
  __syncthreads();
  float* out = part + (long long)blockIdx.x * (kMlpTrained + 1);
  for (int q = tid; q < kMlpTrained; q += kGradThreads) {
    float acc = 0.f;
    if (q < kOffB1) {
      const int j = q / kMlpIn, i = q - j * kMlpIn;
      for (int b = 0; b < nb; ++b) acc += sz1[b][j] * sx[b][i];
    } else if (q < kOffW2) {
      const int j = q - kOffB1;
      for (int b = 0; b < nb; ++b) acc += sz1[b][j];
    } else if (q < kOffB2) {
      const int j = (q - kOffW2) / kMlpH, i = (q - kOffW2) - j * kMlpH;
      for (int b = 0; b < nb; ++b) acc += sz2[b][j] * sh1[b][i];
    } else if (q < kOffW3) {
      const int j = q - kOffB2;
      for (int b = 0; b < nb; ++b) acc += sz2[b][j];
    } else if (q < kOffB3) {
      const int j = q - kOffW3;
      for (int b = 0; b < nb; ++b) acc += sdy[b] * sh2[b][j];
    } else {
      for (int b = 0; b < nb; ++b) acc += sdy[b];
    }
    out[q] = acc;
  }
  if (tid == 0) {
    float L = 0.f;
    for (int b = 0; b < nb; ++b) L += sres[b];
    out[kMlpTrained] = L;
  }
}

// Stage 2: grad[q] = sum over blocks (in block order) of the partials; the
// last entry of each partial row is the block's squared-residual sum.
__global__ void __launch_bounds__(256) mlp_grad_reduce_kernel(const float* __restrict__ part,
                                                              int nblk, int B,
                                                              float* __restrict__ grad,
                                                              float* __restrict__ loss) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q > kMlpTrained) return;
  float s = 0.f;
  for (int c = 0; c < nblk; ++c) s += part[(long long)c * (kMlpTrained + 1) + q];
  if (q < kMlpTrained) grad[q] = s;
  else if (loss) *loss = s / float(B);
}

__global__ void __launch_bounds__(256) mlp_adam_kernel(float* __restrict__ p,
                                                       const float* __restrict__ g,
                                                       float* __restrict__ m,
                                                       float* __restrict__ v, float lr,
                                                       float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kMlpTrained) return;
  // 1 - beta written out: 1.f - 0.999f would carry the rounding of 0.999f
  const float b1 = 0.9f, ob1 = 0.1f, b2 = 0.999f, ob2 = 0.001f, eps = 1e-8f;
  const float mq = b1 * m[q] + ob1 * g[q];
  const float vq = b2 * v[q] + ob2 * (g[q] * g[q]);
  m[q] = mq;
  v[q] = vq;
  // bias-corrected step; c1 = 1 - b1^t, c2 = 1 - b2^t from the host
  p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// Normalization of logged samples.  raw[B][5] are raw features, gamma[B] the
// solved relaxation parameters (samples are expected to be active elements).
// With fit, the model's normalization entries are first set from the samples:
//   scale_j = mean_b |r_bj| (1 if zero), z_bj = asinh(r_bj / scale_j),
//   mean_j, std_j of z_bj (std 1 if zero); target q_b = (gamma_b - 1) / dt_b^2
//   with dt_b = r_b2, out_mean, out_std of q_b.
// Then x_norm[b][j] = (z_bj - mean_j) / std_j and t_norm[b] = (q_b - out_mean) / out_std.
// One 1024-thread block; sums in FP64 over a fixed thread-strided order.
constexpr int kPrepThreads = 1024;

__device__ double block_sum_1024(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = kPrepThreads / 2; s > 0; s /= 2) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

__global__ void __launch_bounds__(kPrepThreads) mlp_prepare_kernel(
    float* __restrict__ p, const float* __restrict__ raw, const double* __restrict__ gamma,
    int B, int fit, float* __restrict__ xn, float* __restrict__ tn) {
  __shared__ double red[kPrepThreads];
  // normalization entries in the model's order: scale[5], mean[5], std[5], out_mean, out_std
  constexpr int kNrm = kMlpModel - kOffScale;
  __shared__ float nrm[kNrm];
  const int tid = threadIdx.x;
  if (tid < kNrm) nrm[tid] = p[kOffScale + tid];
  __syncthreads();
  if (fit) {
    for (int j = 0; j < kMlpIn; ++j) {
      double s = 0.0;
      for (int b = tid; b < B; b += kPrepThreads) s += fabs((double)raw[b * kMlpIn + j]);
      s = block_sum_1024(s, red) / B;
      const double sc = s > 0.0 ? s : 1.0;
      double z1 = 0.0, z2 = 0.0;
      for (int b = tid; b < B; b += kPrepThreads) {
        const double z = asinh((double)raw[b * kMlpIn + j] / (double)(float)sc);
        z1 += z;
        z2 += z * z;
      }
      z1 = block_sum_1024(z1, red) / B;
      z2 = block_sum_1024(z2, red) / B;
      const double var = z2 - z1 * z1;
      if (tid == 0) {
        nrm[j] = (float)sc;
        nrm[kMlpIn + j] = (float)z1;
        nrm[2 * kMlpIn + j] = var > 0.0 ? (float)sqrt(var) : 1.f;
      }
    }
    if (gamma) {
      double q1 = 0.0, q2 = 0.0;
      for (int b = tid; b < B; b += kPrepThreads) {
        const double dt = raw[b * kMlpIn + 2];
        const double q = (gamma[b] - 1.0) / (dt * dt);
        q1 += q;
        q2 += q * q;
      }
      q1 = block_sum_1024(q1, red) / B;
      q2 = block_sum_1024(q2, red) / B;
      const double var = q2 - q1 * q1;
      if (tid == 0) {
        nrm[3 * kMlpIn] = (float)q1;
        nrm[3 * kMlpIn + 1] = var > 0.0 ? (float)sqrt(var) : 1.f;
      }
    }
    __syncthreads();
    if (tid < kNrm) p[kOffScale + tid] = nrm[tid];
  }
  for (int b = tid; b < B; b += kPrepThreads) {
#pragma unroll
    for (int j = 0; j < kMlpIn; ++j) {
      const float z = asinhf(raw[b * kMlpIn + j] / nrm[j]);
      xn[b * kMlpIn + j] = (z - nrm[kMlpIn + j]) / nrm[2 * kMlpIn + j];
    }
    if (gamma && tn) {
      const double dt = raw[b * kMlpIn + 2];
      const double q = (gamma[b] - 1.0) / (dt * dt);
      tn[b] = (float)((q - (double)nrm[3 * kMlpIn]) / (double)nrm[3 * kMlpIn + 1]);
    }
  }
}

hipError_t launch_mlp_prepare(float* p, const float* raw, const double* gamma, int B, int fit,
                              float* xn, float* tn, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_prepare_kernel, dim3(1), dim3(kPrepThreads), 0, s, p, raw, gamma, B,
                     fit, xn, tn);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* p, const float* X, int B, float* Y, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((B + 255) / 256), dim3(256), 0, s, p, X, B, Y);
  return hipGetLastError();
}

int mlp_grad_blocks(int B) { return (B + kChunk - 1) / kChunk; }

hipError_t launch_mlp_grad(const float* p, const float* X, const float* T, int B, float* grad,
                           float* loss, float* part, hipStream_t s) {
  const int nblk = mlp_grad_blocks(B);
  hipLaunchKernelGGL(mlp_grad_part_kernel, dim3(nblk), dim3(kGradThreads), 0, s, p, X, T, B,
                     part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((kMlpTrained + 1 + 255) / 256), dim3(256), 0,
                     s, part, nblk, B, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* p, const float* g, float* m, float* v, int step, float lr,
                           hipStream_t s) {
  // bias corrections in FP64 (1 - 0.999^t cancels for small t)
  const float c1 = (float)(1.0 - pow(0.9, (double)step));
  const float c2 = (float)(1.0 - pow(0.999, (double)step));
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpTrained + 255) / 256), dim3(256), 0, s, p, g, m,
                     v, lr, c1, c2);
  return hipGetLastError();
}

}  // namespace esrk
