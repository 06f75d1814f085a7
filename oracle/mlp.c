/*
 * FP64 reference of the small network that proposes initial relaxation
 * parameters (the learned extension of the relaxation solve; the paper
 * itself only prescribes solving the scalar equation of Sec. 2 per element).
 *
 * Network: 5 -> 32 -> 32 -> 1, tanh hidden layers, linear output:
 *   h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = w3 . h2 + b3.
 * Loss over a batch of B samples: L = (1/B) sum_b (y_b - t_b)^2.
 * Parameter vector (the interface shared with the GPU path), offsets:
 *   W1[32][5] at 0, b1[32] at 160, W2[32][32] at 192, b2[32] at 1216,
 *   w3[32] at 1248, b3 at 1280; 1281 trained parameters in total.
 * Plain loops, no blocking.
 *
 * TEST INFRASTRUCTURE ONLY (see esrk_oracle.h).
 */
#include <math.h>

#include "esrk_oracle.h"

#define H 32
#define NI 5
#define OW1 0
#define OB1 160
#define OW2 192
#define OB2 1216
#define OW3 1248
#define OB3 1280

static void forward_one(const double* p, const double* x, double* h1, double* h2, double* y) {
  for (int j = 0; j < H; ++j) {
    double s = p[OB1 + j];
    for (int i = 0; i < NI; ++i) s += p[OW1 + j * NI + i] * x[i];
    h1[j] = tanh(s);
  }
  for (int j = 0; j < H; ++j) {
    double s = p[OB2 + j];
    for (int i = 0; i < H; ++i) s += p[OW2 + j * H + i] * h1[i];
    h2[j] = tanh(s);
  }
  double s = p[OB3];
  for (int j = 0; j < H; ++j) s += p[OW3 + j] * h2[j];
  *y = s;
}

int orc_mlp_forward(const double* params, const double* X, int B, double* Y) {
  double h1[H], h2[H];
  for (int b = 0; b < B; ++b) forward_one(params, X + b * NI, h1, h2, Y + b);
  return ORC_OK;
}

int orc_mlp_grad(const double* params, const double* X, const double* T, int B, double* grad,
                 double* loss) {
  if (B < 1) return ORC_EINVAL;
  for (int q = 0; q < ORC_MLP_PARAMS; ++q) grad[q] = 0.0;
  double L = 0.0;
  for (int b = 0; b < B; ++b) {
    const double* x = X + b * NI;
    double h1[H], h2[H], y;
    forward_one(params, x, h1, h2, &y);
    const double r = y - T[b];
    L += r * r;
    /* dL/dy for the mean of squares */
    const double dy = 2.0 * r / B;
    double dz2[H], dz1[H];
    grad[OB3] += dy;
    for (int j = 0; j < H; ++j) {
      grad[OW3 + j] += dy * h2[j];
      dz2[j] = dy * params[OW3 + j] * (1.0 - h2[j] * h2[j]);
    }
    for (int j = 0; j < H; ++j) {
      grad[OB2 + j] += dz2[j];
      for (int i = 0; i < H; ++i) grad[OW2 + j * H + i] += dz2[j] * h1[i];
    }
    for (int i = 0; i < H; ++i) {
      double s = 0.0;
      for (int j = 0; j < H; ++j) s += params[OW2 + j * H + i] * dz2[j];
      dz1[i] = s * (1.0 - h1[i] * h1[i]);
    }
    for (int j = 0; j < H; ++j) {
      grad[OB1 + j] += dz1[j];
      for (int i = 0; i < NI; ++i) grad[OW1 + j * NI + i] += dz1[j] * x[i];
    }
  }
  if (loss) *loss = L / B;
  return ORC_OK;
}

/* Adam (Kingma and Ba, 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 on the
 * trained parameters; step t >= 1 counts updates, m and v start at zero. */
int orc_mlp_adam(double* params, const double* grad, double* m, double* v, int step, double lr) {
  if (step < 1) return ORC_EINVAL;
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (int q = 0; q < ORC_MLP_PARAMS; ++q) {
    m[q] = b1 * m[q] + (1.0 - b1) * grad[q];
    v[q] = b2 * v[q] + (1.0 - b2) * grad[q] * grad[q];
    params[q] -= lr * (m[q] / c1) / (sqrt(v[q] / c2) + eps);
  }
  return ORC_OK;
}

/* Normalization of logged samples (model entries after the trained ones:
 * scale[5] at 1281, mean[5] at 1286, std[5] at 1291, out_mean at 1296,
 * out_std at 1297).  With fit: scale_j = mean |r_j| (1 if 0), z = asinh(r/scale),
 * mean_j and (population) std_j of z (std 1 if 0); q = (gamma - 1)/dt^2 with
 * dt = r_2, out_mean and out_std of q.  Then x = (z - mean)/std and
 * t = (q - out_mean)/out_std (t only if gamma is given). */
int orc_mlp_prepare(double* model, const double* raw, const double* gamma, int B, int fit,
                    double* xn, double* tn) {
  if (B < 1) return ORC_EINVAL;
  double* scale = model + 1281;
  double* mean = model + 1286;
  double* sd = model + 1291;
  if (fit) {
    for (int j = 0; j < NI; ++j) {
      double s = 0.0;
      for (int b = 0; b < B; ++b) s += fabs(raw[b * NI + j]);
      s /= B;
      scale[j] = s > 0.0 ? s : 1.0;
      double z1 = 0.0;
      for (int b = 0; b < B; ++b) z1 += asinh(raw[b * NI + j] / scale[j]);
      z1 /= B;
      double z2 = 0.0;
      for (int b = 0; b < B; ++b) {
        const double d = asinh(raw[b * NI + j] / scale[j]) - z1;
        z2 += d * d;
      }
      z2 /= B;
      mean[j] = z1;
      sd[j] = z2 > 0.0 ? sqrt(z2) : 1.0;
    }
    if (gamma) {
      double q1 = 0.0, q2 = 0.0;
      for (int b = 0; b < B; ++b) {
        const double dt = raw[b * NI + 2];
        q1 += (gamma[b] - 1.0) / (dt * dt);
      }
      q1 /= B;
      for (int b = 0; b < B; ++b) {
        const double dt = raw[b * NI + 2];
        const double d = (gamma[b] - 1.0) / (dt * dt) - q1;
        q2 += d * d;
      }
      q2 /= B;
      model[1296] = q1;
      model[1297] = q2 > 0.0 ? sqrt(q2) : 1.0;
    }
  }
  for (int b = 0; b < B; ++b) {
    for (int j = 0; j < NI; ++j)
      xn[b * NI + j] = (asinh(raw[b * NI + j] / scale[j]) - mean[j]) / sd[j];
    if (gamma && tn) {
      const double dt = raw[b * NI + 2];
      tn[b] = ((gamma[b] - 1.0) / (dt * dt) - model[1296]) / model[1297];
    }
  }
  return ORC_OK;
}
