/*
 * Summation-by-parts operators on Legendre-Gauss-Lobatto nodes.
 *
 * The paper's spatial scheme (Sec. 3.1, the element equation and the remark
 * that follows it) is a discontinuous collocated spectral element method
 * built from diagonal-norm SBP operators on LGL nodes.  It does not print the
 * matrices; this file uses the textbook construction:
 *   nodes: -1, +1 and the roots of P_p'(x);
 *   weights: w_i = 2 / (p (p+1) P_p(x_i)^2);
 *   D_ij = l_j'(x_i) (Lagrange basis on the nodes), with the diagonal taken as
 *   minus the off-diagonal row sum so that D applied to a constant is zero.
 * The SBP property Q + Q^T = B with Q = diag(w) D, B = diag(-1,0,..,0,1)
 * follows and is checked by the tests.
 *
 * TEST INFRASTRUCTURE ONLY (see esrk_oracle.h).
 */
#include <math.h>

#include "esrk_oracle.h"

/* Legendre P_p(x) and P_{p-1}(x) by the three-term recurrence. */
static void legendre_pair(int p, double x, double* pp, double* pm1) {
  double a = 1.0, b = x; /* P_0, P_1 */
  if (p == 0) {
    *pp = 1.0;
    *pm1 = 0.0;
    return;
  }
  for (int k = 1; k < p; ++k) {
    double c = ((2.0 * k + 1.0) * x * b - k * a) / (k + 1.0);
    a = b;
    b = c;
  }
  *pp = b;
  *pm1 = a;
}

int orc_lgl(int deg, double* x, double* w) {
  if (deg < 1 || deg > 15) return ORC_EINVAL;
  const int p = deg, n = deg + 1;
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    /* Chebyshev-Gauss-Lobatto start, refined by Newton on P_p'. */
    double xi = -cos(pi * i / p);
    if (i > 0 && i < p) {
      for (int it = 0; it < 100; ++it) {
        double P, Pm1;
        legendre_pair(p, xi, &P, &Pm1);
        /* P_p' from (x^2-1) P_p' = p (x P_p - P_{p-1}); P_p'' from Legendre's ODE. */
        double d1 = p * (xi * P - Pm1) / (xi * xi - 1.0);
        double d2 = (2.0 * xi * d1 - p * (p + 1.0) * P) / (1.0 - xi * xi);
        double step = d1 / d2;
        xi -= step;
        if (fabs(step) < 1e-17) break;
      }
    }
    x[i] = xi;
  }
  /* symmetrize: the node set is symmetric about 0 */
  for (int i = 0; i < n / 2; ++i) {
    double s = 0.5 * (x[n - 1 - i] - x[i]);
    x[i] = -s;
    x[n - 1 - i] = s;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
  for (int i = 0; i < n; ++i) {
    double P, Pm1;
    legendre_pair(p, x[i], &P, &Pm1);
    w[i] = 2.0 / (p * (p + 1.0) * P * P);
  }
  return ORC_OK;
}

int orc_dmat(int deg, double* D) {
  if (deg < 1 || deg > 15) return ORC_EINVAL;
  const int n = deg + 1;
  double x[16], w[16], lam[16];
  orc_lgl(deg, x, w);
  /* barycentric weights lam_j = 1 / prod_{k != j} (x_j - x_k) */
  for (int j = 0; j < n; ++j) {
    double prod = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != j) prod *= (x[j] - x[k]);
    lam[j] = 1.0 / prod;
  }
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double dij = (lam[j] / lam[i]) / (x[i] - x[j]);
      D[i * n + j] = dij;
      diag -= dij;
    }
    D[i * n + i] = diag;
  }
  return ORC_OK;
}
