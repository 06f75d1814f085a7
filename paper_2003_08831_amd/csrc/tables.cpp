// Lobatto nodes, weights and the differentiation matrix for the device tables
// (Sec. 3.1: diagonal-norm SBP operators on Legendre-Gauss-Lobatto nodes).
//
// Built on the host in extended precision from closed forms:
//  - nodes are the roots of q(x) = P_{p+1}(x) - P_{p-1}(x) = c (1 - x^2) P_p'(x),
//    found by Newton with q'(x) = (2p+1) P_p(x);
//  - weights w_i = 2 / (p (p+1) P_p(x_i)^2);
//  - D_ij = P_p(x_i) / (P_p(x_j) (x_i - x_j)) for i != j, D_00 = -p(p+1)/4,
//    D_pp = p(p+1)/4 and D_ii = 0 for the inner nodes.
#include <cmath>

#include "internal.h"

namespace esrk {

static void legendre3(int p, long double x, long double* pm1, long double* pp,
                      long double* pp1) {
  long double a = 1.0L, b = x;  // P_0, P_1
  if (p == 0) {
    *pm1 = 0.0L;
    *pp = 1.0L;
    *pp1 = x;
    return;
  }
  for (int k = 1; k <= p; ++k) {
    long double c = ((2.0L * k + 1.0L) * x * b - k * a) / (k + 1.0L);
    a = b;
    b = c;
  }
  // now a = P_p, b = P_{p+1}; recover P_{p-1} from the recurrence
  *pp = a;
  *pp1 = b;
  *pm1 = ((2.0L * p + 1.0L) * x * a - (p + 1.0L) * b) / p;
}

void lobatto_tables(int deg, double* xout, double* wout, double* D) {
  const int p = deg, n = deg + 1;
  long double x[kMaxN], Pp[kMaxN];
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double xi = -cosl(pi * i / p);
    if (i > 0 && i < p) {
      for (int it = 0; it < 60; ++it) {
        long double pm1, pp, pp1;
        legendre3(p, xi, &pm1, &pp, &pp1);
        const long double q = pp1 - pm1;
        const long double dq = (2.0L * p + 1.0L) * pp;
        const long double step = q / dq;
        xi -= step;
        if (fabsl(step) < 1e-21L) break;
      }
    }
    x[i] = xi;
  }
  for (int i = 0; i < n / 2; ++i) {  // exact symmetry
    const long double s = 0.5L * (x[n - 1 - i] - x[i]);
    x[i] = -s;
    x[n - 1 - i] = s;
  }
  if (n % 2) x[n / 2] = 0.0L;
  for (int i = 0; i < n; ++i) {
    long double pm1, pp, pp1;
    legendre3(p, x[i], &pm1, &pp, &pp1);
    Pp[i] = pp;
    xout[i] = (double)x[i];
    wout[i] = (double)(2.0L / (p * (p + 1.0L) * pp * pp));
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      long double d;
      if (i != j)
        d = Pp[i] / (Pp[j] * (x[i] - x[j]));
      else if (i == 0)
        d = -p * (p + 1.0L) / 4.0L;
      else if (i == p)
        d = p * (p + 1.0L) / 4.0L;
      else
        d = 0.0L;
      D[i * n + j] = (double)d;
    }
}

}  // namespace esrk
