// Device-side building blocks of the entropy-stable flux differencing:
// node primitives, the logarithmic mean and Chandrashekar's entropy-conserving
// two-point flux (Sec. 3.1 names an entropy-conservative volume flux; this one
// satisfies Tadmor's condition for S = -rho s/(gamma-1)).
#pragma once

#include <hip/hip_runtime.h>

namespace esrk {

// Number of terms kept in the series of the logarithmic mean.  The series
// branch is taken for f^2 < 1e-2 with f = (a-b)/(a+b); the first dropped term
// is below 2e-18 (double) or 3e-10 (float) relative.
template <typename T> struct LnSeries;
template <> struct LnSeries<double> {
  static constexpr int terms = 8;
};
template <> struct LnSeries<float> {
  static constexpr int terms = 4;
};

// Short series used when every lane of the wave has f^2 < kLnShortCut (smooth
// flow): 3 terms in double (first dropped term u^3/7 < 1.5e-19), 2 in float
// (u^2/5 < 2e-13).
constexpr double kLnShortCut = 1e-6;
template <typename T> struct LnShort;
template <> struct LnShort<double> {
  static constexpr int terms = 3;
};
template <> struct LnShort<float> {
  static constexpr int terms = 2;
};

// F(u) = atanh(f)/f = sum_k u^k / (2k+1),   u = f^2
template <typename T, int K = LnSeries<T>::terms>
__device__ __forceinline__ T atanh_over(T u) {
  T s = T(1) / T(2 * K - 1);
#pragma unroll
  for (int k = K - 2; k >= 0; --k) s = s * u + T(1) / T(2 * k + 1);
  return s;
}

// G(u) = f/atanh(f) = 1/F(u), series in u with rational coefficients
// g_0 = 1, g_k = -sum_{j<k} g_j / (2(k-j)+1).
template <typename T, int K = LnSeries<T>::terms>
__device__ __forceinline__ T inv_atanh_over(T u) {
  constexpr double g[8] = {1.0,
                           -1.0 / 3.0,
                           -4.0 / 45.0,
                           -44.0 / 945.0,
                           -428.0 / 14175.0,
                           -10196.0 / 467775.0,
                           -10719068.0 / 638512875.0,
                           -25865068.0 / 1915538625.0};
  T s = T(g[K - 1]);
#pragma unroll
  for (int k = K - 2; k >= 0; --k) s = s * u + T(g[k]);
  return s;
}

constexpr double kLnCut = 1e-2;

// Reciprocal: hardware estimate refined by Newton steps (two in double, which
// reach full precision from any estimate better than 2^-14; one in float).
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}
__device__ __forceinline__ float rcp(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(fmaf(-x, r, 1.0f), r, r);
}

// Natural logarithm for x > 0 (finite, normal), double: x = 2^e m with
// m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(t) = 2 t sum_k t^{2k}/(2k+1) with
// t = (m-1)/(m+1), |t| <= 0.1716 (12 terms: first dropped term below 1e-18 of
// the sum), ln x = e ln2_hi + (e ln2_lo + ln m).  About 25 instructions and few
// registers; max error a few ulp (checked on the device against the runtime's
// log over 1e-8..1e8).  The series coefficients live in constant memory so the
// FMAs take them as scalar operands.
__constant__ double kLogAtanh[12] = {1.0,        1.0 / 3.0,  1.0 / 5.0,  1.0 / 7.0,
                                     1.0 / 9.0,  1.0 / 11.0, 1.0 / 13.0, 1.0 / 15.0,
                                     1.0 / 17.0, 1.0 / 19.0, 1.0 / 21.0, 1.0 / 23.0};
__device__ __forceinline__ double log_d(double x) {
  int e;
  double m = frexp(x, &e);  // m in [0.5, 1)
  if (m < 0.70710678118654752440) {
    m += m;
    e -= 1;
  }
  const double t = (m - 1.0) * rcp(m + 1.0);
  const double u = t * t;
  double s = kLogAtanh[11];
#pragma unroll
  for (int k = 10; k >= 0; --k) s = fma(s, u, kLogAtanh[k]);
  const double ed = (double)e;
  // ln 2 = hi + lo with hi = ln 2 truncated to 32 fractional bits (so e * hi
  // is exact for |e| < 2^21) and lo the rounded remainder
  constexpr double kLn2Hi = 0.6931471803691238;
  constexpr double kLn2Lo = 1.9082149292705877e-10;
  return fma(ed, kLn2Hi, fma(ed, kLn2Lo, 2.0 * t * s));
}
__device__ __forceinline__ float log_d(float x) { return logf(x); }

// The three averages of the entropy-conservative flux for one node pair:
// rho^ln, 1/beta^ln and p_hat = {rho}/(2 {beta}).  The logarithmic mean
// (a-b)/(ln a - ln b) = (a+b)/(2 F(f^2)), f = (a-b)/(a+b), is taken from the
// series (no logarithm) unless a jump is large; two reciprocals in the common
// case.
template <typename T>
struct PairMeans {
  T rho_ln, inv_beta_ln, p_hat;
};
// WAVE_UNIFORM: the series length may be chosen per wave (volume pairs, each
// evaluated once).  Interface fluxes are evaluated by both elements of a face
// and must not depend on other lanes: they choose per pair.
template <typename T, bool WAVE_UNIFORM = false>
__device__ __forceinline__ PairMeans<T> pair_means(T ra, T rb, T ba, T bb) {
  const T sr = ra + rb, dr = ra - rb;
  const T sb = ba + bb, db = ba - bb;
  // one reciprocal for both sums
  const T rp = rcp(sr * sb);
  const T rsr = sb * rp, rsb = sr * rp;
  const T fr = dr * rsr, fb = db * rsb;
  const T ur = fr * fr, ub = fb * fb;
  PairMeans<T> m;
  m.p_hat = T(0.5) * sr * rsb;
  // wave-uniform choice of the series length (one ballot, no divergence)
  // short series: wave-uniform choice for volume pairs, per-pair choice (a
  // function of the pair alone, so both elements of a face agree) otherwise
  const bool short_pair = ur < T(kLnShortCut) && ub < T(kLnShortCut);
  if (WAVE_UNIFORM ? __all(short_pair) : short_pair) {
    constexpr int K = LnShort<T>::terms;
    m.rho_ln = T(0.5) * sr * inv_atanh_over<T, K>(ur);
    m.inv_beta_ln = T(2) * rsb * atanh_over<T, K>(ub);
  } else if (ur < T(kLnCut) && ub < T(kLnCut)) {
    m.rho_ln = T(0.5) * sr * inv_atanh_over(ur);
    m.inv_beta_ln = T(2) * rsb * atanh_over(ub);
  } else {
    m.rho_ln = (ur < T(kLnCut)) ? T(0.5) * sr * inv_atanh_over(ur)
                                : dr * rcp(log_d(ra * rcp(rb)));
    m.inv_beta_ln = (ub < T(kLnCut)) ? T(2) * rsb * atanh_over(ub)
                                     : log_d(ba * rcp(bb)) * rcp(db);
  }
  return m;
}

// Primitive set of one node used by the two-point flux.
template <typename T, int DIM>
struct Prim {
  T rho, beta, v[DIM], v2;  // beta = rho / (2 p), v2 = |v|^2
};

template <typename T, int DIM>
__device__ __forceinline__ void prim_from_cons(const T* q, T gg, Prim<T, DIM>& P, T& p) {
  P.rho = q[0];
  const T inv = rcp(q[0]);
  P.v2 = T(0);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    P.v[k] = q[1 + k] * inv;
    P.v2 += P.v[k] * P.v[k];
  }
  p = (gg - T(1)) * (q[DIM + 1] - T(0.5) * P.rho * P.v2);
  P.beta = T(0.5) * P.rho * rcp(p);
}

// Chandrashekar's flux in direction m given the pair averages:
//   f_rho = rho^ln {v_m};  f_mk = f_rho {v_k} + delta_km {rho} / (2 {beta});
//   f_E = f_rho (1/(2 (gamma-1) beta^ln) - {|v|^2}/2) + sum_k {v_k} f_mk.
template <typename T, int DIM>
__device__ __forceinline__ void ec_flux_from_means(int m, const Prim<T, DIM>& A,
                                                   const Prim<T, DIM>& B,
                                                   const PairMeans<T>& mn, T half_inv_gm1,
                                                   T* F) {
  T va[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) va[k] = T(0.5) * (A.v[k] + B.v[k]);
  T vn = va[0];
#pragma unroll
  for (int k = 1; k < DIM; ++k) vn = (m == k) ? va[k] : vn;
  const T frho = mn.rho_ln * vn;
  F[0] = frho;
  T fe = frho * (half_inv_gm1 * mn.inv_beta_ln - T(0.25) * (A.v2 + B.v2));
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const T fm = frho * va[k] + ((m == k) ? mn.p_hat : T(0));
    F[1 + k] = fm;
    fe += va[k] * fm;
  }
  F[DIM + 1] = fe;
}

// ln(1 + x) without cancellation for small |x|: 2 atanh(t), t = x / (2 + x),
// by its series (|x| < 0.1: |t| < 0.048, first dropped term below 1e-21
// relative); log_d(1 + x) beyond, where its absolute error of a few ulp is a
// relative error of at most a few tens of ulp.
// Within a stage the relative changes are small: when every lane of the
// wave has t^2 < 4e-6 three terms suffice (first dropped term below 1e-17).
__device__ __forceinline__ double log1p_d(double x) {
  const double t = x * rcp(2.0 + x);
  const double u = t * t;
  if (__all(u < 4e-6)) return 2.0 * t * atanh_over<double, 3>(u);
  if (fabs(x) < 0.1) return 2.0 * t * atanh_over<double, 8>(u);
  return log_d(1.0 + x);
}

// Change of the entropy variables w = [(g - s)/(g - 1) - K/p, m/p, -rho/p]
// (s = ln p - g ln rho, K = |m|^2/(2 rho)) from state u to state y, written
// in the differences d = y - u so that it keeps its relative accuracy however
// small d is:
//   dK = (rho (2 m.dm + |dm|^2) - drho |m|^2) / (2 rho rho'),
//   dp = (g - 1)(dE - dK),
//   d(-rho/p) = (rho dp - drho p) / (p p'),   d(m/p) = (dm p - m dp) / (p p'),
//   d(K/p) = (dK p - K dp) / (p p'),
//   ds = ln(1 + dp/p) - g ln(1 + drho/rho).
template <int DIM>
__device__ __forceinline__ void entropy_var_change(const double* u, const double* y, double gg,
                                                   double inv_gm1, double* dw) {
  const double rho = u[0], dr = y[0] - u[0];
  const double dE = y[DIM + 1] - u[DIM + 1];
  double m2 = 0.0, mdm = 0.0, dm2 = 0.0, dm[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    dm[d] = y[1 + d] - u[1 + d];
    m2 += u[1 + d] * u[1 + d];
    mdm += u[1 + d] * dm[d];
    dm2 += dm[d] * dm[d];
  }
  const double ir = rcp(rho), ir1 = rcp(y[0]);
  const double K = 0.5 * m2 * ir;
  const double gm1 = gg - 1.0;
  const double p = gm1 * (u[DIM + 1] - K);
  const double dK = 0.5 * (rho * (2.0 * mdm + dm2) - dr * m2) * ir * ir1;
  const double dp = gm1 * (dE - dK);
  const double ip = rcp(p);
  const double ipp = ip * rcp(p + dp);
  dw[DIM + 1] = (rho * dp - dr * p) * ipp;
#pragma unroll
  for (int d = 0; d < DIM; ++d) dw[1 + d] = (dm[d] * p - u[1 + d] * dp) * ipp;
  const double ds = log1p_d(dp * ip) - gg * log1p_d(dr * ir);
  dw[0] = -ds * inv_gm1 - (dK * p - K * dp) * ipp;
}

}  // namespace esrk
