// Local relaxation kernels (Sec. 2: local relaxation equation; the theorem
// that gamma = min_k gamma_k keeps every element's entropy inequality) and
// the step bookkeeping kernels (CFL step size, global minimum, relaxed update).
//
// Per element k, with du = u_new - u_old and deta_k = eta_k^new - eta_k^old,
//   r_k(g) = eta_k(u_old + g du) - eta_k(u_old) - g deta_k = g a_k + B_k(g),
//   a_k    = sum_i M_i w(u_old,i).du_i - deta_k          (= phi_k(0)),
//   B_k(g) = sum_i M_i [S(u_i + g du_i) - S(u_i) - g w(u_i).du_i]   (>= 0),
// and phi_k(g) = r_k(g)/g = a_k + B_k(g)/g.  B_k is the relative entropy of the
// relaxed state with respect to u_old; per node it is evaluated without
// cancellation from the ratios y = rho'/rho and x = p'/p:
//   S(u') - S(u) - w(u).(u'-u) = rho'/(g-1) h(x/y) + rho k(y) + rho rho'/(2p) |v'-v|^2,
//   h(z) = z - 1 - ln z,   k(y) = y ln y - y + 1,
// both taken from their Taylor series near 1.  So phi_k is accurate to round-off
// in a_k even when the entropy change of an element is tiny.
//
// Mapping: one segment of G lanes (G = next power of two >= nodes per element,
// at most 64) per element; each lane keeps its nodes' u_old and du in registers
// for the whole solve, the element sums are segment shuffles.  The root is
// bracketed from [0, 1] and refined by Illinois-modified regula falsi, each new
// point kept at least tol/4 inside the bracket, until the bracket is narrower
// than tol * max(1, gamma); the lower end (phi <= 0) is returned.
#include <cfloat>

#include "device_math.h"
#include "internal.h"

namespace esrk {

__device__ __forceinline__ void latch_r(DevScalars* s, int code, long long elem) {
  atomicCAS(&s->status, 0, code);
  atomicMin((unsigned long long*)&s->bad_elem, (unsigned long long)elem);
}

__device__ __forceinline__ double dbits(unsigned long long b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ unsigned long long bitsd(double d) {
  return (unsigned long long)__double_as_longlong(d);
}

// h(1+t) = t - log1p(t) = sum_{n>=2} (-1)^n t^n / n and
// k(1+t) = (1+t) log1p(t) - t = sum_{n>=2} (-1)^n t^n / (n (n-1)), from their
// series for |t| < 0.1 (16 terms: first dropped term below 1.2e-17 of the
// leading one; 8 terms when every lane of the wave has |t| < 1e-2) and from
// log1p beyond.  The coefficients sit in constant memory, so the kernels take
// them as scalar-register FMA operands (as literals they were rematerialized
// into vector registers with two moves per use).
constexpr int kRelTerms = 16;
__constant__ double kHRel[kRelTerms] = {
    1.0 / 2, -1.0 / 3, 1.0 / 4, -1.0 / 5, 1.0 / 6, -1.0 / 7, 1.0 / 8, -1.0 / 9,
    1.0 / 10, -1.0 / 11, 1.0 / 12, -1.0 / 13, 1.0 / 14, -1.0 / 15, 1.0 / 16, -1.0 / 17};
__constant__ double kKRel[kRelTerms] = {
    1.0 / 2, -1.0 / 6, 1.0 / 12, -1.0 / 20, 1.0 / 30, -1.0 / 42, 1.0 / 56, -1.0 / 72,
    1.0 / 90, -1.0 / 110, 1.0 / 132, -1.0 / 156, 1.0 / 182, -1.0 / 210, 1.0 / 240,
    -1.0 / 272};

template <int K>
__device__ __forceinline__ double rel_series(const double* c, double t) {
  double s = c[K - 1];
#pragma unroll
  for (int n = K - 2; n >= 0; --n) s = s * t + c[n];
  return s * t * t;
}

// h(1 + tz) and k(1 + tr) of one node; `short_ok` is wave-uniform
__device__ __forceinline__ void rel_terms(double tz, double tr, bool short_ok, double& h,
                                          double& k) {
  if (short_ok) {
    h = rel_series<8>(kHRel, tz);
    k = rel_series<8>(kKRel, tr);
    return;
  }
  h = fabs(tz) < 0.1 ? rel_series<kRelTerms>(kHRel, tz) : tz - log1p(tz);
  k = fabs(tr) < 0.1 ? rel_series<kRelTerms>(kKRel, tr) : (1.0 + tr) * log1p(tr) - tr;
}

// reciprocal: hardware estimate + two Newton steps (full double precision)
__device__ __forceinline__ double rcp_d(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

template <int G>
__device__ __forceinline__ double seg_sum(double x) {
#pragma unroll
  for (int off = G / 2; off >= 1; off /= 2) x += __shfl_xor(x, off, 64);
  return x;
}

template <int G>
__device__ __forceinline__ double seg_max(double x) {
#pragma unroll
  for (int off = G / 2; off >= 1; off /= 2) x = fmax(x, __shfl_xor(x, off, 64));
  return x;
}
template <int G>
__device__ __forceinline__ float seg_sum_f(float x) {
#pragma unroll
  for (int off = G / 2; off >= 1; off /= 2) x += __shfl_xor(x, off, 64);
  return x;
}

// Network output for the element of this segment (all G lanes take part; the
// raw features r are the same on every lane of the segment).  Hidden unit j
// is held by lane j mod G; layer 2 gathers layer-1 values by shuffles.
template <int G>
__device__ __forceinline__ float mlp_segment(const float* __restrict__ p, const double* r,
                                             int seg_base, int sl) {
  constexpr int U = (kMlpH + G - 1) / G;
  float x[kMlpIn];
#pragma unroll
  for (int i = 0; i < kMlpIn; ++i)
    x[i] = (asinhf(float(r[i]) / p[kOffScale + i]) - p[kOffMean + i]) / p[kOffStd + i];
  float h1[U], s2[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = sl + u * G;
    float s = 0.f;
    if (j < kMlpH) {
      s = p[kOffB1 + j];
#pragma unroll
      for (int i = 0; i < kMlpIn; ++i) s += p[kOffW1 + j * kMlpIn + i] * x[i];
    }
    h1[u] = j < kMlpH ? tanhf(s) : 0.f;
    s2[u] = j < kMlpH ? p[kOffB2 + j] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < kMlpH; ++i) {
    const float hi = __shfl(h1[i / G], seg_base + (i % G), 64);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = sl + u * G;
      if (j < kMlpH) s2[u] += p[kOffW2 + j * kMlpH + i] * hi;
    }
  }
  float y = 0.f;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = sl + u * G;
    if (j < kMlpH) y += p[kOffW3 + j] * tanhf(s2[u]);
  }
  return seg_sum_f<G>(y) + p[kOffB3];
}

template <int DIM, int N>
struct RelaxCfg {
  static constexpr int ND = (DIM == 1) ? N : (DIM == 2) ? N * N : N * N * N;
  static constexpr int NV = DIM + 2;
  static constexpr int G = ND <= 2 ? 2 : ND <= 4 ? 4 : ND <= 8 ? 8 : ND <= 16 ? 16
                           : ND <= 32 ? 32 : 64;
  static constexpr int NPL = (ND + G - 1) / G;
  static constexpr int SEGS = 64 / G;
  static constexpr int THREADS = 256;
  static constexpr int EPB = (THREADS / 64) * SEGS;  // elements per block
};

// One block's work: EPB elements starting at element kb of the mesh md; the
// block partial goes to a.parts[part].
// Trial-point rules compiled into their own kernels (their per-element state
// costs registers); kRuleRuntime reads a.method (Illinois or bisection).
enum { kRuleRuntime = 0, kRuleBrent = 1, kRuleAlefeld = 2 };

template <int DIM, int N, bool NET, int RULE = kRuleRuntime>
__device__ __forceinline__ void relax_block(const MeshParams& mp, const MeshDims& md,
                                            const RelaxArgs& a, const int kb, const int part,
                                            const long long elem_base) {
  using C = RelaxCfg<DIM, N>;
  constexpr int NV = C::NV, G = C::G, NPL = C::NPL, ND = C::ND;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int seg = lane / G;
  const int sl = lane - seg * G;
  const int k = kb + wave * C::SEGS + seg;
  const bool valid = k < md.ne;
  const long long Ntot = (long long)md.ne * ND;
  const double gg = mp.gg, gm1 = gg - 1.0, inv_gm1 = 1.0 / gm1;
  if (a.check_reject && a.scal->rejected) {
    // a rejected error-controlled attempt: nothing to relax
    if (valid && sl == 0) {
      a.gamma_k[k] = INFINITY;
      if (a.iters) a.iters[k] = 0;
    }
    if (threadIdx.x == 0) a.parts[part] = RelaxPart{INFINITY, 0, 0, 0};
    return;
  }

  // per-node constants along the relaxation line
  double rho[NPL], mom[NPL][DIM], ene[NPL], dr[NPL], dm[NPL][DIM], dE[NPL];
  double invrho[NPL], invp[NPL], m2[NPL], beta[NPL], Mi[NPL];
  bool has[NPL];
  double A = 0.0, scale = 0.0, smax = 0.0;
  const bool want_feats = NET && (a.feats != nullptr || a.model != nullptr);
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int i = sl + j * G;
    has[j] = valid && i < ND;
    const long long gi = (long long)k * ND + i;
    if (has[j]) {
      rho[j] = a.u_old[gi];
      dr[j] = a.du[gi];
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        mom[j][d] = a.u_old[(1 + d) * Ntot + gi];
        dm[j][d] = a.du[(1 + d) * Ntot + gi];
      }
      ene[j] = a.u_old[(NV - 1) * Ntot + gi];
      dE[j] = a.du[(NV - 1) * Ntot + gi];
    } else {
      rho[j] = 1.0;
      dr[j] = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) mom[j][d] = dm[j][d] = 0.0;
      ene[j] = 1.0;
      dE[j] = 0.0;
    }
    invrho[j] = rcp_d(rho[j]);
    double mm = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) mm += mom[j][d] * mom[j][d];
    m2[j] = mm;
    const double p = gm1 * (ene[j] - 0.5 * mm * invrho[j]);
    invp[j] = rcp_d(p);
    beta[j] = 0.5 * rho[j] * invp[j];
    double M = 1.0;
    {
      int ii = i;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int im = ii % N;
        ii /= N;
        M *= md.half_h[d] * mp.w[im];
      }
    }
    Mi[j] = has[j] ? M : 0.0;
    // w(u_old).du and its round-off scale
    const double s_phys = log_d(p) - gg * log_d(rho[j]);
    const double v2 = mm * invrho[j] * invrho[j];
    double t = ((gg - s_phys) * inv_gm1 - beta[j] * v2) * dr[j];
    double sc = fabs(t);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double td = 2.0 * beta[j] * mom[j][d] * invrho[j] * dm[j][d];
      t += td;
      sc += fabs(td);
    }
    const double te = -2.0 * beta[j] * dE[j];
    t += te;
    sc += fabs(te);
    A += Mi[j] * t;
    scale += Mi[j] * sc;
    if (want_feats && has[j]) {
      double sp = 0.0;
      const double c = sqrt(gg * p * invrho[j]);
#pragma unroll
      for (int d = 0; d < DIM; ++d) sp += fabs(mom[j][d] * invrho[j]) + c;
      smax = fmax(smax, sp);
    }
  }
  A = seg_sum<G>(A);
  scale = seg_sum<G>(scale);
  if (want_feats) smax = seg_max<G>(smax);
  // phi_k(0) from the stages when given; the estimate's increment is then
  // Delta eta_k = A_k - phi_k(0) if the caller did not pass it
  const double phi0 = a.phi0_in ? (valid ? a.phi0_in[k] : 0.0) : A - (valid ? a.deta[k] : 0.0);
  const double deta = (valid && a.deta) ? a.deta[k] : A - phi0;
  // round-off level of the element's entropy increments: FP64 increments, or
  // increments built from FP32 flux differences (then the estimate and the
  // update of an element that barely changes are FP32 noise and its root is
  // not determined)
  const double noise_eps = a.fp32_increments ? (double)FLT_EPSILON : DBL_EPSILON;
  const double noise = 64.0 * noise_eps * (scale + fabs(deta));

  // relative entropy sum B(g) and admissibility along the line
  // (an inadmissible node makes the element sum +INF)
  auto Bsum = [&](double g, bool& ok) -> double {
    double part = 0.0;
    bool bad = false;
    double tzs[NPL], trs[NPL], dv2s[NPL];
    bool oks[NPL];
    bool small = true;
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
      const double r0 = rho[j];
      const double drg = g * dr[j];
      const double r1 = r0 + drg;
      double mdm = 0.0, dm2 = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double dmg = g * dm[j][d];
        mdm += mom[j][d] * dmg;
        dm2 += dmg * dmg;
      }
      const double q = rcp_d(r0 * r1);
      const double dke = (r0 * (2.0 * mdm + dm2) - drg * m2[j]) * q;
      const double dp = gm1 * (g * dE[j] - 0.5 * dke);
      const double tr = drg * invrho[j];
      const double tp = dp * invp[j];
      const bool okn = (r1 > 0.0) && (1.0 + tp > 0.0);
      if (!okn && has[j]) bad = true;
      const double tz = okn ? (tp - tr) * r0 * r0 * q : 0.0;
      double dv2 = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double dv = (g * dm[j][d] - drg * mom[j][d] * invrho[j]) * r0 * q;
        dv2 += dv * dv;
      }
      tzs[j] = tz;
      trs[j] = okn ? tr : 0.0;
      dv2s[j] = dv2;
      oks[j] = okn;
      small = small && fabs(tzs[j]) < 1e-2 && fabs(trs[j]) < 1e-2;
    }
    const bool short_ok = __all(small);
#pragma unroll
    for (int j = 0; j < NPL; ++j) {
      double h, kk;
      rel_terms(tzs[j], trs[j], short_ok, h, kk);
      const double r0 = rho[j];
      const double r1 = r0 + g * dr[j];
      const double Dn = oks[j] ? r1 * h * inv_gm1 + r0 * kk + beta[j] * r1 * dv2s[j] : 0.0;
      part += Mi[j] * Dn;
    }
    part = seg_sum<G>(bad ? INFINITY : part);
    ok = !isinf(part);
    return part;
  };

  // root solve: all lanes iterate together; a segment stops updating once done
  const double tol = a.tol, gmax = a.gamma_max;
  double lo = 0.0, flo = phi0, hi = 1.0, fhi = 0.0, gk = 1.0, g_trial = 1.0;
  bool hi_known = false, done = !valid;
  int side = 0, its = 0;
  // Brent's method (own instantiation: its state costs registers): previous
  // iterate (ba, fba), last and second-to-last steps
  double ba = NAN, fba = NAN, bd = 0.0, be = 0.0;
  // Alefeld-Potra-Shi (first method): phase of the next trial point (0 the
  // opening secant, 1 inverse cubic / Newton-quadratic, 2 double-length
  // secant, 3 bisection), the points d and e beside the bracket (e = NaN
  // until known), d-bar of the current iteration and its opening width
  int aph = 0;
  double ad = NAN, fad = NAN, ae = NAN, fae = NAN, adb = NAN, fadb = NAN, aw0 = 0.0;
  constexpr bool BRENT = RULE == kRuleBrent, ALEFELD = RULE == kRuleAlefeld;
  const int method = BRENT     ? ESRK_ROOT_BRENT
                     : ALEFELD ? ESRK_ROOT_ALEFELD
                               : (a.method == ESRK_ROOT_BISECTION ? ESRK_ROOT_BISECTION
                                                                  : ESRK_ROOT_ILLINOIS);
  const bool have_guess = a.guess != nullptr;
  double dtf = 0.0;
  if (want_feats) dtf = a.dt_dev ? *a.dt_dev : a.dt_host;
  float net_guess = 1.f;
  bool first_pass = true;
  while (__any(!done)) {
    bool ok = true;
    const double B = Bsum(done ? 1.0 : g_trial, ok);
    if (first_pass && want_feats) {
      // features of the element at gamma = 1 (every lane of the segment holds them)
      double rf[kMlpIn];
      rf[0] = deta;
      rf[1] = A + B;  // eta(u_new) - eta(u_old)
      rf[2] = dtf;
      rf[3] = smax;
      rf[4] = (valid && a.vfeat) ? dtf * a.vfeat[k] : 0.0;
      if (a.feats && valid && sl == 0) {
#pragma unroll
        for (int q = 0; q < kMlpIn; ++q) a.feats[(long long)k * kMlpIn + q] = float(rf[q]);
      }
      if (NET && a.model) {
        const float y = mlp_segment<G>(a.model, rf, seg * G, sl);
        net_guess = float(1.0 + dtf * dtf * (double(a.model[kOffOutMean]) +
                                             double(a.model[kOffOutStd]) * double(y)));
      }
    }
    first_pass = false;
    if (done) continue;
    ++its;
    const double f = ok ? phi0 + B / g_trial : INFINITY;
    if (its == 1) {
      const double q = ok ? B : INFINITY;  // r(1) - phi(0)
      if (q <= noise) {
        gk = INFINITY;
        done = true;
        continue;
      }
      if (!(phi0 <= -0.5 * q)) {
        // phi(0) ~ 0 against the relative entropy (root below about 1/2:
        // an element reached by a wave only in the last stages of the step
        // has no slope of its own at u_old) or, with FP32-flux increments,
        // an entropy change r(1) within the FP32 rounding level: no
        // determinable root, inactive.  phi(0) above its round-off level:
        // no positive root, an error.
        if (phi0 <= noise || (a.fp32_increments && ok && phi0 + q <= noise)) {
          gk = INFINITY;
          done = true;
          continue;
        }
        gk = 0.0;
        done = true;
        if (sl == 0) latch_r(a.scal, ESRK_ENOROOT, elem_base + k);
        continue;
      }
    }
    if (ALEFELD && f == 0.0) {
      // an exact root ends the enclosure
      gk = g_trial;
      done = true;
      continue;
    }
    // the bracket end the new point replaces (d of the enclosure step)
    const double rep_x = (f <= 0.0) ? lo : hi, rep_f = (f <= 0.0) ? flo : fhi;
    // Illinois: a bracket end kept twice in a row has its value halved
    const bool illinois = method == ESRK_ROOT_ILLINOIS;
    if (f <= 0.0) {
      if (illinois && hi_known && side == -1) fhi *= 0.5;
      lo = g_trial;
      flo = f;
      side = -1;
    } else {
      if (illinois && hi_known && side == +1) flo *= 0.5;
      hi = g_trial;
      fhi = f;
      hi_known = true;
      side = +1;
    }
    // first trial point after gamma = 1: the network's or the caller's guess
    // (used on either side of 1), else the regula falsi / doubling step
    double g0 = -1.0;
    if (its == 1) {
      if (NET && a.model) g0 = (double)net_guess;
      else if (have_guess) g0 = a.guess[k];
      if (!(g0 > 0.0 && g0 <= gmax)) g0 = -1.0;  // also drops +inf (inactive) and NaN
    }
    if (!hi_known) {
      if (lo >= gmax) {
        gk = gmax;
        done = true;
      } else {
        g_trial = (g0 > lo) ? fmin(g0, gmax) : fmin(2.0 * lo, gmax);
      }
      continue;
    }
    const double tw = tol * fmax(1.0, hi);
    if (hi - lo <= tw || its >= a.maxit) {
      gk = lo;
      done = true;
      continue;
    }
    // Alefeld-Potra-Shi bookkeeping for the point just evaluated (a bracketed
    // point only: the doubling search before the bracket is phase 0)
    // (phase 0: the point was gamma = 1, a guess or a doubling step, and the
    // opening secant comes next; phase 4: the opening secant was evaluated)
    int anext = aph;
    if (ALEFELD) {
      if (aph == 4) {
        // d = the replaced end; the first iteration has no e
        ad = rep_x;
        fad = rep_f;
        anext = 1;
      } else if (aph == 1) {
        adb = rep_x;
        fadb = rep_f;
        anext = 2;
      } else if (aph == 2) {
        if (hi - lo < 0.5 * aw0) {
          ae = adb;
          fae = fadb;
          ad = rep_x;
          fad = rep_f;
          anext = 1;
        } else {
          ae = rep_x;
          fae = rep_f;
          anext = 3;
        }
      } else if (aph == 3) {
        ad = rep_x;
        fad = rep_f;
        anext = 1;
      }
    }
    double g;
    if (g0 > 0.0) {
      g = g0;
    } else if (method == ESRK_ROOT_BISECTION || isinf(fhi)) {
      g = 0.5 * (lo + hi);
      if (ALEFELD) {
        // the midpoint stands in for the phase's own trial point
        aph = anext == 0 ? 4 : anext;
        if (aph == 1) aw0 = hi - lo;
      }
    } else if (ALEFELD) {
      aph = anext;
      const double mid = 0.5 * (lo + hi);
      if (aph == 0) {
        g = lo - flo * (hi - lo) / (fhi - flo);
        aph = 4;
      } else if (aph == 1) {
        aw0 = hi - lo;
        g = NAN;
        // inverse cubic interpolation through (lo, hi, d, e) at zero when the
        // four values are finite and pairwise distinct, else the
        // Newton-quadratic step (two Newton steps on the quadratic through
        // lo, hi, d)
        const double xs[4] = {lo, hi, ad, ae}, fs[4] = {flo, fhi, fad, fae};
        bool distinct = isfinite(fad) && isfinite(fae) && ad == ad && ae == ae;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = i + 1; j < 4; ++j) distinct = distinct && fs[i] != fs[j];
        if (distinct) {
          double x = 0.0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            double l = xs[i];
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (j != i) l *= fs[j] / (fs[j] - fs[i]);
            x += l;
          }
          if (x > lo && x < hi) g = x;
        }
        if (!(g == g) && isfinite(fad) && ad == ad && ad != lo && ad != hi) {
          const double fab = (fhi - flo) / (hi - lo);
          const double fbd = (fad - fhi) / (ad - hi);
          const double qa = (fbd - fab) / (ad - lo);
          double x = (qa * flo > 0.0) ? lo : hi;
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const double P = flo + (fab + qa * (x - hi)) * (x - lo);
            const double dP = fab + qa * (2.0 * x - lo - hi);
            x -= P / dP;
          }
          if (x > lo && x < hi) g = x;
        }
        if (!(g == g)) g = lo - flo * (hi - lo) / (fhi - flo);
      } else if (aph == 2) {
        // double-length secant from the end with the smaller |phi|, bisection
        // when it would leave the middle half of the bracket
        const bool lo_best = fabs(flo) < fabs(fhi);
        const double uu = lo_best ? lo : hi, fu = lo_best ? flo : fhi;
        g = uu - 2.0 * fu * (hi - lo) / (fhi - flo);
        if (fabs(g - uu) > 0.5 * (hi - lo)) g = mid;
      } else {
        g = mid;
      }
    } else if (BRENT) {
      // Brent's step from the better bracket end b towards the other end c:
      // inverse quadratic interpolation through (a, b, c), a the previous b,
      // when the three values differ, else the secant through (a, b); taken
      // only while the steps shrink faster than bisection's, else bisection
      const bool lo_best = fabs(flo) <= fabs(fhi);
      const double b = lo_best ? lo : hi, fb = lo_best ? flo : fhi;
      const double c = lo_best ? hi : lo, fc = lo_best ? fhi : flo;
      // a: the previous b if the newest point became b, else the newest point
      double pa = (g_trial == b) ? ba : g_trial, fpa = (g_trial == b) ? fba : f;
      if (!(pa == pa)) {
        // first Brent step: a = c and the last steps as wide as the bracket
        pa = c;
        fpa = fc;
        bd = be = c - b;
      }
      const double m = 0.5 * (c - b);
      const double tolb = 0.25 * tw;
      double step = m;
      if (fabs(be) >= tolb && fabs(fpa) > fabs(fb) && isfinite(fpa)) {
        const double s = fb / fpa;
        double p, q;
        if (pa == c || fpa == fc) {
          p = 2.0 * m * s;
          q = 1.0 - s;
        } else {
          const double qq = fpa / fc, rr = fb / fc;
          p = s * (2.0 * m * qq * (qq - rr) - (b - pa) * (rr - 1.0));
          q = (qq - 1.0) * (rr - 1.0) * (s - 1.0);
        }
        if (p > 0.0) q = -q;
        else p = -p;
        if (2.0 * p < fmin(3.0 * m * q - fabs(tolb * q), fabs(be * q))) {
          be = bd;
          step = p / q;
        } else {
          be = m;
        }
      } else {
        be = m;
      }
      bd = step;
      ba = b;
      fba = fb;
      g = b + (fabs(step) > tolb ? step : copysign(tolb, m));
    } else {
      g = lo - flo * (hi - lo) / (fhi - flo);
    }
    if (!(g == g)) g = 0.5 * (lo + hi);
    g = fmin(fmax(g, lo + 0.25 * tw), hi - 0.25 * tw);
    g_trial = g;
  }

  // per-element outputs and the block partials (min gamma, inactive count, iterations)
  const bool leader = valid && sl == 0;
  if (leader) {
    a.gamma_k[k] = gk;
    if (a.iters) a.iters[k] = its;
  }
  double gl = (leader && !isinf(gk) && gk > 0.0) ? gk : INFINITY;
  int inact = (leader && isinf(gk)) ? 1 : 0;
  int itl = leader ? its : 0;
  int its_sum = itl;
#pragma unroll
  for (int off = 32; off >= 1; off /= 2) {
    gl = fmin(gl, __shfl_xor(gl, off, 64));
    inact += __shfl_xor(inact, off, 64);
    itl = max(itl, __shfl_xor(itl, off, 64));
    its_sum += __shfl_xor(its_sum, off, 64);
  }
  __shared__ double wg[C::THREADS / 64];
  __shared__ int wi[C::THREADS / 64], wm[C::THREADS / 64], ws[C::THREADS / 64];
  if (lane == 0) {
    wg[wave] = gl;
    wi[wave] = inact;
    wm[wave] = itl;
    ws[wave] = its_sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    RelaxPart p{INFINITY, 0, 0, 0};
    for (int q = 0; q < C::THREADS / 64; ++q) {
      p.gmin = fmin(p.gmin, wg[q]);
      p.n_inactive += wi[q];
      p.max_iters = max(p.max_iters, wm[q]);
      p.sum_iters += ws[q];
    }
    a.parts[part] = p;
  }
}

template <int DIM, int N, bool NET>
__global__ void __launch_bounds__(256) relax_kernel(const MeshParams mp, const RelaxArgs a) {
  const MeshDims md = dims_of(mp);
  relax_block<DIM, N, NET>(mp, md, a, blockIdx.x * RelaxCfg<DIM, N>::EPB, blockIdx.x, 0);
}
// The same with the register budget of four waves per SIMD (one node per
// lane: 3-D p=3 fits with a few spilled setup values, so all blocks of a
// 16^3 mesh are resident at once) and of three (two nodes per lane, 3-D p=4).
template <int DIM, int N, bool NET>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
    relax_kernel_w4(const MeshParams mp, const RelaxArgs a) {
  const MeshDims md = dims_of(mp);
  relax_block<DIM, N, NET>(mp, md, a, blockIdx.x * RelaxCfg<DIM, N>::EPB, blockIdx.x, 0);
}
template <int DIM, int N, bool NET>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
    relax_kernel_w3(const MeshParams mp, const RelaxArgs a) {
  const MeshDims md = dims_of(mp);
  relax_block<DIM, N, NET>(mp, md, a, blockIdx.x * RelaxCfg<DIM, N>::EPB, blockIdx.x, 0);
}
// Brent's trial points (no network guess on this path).
template <int DIM, int N>
__global__ void __launch_bounds__(256) relax_kernel_brent(const MeshParams mp, const RelaxArgs a) {
  const MeshDims md = dims_of(mp);
  relax_block<DIM, N, false, kRuleBrent>(mp, md, a, blockIdx.x * RelaxCfg<DIM, N>::EPB,
                                         blockIdx.x, 0);
}
// Alefeld-Potra-Shi trial points (no network guess on this path).
template <int DIM, int N>
__global__ void __launch_bounds__(256) relax_kernel_alefeld(const MeshParams mp, const RelaxArgs a) {
  const MeshDims md = dims_of(mp);
  relax_block<DIM, N, false, kRuleAlefeld>(mp, md, a, blockIdx.x * RelaxCfg<DIM, N>::EPB,
                                           blockIdx.x, 0);
}

// Batched form over (simulation, first element) items; partial per item.
template <int DIM, int N>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
    relax_batch_kernel(const MeshParams mp, const RelaxArgs a0, const SimParams* __restrict__ sims,
                       const int2* __restrict__ items, int nitems) {
  // one work item per block (no block-stride loop: it made the compiler keep
  // loop-invariant constants in vector registers)
  {
    const int it = blockIdx.x;
    if (it >= nitems) return;
    // the item is the same for the whole block: keep it (and everything
    // derived from it: offsets, pointers, mesh sizes) in scalar registers
    int2 w = items[it];
    w.x = __builtin_amdgcn_readfirstlane(w.x);
    w.y = __builtin_amdgcn_readfirstlane(w.y);
    const SimParams& P = sims[w.x];
    RelaxArgs a = a0;
    a.u_old = a0.u_old + P.base;
    a.du = a0.du + P.base;
    a.deta = a0.deta ? a0.deta + P.elem_base : nullptr;
    a.phi0_in = a0.phi0_in ? a0.phi0_in + P.elem_base : nullptr;
    a.guess = a0.guess ? a0.guess + P.elem_base : nullptr;
    a.gamma_k = a0.gamma_k + P.elem_base;
    a.iters = a0.iters ? a0.iters + P.elem_base : nullptr;
    a.feats = a0.feats ? a0.feats + P.elem_base * kMlpIn : nullptr;
    a.vfeat = a0.vfeat ? a0.vfeat + P.elem_base : nullptr;
    relax_block<DIM, N, false>(mp, P.md, a, w.y, it, P.elem_base);
    __syncthreads();
  }
}

template <int DIM, int N>
static int relax_epb() {
  return RelaxCfg<DIM, N>::EPB;
}

int relax_blocks(const MeshParams& mp) {
  int epb = 1;
#define ESRK_EPB(D)                          \
  switch (mp.n) {                            \
    case 2: epb = relax_epb<D, 2>(); break;  \
    case 3: epb = relax_epb<D, 3>(); break;  \
    case 4: epb = relax_epb<D, 4>(); break;  \
    case 5: epb = relax_epb<D, 5>(); break;  \
    case 6: epb = relax_epb<D, 6>(); break;  \
  }
  if (mp.dim == 1) { ESRK_EPB(1) }
  if (mp.dim == 2) { ESRK_EPB(2) }
  if (mp.dim == 3) { ESRK_EPB(3) }
#undef ESRK_EPB
  return (mp.ne + epb - 1) / epb;
}

template <int DIM, int N>
static hipError_t relax_one(const MeshParams& mp, const RelaxArgs& a, hipStream_t s) {
  using C = RelaxCfg<DIM, N>;
  const int blocks = (mp.ne + C::EPB - 1) / C::EPB;
  if (a.model || a.feats)
    hipLaunchKernelGGL((relax_kernel<DIM, N, true>), dim3(blocks), dim3(C::THREADS), 0, s, mp, a);
  else if (a.method == ESRK_ROOT_BRENT)
    hipLaunchKernelGGL((relax_kernel_brent<DIM, N>), dim3(blocks), dim3(C::THREADS), 0, s, mp, a);
  else if (a.method == ESRK_ROOT_ALEFELD)
    hipLaunchKernelGGL((relax_kernel_alefeld<DIM, N>), dim3(blocks), dim3(C::THREADS), 0, s, mp,
                       a);
  else if constexpr (DIM == 3 && C::NPL == 1)
    hipLaunchKernelGGL((relax_kernel_w4<DIM, N, false>), dim3(blocks), dim3(C::THREADS), 0, s, mp,
                       a);
  else if constexpr (DIM == 3 && C::NPL == 2)
    hipLaunchKernelGGL((relax_kernel_w3<DIM, N, false>), dim3(blocks), dim3(C::THREADS), 0, s, mp,
                       a);
  else
    hipLaunchKernelGGL((relax_kernel<DIM, N, false>), dim3(blocks), dim3(C::THREADS), 0, s, mp, a);
  return hipGetLastError();
}

template <int DIM>
static hipError_t relax_dim(const MeshParams& mp, const RelaxArgs& a, hipStream_t s) {
  switch (mp.n) {
    case 2: return relax_one<DIM, 2>(mp, a, s);
    case 3: return relax_one<DIM, 3>(mp, a, s);
    case 4: return relax_one<DIM, 4>(mp, a, s);
    case 5: return relax_one<DIM, 5>(mp, a, s);
    case 6: return relax_one<DIM, 6>(mp, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_relax(const MeshParams& mp, const RelaxArgs& a, hipStream_t s) {
  if (mp.dim == 1) return relax_dim<1>(mp, a, s);
  if (mp.dim == 2) return relax_dim<2>(mp, a, s);
  if (mp.dim == 3) return relax_dim<3>(mp, a, s);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- bookkeeping

// Block-wide reduction helpers over 256 threads (4 waves).
__device__ __forceinline__ double block_min256(double x, double* sh) {
#pragma unroll
  for (int off = 32; off >= 1; off /= 2) x = fmin(x, __shfl_xor(x, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
  __syncthreads();
  x = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
  __syncthreads();
  return x;
}

__device__ __forceinline__ double block_sum256(double x, double* sh) {
#pragma unroll
  for (int off = 32; off >= 1; off /= 2) x += __shfl_xor(x, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
  __syncthreads();
  x = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return x;
}

// Maximum over the block's nodes of sum_m (|v_m| + c).
template <int DIM>
__global__ void __launch_bounds__(256) speed_kernel(const double* u, long long Ntot, double gg,
                                                    double* parts) {
  double best = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < Ntot;
       i += (long long)gridDim.x * blockDim.x) {
    const double rho = u[i];
    double mm = 0.0, v[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double m = u[(1 + d) * Ntot + i];
      v[d] = m / rho;
      mm += v[d] * m;
    }
    const double p = (gg - 1.0) * (u[(DIM + 1) * Ntot + i] - 0.5 * mm);
    const double c = sqrt(gg * p / rho);
    double sp = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) sp += fabs(v[d]) + c;
    best = fmax(best, sp);
  }
#pragma unroll
  for (int off = 32; off >= 1; off /= 2) best = fmax(best, __shfl_xor(best, off, 64));
  __shared__ double sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) parts[blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

hipError_t launch_speed(const MeshParams& mp, const double* u, double* parts, hipStream_t s) {
  const long long Ntot = (long long)mp.ne * mp.nd;
  if (mp.dim == 1)
    hipLaunchKernelGGL(speed_kernel<1>, dim3(kSpeedBlocks), dim3(256), 0, s, u, Ntot, mp.gg, parts);
  else if (mp.dim == 2)
    hipLaunchKernelGGL(speed_kernel<2>, dim3(kSpeedBlocks), dim3(256), 0, s, u, Ntot, mp.gg, parts);
  else
    hipLaunchKernelGGL(speed_kernel<3>, dim3(kSpeedBlocks), dim3(256), 0, s, u, Ntot, mp.gg, parts);
  return hipGetLastError();
}

// gamma = min over the relaxation partials (fixed order per block).
__device__ __forceinline__ double reduce_gamma(const RelaxPart* parts, int nparts, double* sh) {
  double g = INFINITY;
  for (int q = threadIdx.x; q < nparts; q += blockDim.x) g = fmin(g, parts[q].gmin);
  g = block_min256(g, sh);
  return isinf(g) ? 1.0 : g;
}

__global__ void __launch_bounds__(256) relax_finish_kernel(const RelaxPart* parts, int nparts,
                                                           DevScalars* s, double* gamma) {
  __shared__ double sh[4];
  const double g = reduce_gamma(parts, nparts, sh);
  if (threadIdx.x == 0) {
    s->gamma = g;
    if (gamma) *gamma = g;
  }
}

hipError_t launch_relax_finish(const RelaxPart* parts, int nparts, DevScalars* scal,
                               double* gamma, hipStream_t s) {
  hipLaunchKernelGGL(relax_finish_kernel, dim3(1), dim3(256), 0, s, parts, nparts, scal, gamma);
  return hipGetLastError();
}

// u <- u + gamma du (skipped when a device error is latched), t <- t + gamma dt.
// Every block reduces the relaxation partials itself (same order, same gamma).
__global__ void __launch_bounds__(256) apply_kernel(double* u, const double* du, long long len,
                                                    double* t, const RelaxPart* parts,
                                                    int nparts, DevScalars* s,
                                                    const double* dt_dev, double* stats_out,
                                                    int adaptive) {
  __shared__ double sh[4];
  const double g = reduce_gamma(parts, nparts, sh);
  const bool rejected = adaptive && s->rejected;
  const bool err = s->status != 0 || rejected;
  if (!err) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < len;
         i += (long long)gridDim.x * blockDim.x)
      u[i] = u[i] + g * du[i];
  }
  if (blockIdx.x == 0) {
    double inact = 0.0, isum = 0.0, imax = 0.0;
    if (stats_out) {
      for (int q = threadIdx.x; q < nparts; q += blockDim.x) {
        inact += parts[q].n_inactive;
        isum += parts[q].sum_iters;
        imax = fmax(imax, (double)parts[q].max_iters);
      }
      inact = block_sum256(inact, sh);
      isum = block_sum256(isum, sh);
      imax = -block_min256(-imax, sh);
    }
    if (threadIdx.x == 0) {
      const double dt = *dt_dev;
      double tn = *t;
      if (!err) {
        tn = tn + g * dt;
        *t = tn;
      }
      s->gamma = g;
      if (stats_out) {
        stats_out[0] = g;
        stats_out[1] = dt;
        stats_out[2] = tn;
        stats_out[3] = inact;
        stats_out[4] = imax;
        stats_out[5] = isum;
        stats_out[6] = adaptive ? s->err : 0.0;
        stats_out[7] = rejected ? 0.0 : 1.0;
      }
    }
  }
}

hipError_t launch_apply(const MeshParams& mp, double* u, const double* du, double* t,
                        const RelaxPart* parts, int nparts, DevScalars* scal,
                        const double* dt_dev, double* stats_out, int adaptive,
                        hipStream_t s) {
  const long long len = (long long)(mp.dim + 2) * mp.ne * mp.nd;
  long long blocks = (len + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(apply_kernel, dim3(blocks), dim3(256), 0, s, u, du, len, t, parts, nparts,
                     scal, dt_dev, stats_out, adaptive);
  return hipGetLastError();
}

// Error control of the embedded pairs: one block sums the per-element
// squared weighted errors in a fixed order and decides the attempt.
__global__ void __launch_bounds__(256) adapt_kernel(const double* errk, int ne, double count,
                                                    int q, int decide, DevScalars* s,
                                                    double* norm_out) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int k = threadIdx.x; k < ne; k += 256) acc += errk[k];
  acc = block_sum256(acc, sh);
  if (threadIdx.x == 0) {
    const double err = sqrt(acc / count);
    const bool ok = err <= 1.0;
    double f;
    if (!(err == err) || isinf(err))
      f = 0.1;
    else if (err > 0.0)
      f = (ok ? 0.9 : 0.45) * pow(err, -1.0 / (q + 1));
    else
      f = 10.0;
    f = fmin(10.0, fmax(0.1, f));
    if (norm_out) *norm_out = err;
    if (decide) {
      s->err = err;
      s->rejected = ok ? 0 : 1;
      s->dt_next = s->dt * f;
    }
  }
}

hipError_t launch_adapt(const double* errk, int ne, double count, int q, int decide,
                        DevScalars* scal, double* norm_out, hipStream_t s) {
  hipLaunchKernelGGL(adapt_kernel, dim3(1), dim3(256), 0, s, errk, ne, count, q, decide, scal,
                     norm_out);
  return hipGetLastError();
}

// ---- global relaxation (one gamma for the total entropy) ----
// Per node (thread per node over the whole mesh): the contributions to
//   A = sum M w(u_old).du, its round-off scale sum M |w_v du_v|, sum_k deta_k,
//   sum_k |deta_k| (first pass only) and B(g_j) = sum M [relative entropy of
//   u_old + g_j du w.r.t. u_old] for kGlobTrials trial values g_j,
// summed per block into parts[block][kGlobParts].  The trial values come from
// the host, which runs the bracket logic between passes.
template <int DIM, int N>
__global__ void __launch_bounds__(256) glob_eval_kernel(const MeshParams mp, const double* u_old,
                                                        const double* du, const double* deta,
                                                        const double* phi0_in,
                                                        const GlobState* st, double* parts) {
  if (st->stage == 3) return;  // converged: the remaining sweeps do nothing
  const int first = st->stage == 0;
  GlobTrials trials;
#pragma unroll
  for (int j = 0; j < kGlobTrials; ++j) trials.g[j] = st->g[j];
  constexpr int ND = (DIM == 1) ? N : (DIM == 2) ? N * N : N * N * N;
  constexpr int NV = DIM + 2;
  const MeshDims md = dims_of(mp);
  const int Ntot = md.ne * ND;
  const int gi = blockIdx.x * 256 + threadIdx.x;
  const bool valid = gi < Ntot;
  const double gg = mp.gg, gm1 = gg - 1.0, inv_gm1 = 1.0 / gm1;
  double acc[kGlobParts];
#pragma unroll
  for (int q = 0; q < kGlobParts; ++q) acc[q] = 0.0;
  bool bad[kGlobTrials];
#pragma unroll
  for (int j = 0; j < kGlobTrials; ++j) bad[j] = false;
  if (valid) {
    const int i = gi % ND;
    const double rho = u_old[gi], dr = du[gi];
    double mom[DIM], dm[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      mom[d] = u_old[(1 + d) * Ntot + gi];
      dm[d] = du[(1 + d) * Ntot + gi];
    }
    const double ene = u_old[(NV - 1) * Ntot + gi], dE = du[(NV - 1) * Ntot + gi];
    const double invrho = rcp_d(rho);
    double m2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) m2 += mom[d] * mom[d];
    const double p = gm1 * (ene - 0.5 * m2 * invrho);
    const double invp = rcp_d(p);
    const double beta = 0.5 * rho * invp;
    double M = 1.0;
    {
      int ii = i;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int im = ii % N;
        ii /= N;
        double wq = mp.w[0];
#pragma unroll
        for (int t = 1; t < N; ++t) wq = (im == t) ? mp.w[t] : wq;
        M *= md.half_h[d] * wq;
      }
    }
    if (first) {
      const double s_phys = log_d(p) - gg * log_d(rho);
      const double v2 = m2 * invrho * invrho;
      double t = ((gg - s_phys) * inv_gm1 - beta * v2) * dr;
      double sc = fabs(t);
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double td = 2.0 * beta * mom[d] * invrho * dm[d];
        t += td;
        sc += fabs(td);
      }
      const double te = -2.0 * beta * dE;
      t += te;
      sc += fabs(te);
      acc[1] = M * sc;
      if (phi0_in) {
        // phi(0) = sum_k phi_k(0) from the stages; the scale stays
        acc[0] = (i == 0) ? phi0_in[gi / ND] : 0.0;
      } else {
        acc[0] = M * t;
      }
      if (deta) {
        if (i == 0) {
          const double de = deta[gi / ND];
          acc[2] = phi0_in ? 0.0 : de;
          acc[3] = fabs(de);
        }
      } else {
        // no estimate passed (phi0_in given): |Delta eta_k| = |A_k - phi_k(0)|
        // is at most the element's scale plus |phi_k(0)|
        acc[1] *= 2.0;
        if (i == 0) acc[3] = fabs(phi0_in[gi / ND]);
      }
    }
#pragma unroll
    for (int j = 0; j < kGlobTrials; ++j) {
      const double g = trials.g[j];
      const double drg = g * dr;
      const double r1 = rho + drg;
      double mdm = 0.0, dm2 = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double dmg = g * dm[d];
        mdm += mom[d] * dmg;
        dm2 += dmg * dmg;
      }
      const double q = rcp_d(rho * r1);
      const double dke = (rho * (2.0 * mdm + dm2) - drg * m2) * q;
      const double dp = gm1 * (g * dE - 0.5 * dke);
      const double tr = drg * invrho;
      const double tp = dp * invp;
      const bool okn = (r1 > 0.0) && (1.0 + tp > 0.0);
      if (!okn) {
        bad[j] = true;
        continue;
      }
      const double tz = (tp - tr) * rho * rho * q;
      double dv2 = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double dv = (g * dm[d] - drg * mom[d] * invrho) * rho * q;
        dv2 += dv * dv;
      }
      double h, k;
      rel_terms(tz, tr, false, h, k);
      acc[4 + j] = M * (r1 * h * inv_gm1 + rho * k + beta * r1 * dv2);
    }
  }
  // block sums in a fixed order (inadmissible trials: +inf)
  __shared__ double red[256];
  __shared__ int sbad[kGlobTrials];
  if (threadIdx.x < kGlobTrials) sbad[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kGlobTrials; ++j)
    if (bad[j]) sbad[j] = 1;
  for (int q = 0; q < kGlobParts; ++q) {
    red[threadIdx.x] = acc[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double v = red[0];
      if (q >= 4 && sbad[q - 4]) v = INFINITY;
      parts[(long long)blockIdx.x * kGlobParts + q] = v;
    }
    __syncthreads();
  }
}

// Trial points of the next refining sweep: four points around the regula
// falsi estimate c (+-w/2, +-3w/2, w twice the last correction), or four
// evenly spaced points when the last sweep did not halve the bracket.
__device__ void glob_choose(GlobState& S, double tol) {
  const double width = S.hi - S.lo;
  const double tw = tol * fmax(1.0, S.hi);
  if (S.halved) {
    double c = isinf(S.fhi) ? 0.5 * (S.lo + S.hi) : S.lo - S.flo * width / (S.fhi - S.flo);
    if (!(c == c)) c = 0.5 * (S.lo + S.hi);
    c = fmin(fmax(c, S.lo + 0.25 * tw), S.hi - 0.25 * tw);
    double w = (S.s_prev == S.s_prev) ? 2.0 * fabs(c - S.s_prev) : 1e-3 * width;
    w = fmax(w, 0.25 * tw);
    for (int j = 0; j < kGlobTrials; ++j) {
      const double g = c + (j - 0.5 * (kGlobTrials - 1)) * w;
      S.g[j] = fmin(fmax(g, S.lo + 0.125 * tw), S.hi - 0.125 * tw);
    }
    S.s_prev = c;
  } else {
    for (int j = 0; j < kGlobTrials; ++j) S.g[j] = S.lo + (j + 1) * width / (kGlobTrials + 1);
  }
}

__device__ void glob_expand(GlobState& S, double gmax) {
  for (int j = 0; j < kGlobTrials; ++j) S.g[j] = fmin(S.lo * (double)(2 << j), gmax);
}

// Sum of the block partials (fixed order), then one step of the bracket logic
// (thread 0): inactive (gamma = 1) when B(1) is at the round-off level,
// ESRK_ENOROOT when phi(0) >= 0, bracket [0, 1] doubled up to gmax, then
// refining sweeps until the bracket is narrower than tol max(1, gamma); the
// lower end is the result.
__global__ void __launch_bounds__(256) glob_logic_kernel(const double* parts, int nparts,
                                                         GlobState* st, RelaxPart* rparts,
                                                         DevScalars* scal, int latch,
                                                         int check_reject, double tol,
                                                         double gmax, int max_passes) {
  if (st->stage == 3) return;
  __shared__ double red[256];
  __shared__ double o[kGlobParts];
  for (int q = 0; q < kGlobParts; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nparts; b += 256) s += parts[(long long)b * kGlobParts + q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) o[q] = red[0];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  GlobState S = *st;
  S.passes += 1;
  auto phi_at = [&](double g, double Bg) { return isfinite(Bg) ? S.phi0 + Bg / g : INFINITY; };
  bool done = false;
  double result = INFINITY;
  if (S.stage == 0) {
    if ((check_reject && scal->rejected) || (latch && scal->status != 0)) {
      done = true;  // nothing to relax: a rejected attempt, or an error already latched
    } else if (!isfinite(o[0]) || !isfinite(o[1]) || !isfinite(o[3])) {
      S.status = ESRK_ENAN;
      if (latch) latch_r(scal, ESRK_ENAN, 0x7fffffffffffffffLL);
      done = true;
    } else {
      S.phi0 = o[0] - o[2];
      S.noise = 64.0 * DBL_EPSILON * (o[1] + o[3]);
      const double B1 = o[4];
      if (isfinite(B1) && B1 <= S.noise) {
        result = 1.0;
        done = true;
      } else if (!(S.phi0 < 0.0)) {
        S.status = ESRK_ENOROOT;
        if (latch) latch_r(scal, ESRK_ENOROOT, 0x7fffffffffffffffLL);
        done = true;
      } else {
        S.lo = 0.0;
        S.flo = S.phi0;
        S.hi = 1.0;
        S.fhi = phi_at(1.0, B1);
        S.s_prev = NAN;
        S.halved = 1;
        if (!(S.fhi > 0.0)) {
          S.lo = 1.0;
          S.flo = S.fhi;
          S.stage = 1;
          glob_expand(S, gmax);
        } else {
          S.stage = 2;
          glob_choose(S, tol);
        }
      }
    }
  } else if (S.stage == 1) {
    bool found = false;
    for (int j = 0; j < kGlobTrials; ++j) {
      if (found) continue;
      const double f = phi_at(S.g[j], o[4 + j]);
      if (f > 0.0) {
        S.hi = S.g[j];
        S.fhi = f;
        found = true;
      } else {
        S.lo = S.g[j];
        S.flo = f;
      }
    }
    if (found) {
      S.stage = 2;
      S.halved = 1;
      S.s_prev = NAN;
      if (S.hi - S.lo <= tol * fmax(1.0, S.hi)) {
        result = S.lo;
        done = true;
      } else {
        glob_choose(S, tol);
      }
    } else if (S.lo >= gmax) {
      result = gmax;
      done = true;
    } else {
      glob_expand(S, gmax);
    }
  } else {
    const double width = S.hi - S.lo;
    for (int j = 0; j < kGlobTrials; ++j) {
      const double f = phi_at(S.g[j], o[4 + j]);
      if (f <= 0.0) {
        if (S.g[j] > S.lo) {
          S.lo = S.g[j];
          S.flo = f;
        }
      } else if (S.g[j] < S.hi) {
        S.hi = S.g[j];
        S.fhi = f;
      }
    }
    S.halved = (S.hi - S.lo) <= 0.5 * width;
    if (S.hi - S.lo <= tol * fmax(1.0, S.hi)) {
      result = S.lo;
      done = true;
    } else {
      glob_choose(S, tol);
    }
  }
  if (!done && S.passes >= max_passes) {
    result = S.lo;  // phi(lo) <= 0: the relaxed total entropy does not exceed the estimate
    done = true;
  }
  if (done) {
    S.gamma = result;
    S.stage = 3;
    rparts[0] = RelaxPart{result, 0, 0, 0};
  }
  *st = S;
}

// Starts a global solve: first sweep at gamma = 1.
__global__ void glob_init_kernel(GlobState* st, RelaxPart* rparts) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  GlobState S;
  S.lo = S.flo = S.hi = S.fhi = S.phi0 = S.noise = 0.0;
  S.s_prev = NAN;
  S.gamma = INFINITY;
  for (int j = 0; j < kGlobTrials; ++j) S.g[j] = 1.0;
  S.stage = 0;
  S.halved = 1;
  S.passes = 0;
  S.status = ESRK_OK;
  *st = S;
  rparts[0] = RelaxPart{INFINITY, 0, 0, 0};
}

// One relaxation partial carrying a given gamma (+inf: relaxation off), for
// the update kernel's reduction.
__global__ void set_part_kernel(RelaxPart* parts, double g) {
  if (threadIdx.x == 0 && blockIdx.x == 0) parts[0] = RelaxPart{g, 0, 0, 0};
}

int glob_blocks(const MeshParams& mp) { return (mp.ne * mp.nd + 255) / 256; }

hipError_t launch_glob_solve(const MeshParams& mp, const double* u_old, const double* du,
                             const double* deta, const double* phi0_in, GlobState* st,
                             double* parts, RelaxPart* rparts, DevScalars* scal, int latch,
                             int check_reject, double tol, double gmax, int max_passes,
                             hipStream_t s) {
  const int blocks = glob_blocks(mp);
  hipLaunchKernelGGL(glob_init_kernel, dim3(1), dim3(64), 0, s, st, rparts);
  hipError_t e = hipGetLastError();
  for (int pass = 0; pass < max_passes && e == hipSuccess; ++pass) {
#define ESRK_GE(D, NN)                                                                  \
  hipLaunchKernelGGL((glob_eval_kernel<D, NN>), dim3(blocks), dim3(256), 0, s, mp, u_old, \
                     du, deta, phi0_in, st, parts)
#define ESRK_GD(D)                     \
  switch (mp.n) {                      \
    case 2: ESRK_GE(D, 2); break;      \
    case 3: ESRK_GE(D, 3); break;      \
    case 4: ESRK_GE(D, 4); break;      \
    case 5: ESRK_GE(D, 5); break;      \
    case 6: ESRK_GE(D, 6); break;      \
    default: return hipErrorInvalidValue; \
  }
    if (mp.dim == 1) { ESRK_GD(1) } else if (mp.dim == 2) { ESRK_GD(2) } else { ESRK_GD(3) }
#undef ESRK_GD
#undef ESRK_GE
    e = hipGetLastError();
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(glob_logic_kernel, dim3(1), dim3(256), 0, s, parts, blocks, st, rparts,
                       scal, latch, check_reject, tol, gmax, max_passes);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_set_part(RelaxPart* parts, double g, hipStream_t s) {
  hipLaunchKernelGGL(set_part_kernel, dim3(1), dim3(64), 0, s, parts, g);
  return hipGetLastError();
}

// ---- batched relaxation launch (2-D meshes) ----
int relax_batch_epb(const MeshParams& mp) {
  switch (mp.n) {
    case 2: return RelaxCfg<2, 2>::EPB;
    case 3: return RelaxCfg<2, 3>::EPB;
    case 4: return RelaxCfg<2, 4>::EPB;
    case 5: return RelaxCfg<2, 5>::EPB;
    case 6: return RelaxCfg<2, 6>::EPB;
  }
  return 0;
}

hipError_t launch_relax_batch(const MeshParams& mp, const RelaxArgs& a, const SimParams* sims,
                              const int2* items, int nitems, int grid, hipStream_t s) {
  if (mp.dim != 2) return hipErrorInvalidValue;
  if (nitems <= 0) return hipSuccess;
  grid = nitems;  // one block per item
  switch (mp.n) {
    case 2: hipLaunchKernelGGL((relax_batch_kernel<2, 2>), dim3(grid), dim3(256), 0, s, mp, a, sims, items, nitems); break;
    case 3: hipLaunchKernelGGL((relax_batch_kernel<2, 3>), dim3(grid), dim3(256), 0, s, mp, a, sims, items, nitems); break;
    case 4: hipLaunchKernelGGL((relax_batch_kernel<2, 4>), dim3(grid), dim3(256), 0, s, mp, a, sims, items, nitems); break;
    case 5: hipLaunchKernelGGL((relax_batch_kernel<2, 5>), dim3(grid), dim3(256), 0, s, mp, a, sims, items, nitems); break;
    case 6: hipLaunchKernelGGL((relax_batch_kernel<2, 6>), dim3(grid), dim3(256), 0, s, mp, a, sims, items, nitems); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Batched wave-speed maxima: items (simulation, first node) of 256 nodes each.
__global__ void __launch_bounds__(256) speed_batch_kernel(const double* u, double gg,
                                                          const SimParams* __restrict__ sims,
                                                          const int2* __restrict__ items,
                                                          int nitems, int nd, double* parts) {
  __shared__ double sh[4];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    // the item is the same for the whole block: keep it (and everything
    // derived from it: offsets, pointers, mesh sizes) in scalar registers
    int2 w = items[it];
    w.x = __builtin_amdgcn_readfirstlane(w.x);
    w.y = __builtin_amdgcn_readfirstlane(w.y);
    const SimParams& P = sims[w.x];
    const long long Ntot = (long long)P.md.ne * nd;
    const long long i = (long long)w.y + threadIdx.x;
    double best = 0.0;
    if (i < Ntot) {
      const double* us = u + P.base;
      const double rho = us[i];
      double mm = 0.0, v[2];
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const double m = us[(1 + d) * Ntot + i];
        v[d] = m / rho;
        mm += v[d] * m;
      }
      const double p = (gg - 1.0) * (us[3 * Ntot + i] - 0.5 * mm);
      const double c = sqrt(gg * p / rho);
      best = (fabs(v[0]) + c) + (fabs(v[1]) + c);
    }
#pragma unroll
    for (int off = 32; off >= 1; off /= 2) best = fmax(best, __shfl_xor(best, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) parts[it] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
  }
}

hipError_t launch_speed_batch(const MeshParams& mp, const double* u, const SimParams* sims,
                              const int2* items, int nitems, int grid, double* parts,
                              hipStream_t s) {
  hipLaunchKernelGGL(speed_batch_kernel, dim3(grid), dim3(256), 0, s, u, mp.gg, sims, items,
                     nitems, mp.nd, parts);
  return hipGetLastError();
}

// Batched relaxed update: items (simulation, first node) of 256 nodes; every
// block reduces its simulation's relaxation partials (fixed order).
__global__ void __launch_bounds__(256) apply_batch_kernel(double* u, const double* du, int nv,
                                                          const SimParams* __restrict__ sims,
                                                          const int2* __restrict__ items,
                                                          int nitems, int nd,
                                                          const RelaxPart* parts, DevScalars* s,
                                                          const double* dt_sims, double* t,
                                                          double* gamma_out) {
  __shared__ double sh[4];
  const bool err = s->status != 0;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    // the item is the same for the whole block: keep it (and everything
    // derived from it: offsets, pointers, mesh sizes) in scalar registers
    int2 w = items[it];
    w.x = __builtin_amdgcn_readfirstlane(w.x);
    w.y = __builtin_amdgcn_readfirstlane(w.y);
    const SimParams& P = sims[w.x];
    double g = INFINITY;
    for (int q = P.relax_p0 + threadIdx.x; q < P.relax_p1; q += blockDim.x)
      g = fmin(g, parts[q].gmin);
    g = block_min256(g, sh);
    if (isinf(g)) g = 1.0;
    const long long Ntot = (long long)P.md.ne * nd;
    const long long i = (long long)w.y + threadIdx.x;
    if (!err && i < Ntot) {
      for (int v = 0; v < nv; ++v) {
        const long long q = P.base + v * Ntot + i;
        u[q] = u[q] + g * du[q];
      }
    }
    if (w.y == 0 && threadIdx.x == 0) {
      if (!err) t[w.x] = t[w.x] + g * dt_sims[w.x];
      if (gamma_out) gamma_out[w.x] = g;
    }
  }
}

hipError_t launch_apply_batch(const MeshParams& mp, double* u, const double* du,
                              const SimParams* sims, const int2* items, int nitems, int grid,
                              const RelaxPart* parts, DevScalars* scal, const double* dt_sims,
                              double* t, double* gamma_out, hipStream_t s) {
  hipLaunchKernelGGL(apply_batch_kernel, dim3(grid), dim3(256), 0, s, u, du, mp.dim + 2, sims,
                     items, nitems, mp.nd, parts, scal, dt_sims, t, gamma_out);
  return hipGetLastError();
}

}  // namespace esrk
