// Loop derivative of one (q, p) pair: temperature flow (below) and Omega
// cutoff at zero temperature (at the end of this file).
//
// With alpha = eps(p + q/2)/(2T), beta = eps(p - q/2)/(2T) and
// h(y) = y sech^2(y), the T-derivatives of the Matsubara-summed loops of
// eqn. chis are divided differences of h:
//   dL^ph/dT = +Dh(alpha, beta)  / (4 T^2),
//   dL^pp/dT = -Dh(alpha, -beta) / (4 T^2),
//   Dh(a, b) = (h(a) - h(b)) / (a - b).
// (L^ph = (n_F(eps1) - n_F(eps2))/(eps1 - eps2), L^pp = (1 - n_F(eps1) -
// n_F(eps2))/(eps1 + eps2); d/dT at fixed energies.)  Close to the
// diagonal (|a - b| < tau) the divided difference cancels, and the exact
// identity
//   Dh(a, b) = sech^2 b - a (tanh a + tanh b) sinhc(a - b) sech a sech b
// is used instead; it involves only bounded factors, so nothing overflows
// at |eps/T| ~ 1e4.  Both branches are accurate to a few ulp of max |Dh|.
//
// The functions compile for host and device; the reciprocal is a template
// parameter so that the device can use its hardware reciprocal.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace tufrg {

struct IeeeRcp {
  __host__ __device__ double operator()(double x) const { return 1.0 / x; }
};

// e^{-x} for x >= 0 by Cody-Waite argument reduction: k = rint(x / ln2),
// r = k ln2 - x in [-ln2/2, ln2/2] with ln2 split into a high part exact in
// k * ln2_hi and a low part (fdlibm's split), e^{-x} = 2^{-k} e^{r}, and e^{r}
// from its degree-13 Taylor polynomial (truncation < 5e-18).
__host__ __device__ inline double exp_neg(double x) {
  const double kLn2Hi = 6.93147180369123816490e-01;
  const double kLn2Lo = 1.90821492927058770002e-10;
  const double kInvLn2 = 1.44269504088896338700e+00;
  x = fmin(x, 746.0);
  const double k = rint(x * kInvLn2);
  double r = fma(k, kLn2Hi, -x);
  r = fma(k, kLn2Lo, r);           // r = k ln2 - x in [-ln2/2, ln2/2]
  double p = 1.0 / 6227020800.0;   // 1/13!
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, -(int)k);        // e^{-x} = 2^{-k} e^{r}
}

// sinh(d)/d for |d| < 1/4: Taylor series to d^12 (next term < 1e-17)
__host__ __device__ inline double sinhc_small(double d) {
  const double z = d * d;
  double p = 1.0 / 6227020800.0;
  p = fma(p, z, 1.0 / 39916800.0);
  p = fma(p, z, 1.0 / 362880.0);
  p = fma(p, z, 1.0 / 5040.0);
  p = fma(p, z, 1.0 / 120.0);
  p = fma(p, z, 1.0 / 6.0);
  return fma(p, z, 1.0);
}

constexpr double kNearDiag = 0.25;

// Dh(a, b) and Dh(a, -b) (the ph and pp divided differences).  Two refined
// reciprocals per pair: 1/(1+qa) and 1/(1+qb) come from the reciprocal of
// their product (in [1, 4]), and the two far-branch divisors from the
// reciprocal of theirs (a divisor the near form replaces counts as 1, so the
// product lies in [1/16, ~1e8] for |eps/T| up to ~1e4).  The near form is a
// branch of its own: a wave runs it only when one of its pairs needs it.
template <class Rcp>
__host__ __device__ inline void loop_dot_pair_t(double a, double b, double& dph, double& dpp,
                                                Rcp rcp) {
  const double ea = exp_neg(fabs(a)), eb = exp_neg(fabs(b));   // e^{-|a|}, e^{-|b|}
  const double qa = ea * ea, qb = eb * eb;
  const double pa = 1.0 + qa, pb = 1.0 + qb;
  const double rab = rcp(pa * pb);
  const double ra = rab * pb, rb = rab * pa;                   // 1/(1+qa), 1/(1+qb)
  const double sa = 2.0 * ea * ra, sb = 2.0 * eb * rb;        // sech
  const double ta = copysign((1.0 - qa) * ra, a);              // tanh
  const double tb = copysign((1.0 - qb) * rb, b);
  const double s2b = sb * sb;
  const double ha = a * sa * sa, hb = b * s2b;                 // h = y sech^2 y
  const double sab = a * sa * sb;
  const double dm = a - b, dp = a + b;
  const bool near_m = fabs(dm) < kNearDiag, near_p = fabs(dp) < kNearDiag;
  // far from the diagonal: plain divided differences
  const double gm = near_m ? 1.0 : dm, gp = near_p ? 1.0 : dp;
  const double rmp = rcp(gm * gp);
  dph = (ha - hb) * (gp * rmp);
  dpp = (ha + hb) * (gm * rmp);
  // near the diagonal: bounded identity
  if (near_m || near_p) {
    if (near_m) dph = fma(-sab * (ta + tb), sinhc_small(dm), s2b);
    if (near_p) dpp = fma(-sab * (ta - tb), sinhc_small(dp), s2b);
  }
}

}  // namespace tufrg

namespace tufrg {

// ------------------------------------------------------------- FP32 form
// The same divided differences in single precision, for the mixed-precision
// loops.  The caller forms a = alpha, b = beta and dm = alpha - beta,
// dp = alpha + beta in FP64 (the energies carry |eps/T| up to ~1e4 at the
// lowest temperatures, where FP32 energies would lose the Fermi surface) and
// passes them rounded to FP32.  Exp2 and the reciprocal are template
// parameters (hardware v_exp_f32 / v_rcp_f32 on the device, libm on the host).
template <class Exp2, class Rcp>
__host__ __device__ inline void loop_dot_pair_f32(float a, float b, float dm, float dp, float& dph,
                                                  float& dpp, Exp2 ex2, Rcp rcp) {
  const float kLog2e = 1.44269504088896341f;
  const float ea = ex2(-fabsf(a) * kLog2e), eb = ex2(-fabsf(b) * kLog2e);   // e^{-|a|}, e^{-|b|}
  const float qa = ea * ea, qb = eb * eb;
  const float ra = rcp(1.0f + qa), rb = rcp(1.0f + qb);
  const float sa = 2.0f * ea * ra, sb = 2.0f * eb * rb;                      // sech
  const float ta = copysignf((1.0f - qa) * ra, a);                             // tanh
  const float tb = copysignf((1.0f - qb) * rb, b);
  const float s2b = sb * sb;
  const float ha = a * sa * sa, hb = b * s2b;                                  // y sech^2 y
  const float sab = a * sa * sb;
  const float far_ph = (ha - hb) * rcp(dm);
  const float far_pp = (ha + hb) * rcp(dp);
  // The near-diagonal branch reaches out to |d| < 1 in single precision, so
  // the far branch's cancellation is amplified by at most max|h|/1 (FP64 uses
  // 1/4 with a shorter series).  sinh(d)/d to d^12 (next term < 2e-10 at |d| = 1).
  auto sinhc1 = [](float d) {
    const float z = d * d;
    float p = 1.0f / 6227020800.0f;
    p = fmaf(p, z, 1.0f / 39916800.0f);
    p = fmaf(p, z, 1.0f / 362880.0f);
    p = fmaf(p, z, 1.0f / 5040.0f);
    p = fmaf(p, z, 1.0f / 120.0f);
    p = fmaf(p, z, 1.0f / 6.0f);
    return fmaf(p, z, 1.0f);
  };
  const float near_ph = fmaf(-sab * (ta + tb), sinhc1(dm), s2b);
  const float near_pp = fmaf(-sab * (ta - tb), sinhc1(dp), s2b);
  dph = fabsf(dm) < 1.0f ? near_ph : far_ph;
  dpp = fabsf(dp) < 1.0f ? near_pp : far_pp;
}

}  // namespace tufrg

namespace tufrg {

// ------------------------------------------------- Omega cutoff at T = 0
// With the regulated propagator G = chi(w)/(i w - eps), chi(w) = w^2/(w^2 +
// Om^2), the loops are integrals over real frequencies, and their
// Omega-derivatives are divided differences of one odd function: with
// x = eps1/Om, y = eps2/Om,
//   dL^ph/dOm = +Df(x, y)  / (4 Om^2),
//   dL^pp/dOm = -Df(x, -y) / (4 Om^2),
//   f(v) = v (1 + 3|v|) / (1 + |v|)^3,   Df(x, y) = (f(x) - f(y))/(x - y),
// the structure of the temperature flow with h -> f and eps/(2T) -> eps/Om.
// With u = 1/(1+|x|), w = 1/(1+|y|), a = |x| u, b = |y| w (all in [0, 1]):
//   x, y of one sign:       Df = u w (1 + a + b - 2 (a^2 + a b + b^2))
//     (an exact rational identity: f(x) - f(y) never cancels),
//   x, y of opposite signs: Df = (a u (3 - 2u) + b w (3 - 2w)) / (|x| + |y|)
//     (a weighted mean of bounded terms; f(|x|) = a u (3 - 2u)).
// Both channels share u, w, a and b: ph takes the one-sign form when
// x y >= 0, pp (y -> -y) when x y <= 0.
template <class Rcp>
__host__ __device__ inline void omega_dot_pair_t(double x, double y, double& dph, double& dpp,
                                                 Rcp rcp) {
  const double ax = fabs(x), ay = fabs(y);
  const double u = rcp(1.0 + ax), w = rcp(1.0 + ay);
  const double a = ax * u, b = ay * w;
  const double one = u * w * (1.0 + a + b - 2.0 * (a * a + a * b + b * b));
  const double den = ax + ay;
  const double opp = (a * u * (3.0 - 2.0 * u) + b * w * (3.0 - 2.0 * w)) * rcp(den > 0.0 ? den : 1.0);
  const double xy = x * y;
  dph = xy >= 0.0 ? one : opp;
  dpp = xy <= 0.0 ? one : opp;
}

// The same in single precision (mixed-precision loops); x and y are formed
// in FP64 and rounded.
template <class Rcp>
__host__ __device__ inline void omega_dot_pair_f32(float x, float y, float& dph, float& dpp, Rcp rcp) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float u = rcp(1.0f + ax), w = rcp(1.0f + ay);
  const float a = ax * u, b = ay * w;
  const float one = u * w * (1.0f + a + b - 2.0f * (a * a + a * b + b * b));
  const float den = ax + ay;
  const float opp = (a * u * (3.0f - 2.0f * u) + b * w * (3.0f - 2.0f * w)) * rcp(den > 0.0f ? den : 1.0f);
  const float xy = x * y;
  dph = xy >= 0.0f ? one : opp;
  dpp = xy <= 0.0f ? one : opp;
}

}  // namespace tufrg
