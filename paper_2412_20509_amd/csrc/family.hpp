// Per-entry family algebra on the device: inverse link, the first derivative
// and Fisher weight of the per-entry negative log-likelihood in eta, and the
// unit deviance.
//
//   D1 = -w (y - mu) / (phi nu(mu) g'(mu)),   D2 = w / (phi nu(mu) g'(mu)^2)
//   (Section 3, the derivatives of the deviance in the linear predictor, with
//   the sign of the negative log-likelihood; Fisher form, alpha(mu) = 1).
//
//   Poisson, log link:   nu = mu,               g' = 1/mu  -> D1 = w(mu - y)/phi,
//                                                             D2 = w mu/phi
//   NB(alpha), log link: nu = mu(1 + mu/alpha), g' = 1/mu  -> D1 = w alpha (mu - y)/((alpha+mu) phi),
//                                                             D2 = w alpha mu/((alpha+mu) phi)
//   Gaussian, identity:  nu = 1,                g' = 1     -> D1 = w (mu - y)/phi, D2 = w/phi
//
//   Unit deviances (Supplementary Table 1 times 2; NB form of Appendix B):
//   Poisson 2[y log(y/mu) - (y - mu)], NB 2[y log(y/mu) - (y+a) log((y+a)/(mu+a))],
//   Gaussian (y - mu)^2.  For the log link log(mu) is the clamped eta itself.
//   The Poisson and NB deviances split into a part that depends on the count
//   only and a part that depends on mu (using (y+a)/(mu+a) = (1 + y/a)/(1 + mu/a)):
//     Poisson  D/2 = c(y) + [mu - y log mu],                 c(y) = y log y - y,
//     NB       D/2 = c(y) + [(y+a) log1p(mu/a) - y log mu],  c(y) = y log y - (y+a) log1p(y/a),
//   with c(0) = 0.  The per-entry epilogue forms only the mu part ("dev" below);
//   sums of w c(y) over a block never change during a fit, so they are formed
//   once, in float64, and added to the block and full deviances.
//   log1p(mu/a) is log(q) for the rounded q = 1 + mu/a plus the correction
//   for that rounding, which keeps full relative accuracy for small mu/a (the
//   zero counts); 1/q = a/(a + mu) reuses the reciprocal of the Fisher weight.
//
// Arithmetic: the hardware exp2 / log2 / reciprocal instructions (1-ulp
// class, no denormal range reduction: every argument here is a normal number),
// float32 per entry; the callers accumulate deviances in float64.
#pragma once

#include <hip/hip_runtime.h>

#include "gmf_kernels.hpp"

namespace gmf {

__device__ __forceinline__ float fast_exp(float x) {
  return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
}
__device__ __forceinline__ float fast_log(float x) {
  return __builtin_amdgcn_logf(x) * 0.6931471805599453f;
}

// log(1 + z) for z >= 0 given inv_q = 1/(1 + z): the logarithm of the rounded
// q = 1 + z plus the first-order correction for that rounding, (z - (q - 1))/q
// (q - 1 is exact); accurate to a few ulps of log(1 + z) for every z >= 0.
__device__ __forceinline__ float log1p_pos(float z, float inv_q) {
  const float q = 1.0f + z;
  return fmaf(z - (q - 1.0f), inv_q, fast_log(q));
}

// Per-launch constants of the epilogue.
struct FamilyConst {
  float phi_inv, a, a_phi, inv_a, lo, hi;
};

__device__ __forceinline__ FamilyConst family_const(const FamilyArgs& f) {
  FamilyConst c;
  c.phi_inv = f.phi_inv;
  c.a = f.nb_alpha;
  c.a_phi = f.nb_alpha * f.phi_inv;
  c.inv_a = 1.0f / f.nb_alpha;
  c.lo = f.eta_lo;
  c.hi = f.eta_hi;
  return c;
}

// The count-only part c(y) of half the unit deviance (see above), float64.
template <int FAM>
__device__ __forceinline__ double count_part(double y, double a) {
  if (FAM == kGaussian || y <= 0.0) return 0.0;
  if constexpr (FAM == kPoisson) return y * log(y) - y;
  else return y * log(y) - (y + a) * log1p(y / a);
}

// eta: linear predictor, y: response, w: weight (1 when there are none).
// dev (WANT_DEV): the mu part of the unit deviance times w -- the full unit
// deviance for the Gaussian family, 2 w [D/2 - c(y)] for Poisson and NB
// (HALF: without that factor 2, which the caller applies to its float sum;
// doubling is exact, so both give the same sums).
template <int FAM, bool WANT_DEV, bool HALF = false>
__device__ __forceinline__ void family_entry(float eta, float y, float w, const FamilyConst& c,
                                             float& d1, float& d2, float& dev) {
  if constexpr (FAM == kGaussian) {
    const float r = eta - y;
    const float wp = w * c.phi_inv;
    d1 = wp * r;
    d2 = wp;
    if constexpr (WANT_DEV) dev = w * r * r;
  } else {
    const float ec = __builtin_amdgcn_fmed3f(eta, c.lo, c.hi);   // clamp to [lo, hi]
    const float mu = fast_exp(ec);
    if constexpr (FAM == kPoisson) {
      const float wp = w * c.phi_inv;
      d1 = wp * (mu - y);
      d2 = wp * mu;
      if constexpr (WANT_DEV) {
        dev = (HALF ? 1.f : 2.f) * w * fmaf(-y, ec, mu);
      }
    } else {
      const float s = c.a + mu;
      const float inv = __builtin_amdgcn_rcpf(s);
      const float wa = w * c.a_phi * inv;
      d1 = wa * (mu - y);
      d2 = wa * mu;
      if constexpr (WANT_DEV) {
        dev = (HALF ? 1.f : 2.f) * w * fmaf(y + c.a, log1p_pos(mu * c.inv_a, c.a * inv), -y * ec);
      }
    }
  }
}

}  // namespace gmf
