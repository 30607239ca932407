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
//   Unit deviances (Supplementary Table 1 times 2; NB form of Appendix A):
//   Poisson 2[y log(y/mu) - (y - mu)], NB 2[y log(y/mu) - (y+a) log((y+a)/(mu+a))],
//   Gaussian (y - mu)^2.  For the log link log(mu) is the clamped eta itself;
//   at y = 0 the NB term is 2 a log(1 + mu/a), formed without cancellation.
//
// Arithmetic: hardware exp2/log2/reciprocal (1-ulp class), float32 per entry;
// the callers accumulate deviances in float64.
#pragma once

#include <hip/hip_runtime.h>

#include "gmf_kernels.hpp"

namespace gmf {

// log(1 + x) for x >= 0: series below 1/8 (truncation < 1e-8 relative),
// the logarithm of 1 + x above.  Branch free.
__device__ __forceinline__ float log1p_nonneg(float x) {
  float p = fmaf(x, -0.125f, 0.14285714f);
  p = fmaf(x, p, -0.16666667f);
  p = fmaf(x, p, 0.2f);
  p = fmaf(x, p, -0.25f);
  p = fmaf(x, p, 0.33333333f);
  p = fmaf(x, p, -0.5f);
  p = fmaf(x, p, 1.0f);
  const float series = x * p;
  const float direct = __logf(1.0f + x);
  return (x < 0.125f) ? series : direct;
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

// eta: linear predictor, y: response, w: weight (1 when there are none).
template <int FAM, bool WANT_DEV>
__device__ __forceinline__ void family_entry(float eta, float y, float w, const FamilyConst& c,
                                             float& d1, float& d2, float& dev) {
  if constexpr (FAM == kGaussian) {
    const float r = eta - y;
    const float wp = w * c.phi_inv;
    d1 = wp * r;
    d2 = wp;
    if constexpr (WANT_DEV) dev = w * r * r;
  } else {
    const float ec = fminf(fmaxf(eta, c.lo), c.hi);
    const float mu = __expf(ec);
    if constexpr (FAM == kPoisson) {
      const float wp = w * c.phi_inv;
      d1 = wp * (mu - y);
      d2 = wp * mu;
      if constexpr (WANT_DEV) {
        const float ly = __logf(fmaxf(y, 1.0f));
        const float t = (y > 0.f) ? fmaf(y, ly - ec, mu - y) : mu;
        dev = 2.f * w * t;
      }
    } else {
      const float s = c.a + mu;
      const float inv = __builtin_amdgcn_rcpf(s);
      const float wa = w * c.a_phi * inv;
      d1 = wa * (mu - y);
      d2 = wa * mu;
      if constexpr (WANT_DEV) {
        const float ly = __logf(fmaxf(y, 1.0f));
        const float pos = y * (ly - ec) - (y + c.a) * (__logf(y + c.a) - __logf(s));
        const float zero = c.a * log1p_nonneg(mu * c.inv_a);
        dev = 2.f * w * ((y > 0.f) ? pos : zero);
      }
    }
  }
}

}  // namespace gmf
