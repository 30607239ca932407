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
//   Gaussian (y - mu)^2.  For the log link log(mu) is the clamped eta itself;
//   the NB term uses (y+a)/(mu+a) = 1 + (y-mu)/(mu+a) and a log1p that keeps
//   full relative accuracy when y is close to mu (and at y = 0).
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

// log(1 + x) for x > -1: series for |x| < 1/8 (truncation below 1e-8
// relative), the logarithm of 1 + x otherwise.  Branch free.
__device__ __forceinline__ float log1p_small(float x) {
  float p = fmaf(x, -0.125f, 0.14285714f);
  p = fmaf(x, p, -0.16666667f);
  p = fmaf(x, p, 0.2f);
  p = fmaf(x, p, -0.25f);
  p = fmaf(x, p, 0.33333333f);
  p = fmaf(x, p, -0.5f);
  p = fmaf(x, p, 1.0f);
  const float series = x * p;
  const float direct = fast_log(1.0f + x);
  return (fabsf(x) < 0.125f) ? series : direct;
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
    const float mu = fast_exp(ec);
    if constexpr (FAM == kPoisson) {
      const float wp = w * c.phi_inv;
      d1 = wp * (mu - y);
      d2 = wp * mu;
      if constexpr (WANT_DEV) {
        const float ly = fast_log(fmaxf(y, 1.0f));
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
        // y log(y/mu) - (y+a) log((y+a)/(mu+a)) with log(mu) = ec and
        // (y+a)/(mu+a) = 1 + (y - mu)/(mu + a)
        const float ylogy = (y > 0.f) ? y * fast_log(y) : 0.f;
        const float t = ylogy - y * ec - (y + c.a) * log1p_small((y - mu) * inv);
        dev = 2.f * w * t;
      }
    }
  }
}

}  // namespace gmf
