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
//   Gaussian (y - mu)^2.  For the log link log(mu) is the clamped eta itself.
#pragma once

#include <hip/hip_runtime.h>

#include "gmf_kernels.hpp"

namespace gmf {

template <int FAM>
struct EntryOut {
  float d1, d2, dev;
};

// eta: linear predictor, y: response, w: weight.  dev is only formed when
// want_dev is true.
template <int FAM>
__device__ __forceinline__ void family_entry(float eta, float y, float w,
                                             const FamilyArgs& f, bool want_dev,
                                             float& d1, float& d2, float& dev) {
  if constexpr (FAM == kGaussian) {
    const float mu = eta;
    const float r = mu - y;
    const float wp = w * f.phi_inv;
    d1 = wp * r;
    d2 = wp;
    if (want_dev) dev = w * r * r;
  } else {
    const float ec = fminf(fmaxf(eta, f.eta_lo), f.eta_hi);
    const float mu = __expf(ec);
    const float wp = w * f.phi_inv;
    if constexpr (FAM == kPoisson) {
      d1 = wp * (mu - y);
      d2 = wp * mu;
      if (want_dev) {
        // y log(y/mu) - (y - mu), with log(mu) = ec and the y = 0 limit mu
        const float t = (y > 0.f) ? y * (__logf(y) - ec) - (y - mu) : mu;
        dev = 2.f * w * t;
      }
    } else {
      const float a = f.nb_alpha;
      const float inv = 1.0f / (a + mu);
      const float wa = wp * a * inv;
      d1 = wa * (mu - y);
      d2 = wa * mu;
      if (want_dev) {
        float t;
        if (y > 0.f) {
          t = y * (__logf(y) - ec) - (y + a) * (__logf(y + a) - __logf(mu + a));
        } else {
          t = a * log1pf(mu / a);   // (y + a) log((mu + a)/a) at y = 0
        }
        dev = 2.f * w * t;
      }
    }
  }
}

}  // namespace gmf
