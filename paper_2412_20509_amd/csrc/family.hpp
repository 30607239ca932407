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
//   In the NB step epilogue log1p(mu/a) is log2 of q = 1 + mu/a rounded
//   once (a fused multiply-add), and the mu part is formed in base-2 units,
//   (y+a) log2(q) - y t with t = eta log2(e) (the exponent of mu), times ln 2:
//   the rounding of q costs at most 2^-24 absolute in log(q), unbiased, so
//   per entry at most (y + a) 2^-24 of the deviance.  The generic path keeps
//   the correction for that rounding (log1p_pos).
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
  int code, link;
  const float* alpha_col;
};

__device__ __forceinline__ FamilyConst family_const(const FamilyArgs& f) {
  FamilyConst c;
  float phi_inv = f.phi_inv, a = f.nb_alpha;
  if (f.est) {   // dispersion and NB shape as currently estimated
    phi_inv = (float)(1.0 / f.est[0]);
    a = (float)f.est[1];
  }
  c.phi_inv = phi_inv;
  c.a = a;
  c.a_phi = a * phi_inv;
  c.inv_a = 1.0f / a;
  c.lo = f.eta_lo;
  c.hi = f.eta_hi;
  c.code = f.code;
  c.link = f.link;
  c.alpha_col = f.alpha_col;
  return c;
}

// NB shape of permuted column `col` on the generic path.
__device__ __forceinline__ float column_alpha(const FamilyConst& c, int64_t col) {
  return c.alpha_col ? c.alpha_col[col] : c.a;
}

// The count-only part c(y) of half the unit deviance (see above), float64.
template <int FAM>
__device__ __forceinline__ double count_part(double y, double a) {
  if (FAM == kGaussian || y <= 0.0) return 0.0;
  if constexpr (FAM == kPoisson) return y * log(y) - y;
  else return y * log(y) - (y + a) * log1p(y / a);
}

// The count-only part c(y) of half the unit deviance on the generic path
// (float64): Poisson y log y - y, NB y log y - (y+a) log1p(y/a), Gamma
// -1 - log y, inverse Gaussian 1/(2y), Gaussian and Bernoulli 0; 0 for a
// missing entry.
__device__ __forceinline__ double count_part_generic(int code, double y, double a) {
  if (!(y == y)) return 0.0;
  switch (code) {
    case kCodePoisson: return y > 0.0 ? y * log(y) - y : 0.0;
    case kCodeNegBin: return y > 0.0 ? y * log(y) - (y + a) * log1p(y / a) : 0.0;
    case kCodeGamma: return -1.0 - log(y);
    case kCodeInvGauss: return 0.5 / y;
    default: return 0.0;
  }
}

// log(1 + e^x) without overflow.
__device__ __forceinline__ float softplus(float x) {
  const float z = fast_exp(-fabsf(x));
  return fmaxf(x, 0.f) + log1p_pos(z, __builtin_amdgcn_rcpf(1.0f + z));
}

// Generic epilogue: the six families with their links (Poisson, NB, Gamma and
// inverse Gaussian with the log link, Gaussian with the identity link,
// Bernoulli with the logit link), alpha the entry's NB shape.  A missing entry
// (y NaN) is imputed by its mean, y <- mu (Section 3.2.2): D1 = 0, D2 the
// Fisher weight at mu, no deviance.  dev: w times the mu part of half the
// unit deviance (HALF), or of the unit deviance:
//   Gamma     D/2 = c(y) + y/mu + log mu
//   inv. Gau. D/2 = c(y) + y/(2 mu^2) - 1/mu
//   Bernoulli D/2 = y softplus(-eta) + (1 - y) softplus(eta)   (c = 0)
//   Gaussian  D/2 = (y - mu)^2 / 2                             (c = 0)
// and D1, D2 = -w (y - mu)/(phi nu g'), w/(phi nu g'^2):
//   Gamma-log D1 = w (1 - y/mu)/phi, D2 = w/phi; inv. Gaussian-log
//   D1 = w (mu - y)/(phi mu^2), D2 = w/(phi mu); Bernoulli-logit
//   D1 = w (mu - y)/phi, D2 = w mu (1 - mu)/phi.
template <bool WANT_DEV, bool HALF = false>
__device__ __forceinline__ void family_entry_generic(float eta, float y, float w, float alpha,
                                                     const FamilyConst& c, float& d1, float& d2,
                                                     float& dev) {
  const bool miss = !(y == y);
  float ec, mu;
  if (c.link == kLinkIdentity) {
    ec = eta;
    mu = eta;
  } else if (c.link == kLinkLogit) {
    ec = __builtin_amdgcn_fmed3f(eta, -c.hi, c.hi);
    mu = __builtin_amdgcn_rcpf(1.0f + fast_exp(-ec));
  } else {
    ec = __builtin_amdgcn_fmed3f(eta, c.lo, c.hi);
    mu = fast_exp(ec);
  }
  const float yy = miss ? mu : y;
  const float wp = w * c.phi_inv;
  float dh = 0.f;
  switch (c.code) {
    case kCodePoisson:
      d1 = wp * (mu - yy);
      d2 = wp * mu;
      dh = fmaf(-yy, ec, mu);
      break;
    case kCodeNegBin: {
      const float inv = __builtin_amdgcn_rcpf(alpha + mu);
      const float wa = wp * alpha * inv;
      d1 = wa * (mu - yy);
      d2 = wa * mu;
      dh = fmaf(yy + alpha, log1p_pos(mu / alpha, alpha * inv), -yy * ec);
      break;
    }
    case kCodeGamma: {
      const float r = yy * __builtin_amdgcn_rcpf(mu);
      d1 = wp * (1.0f - r);
      d2 = wp;
      dh = r + ec;
      break;
    }
    case kCodeInvGauss: {
      const float inv = __builtin_amdgcn_rcpf(mu);
      d1 = wp * (mu - yy) * inv * inv;
      d2 = wp * inv;
      dh = fmaf(0.5f * yy * inv, inv, -inv);
      break;
    }
    case kCodeBernoulli:
      d1 = wp * (mu - yy);
      d2 = wp * mu * (1.0f - mu);
      dh = fmaf(yy, softplus(-ec), (1.0f - yy) * softplus(ec));
      break;
    default: {   // Gaussian
      const float r = mu - yy;
      d1 = wp * r;
      d2 = wp;
      dh = 0.5f * r * r;
      break;
    }
  }
  if constexpr (WANT_DEV) dev = miss ? 0.f : (HALF ? 1.f : 2.f) * w * dh;
}

// Mean of the linear predictor for a link code, with the fit's clamps.
__device__ __forceinline__ float inverse_link_code(int link, float eta, float lo, float hi) {
  if (link == kLinkIdentity) return eta;
  if (link == kLinkLogit) return 1.0f / (1.0f + expf(-fminf(fmaxf(eta, -hi), hi)));
  return expf(fminf(fmaxf(eta, lo), hi));
}

// Variance function nu(mu) of a family code (Supplementary Table 1).
__device__ __forceinline__ float variance_code(int code, float mu, float alpha) {
  switch (code) {
    case kCodePoisson: return mu;
    case kCodeNegBin: return mu * (1.0f + mu / alpha);
    case kCodeGamma: return mu * mu;
    case kCodeInvGauss: return mu * mu * mu;
    case kCodeBernoulli: return mu * (1.0f - mu);
    default: return 1.0f;
  }
}

// The unit deviance D(y, mu) of a family code in its plain form (float32,
// accurate libm functions; for monitoring outside the fit).
__device__ __forceinline__ float unit_deviance_code(int code, float y, float mu, float alpha) {
  const float ylog = y > 0.f ? y * logf(y / mu) : 0.f;
  switch (code) {
    case kCodePoisson: return 2.f * (ylog - (y - mu));
    case kCodeNegBin: return 2.f * (ylog - (y + alpha) * logf((y + alpha) / (mu + alpha)));
    case kCodeGamma: return 2.f * ((y - mu) / mu - logf(y / mu));
    case kCodeInvGauss: return (y - mu) * (y - mu) / (y * mu * mu);
    case kCodeBernoulli: {
      const float ylog1 = y < 1.f ? (1.f - y) * logf((1.f - y) / (1.f - mu)) : 0.f;
      return 2.f * (ylog + ylog1);
    }
    default: return (y - mu) * (y - mu);
  }
}

// eta: linear predictor, y: response, w: weight (1 when there are none).
// dev (WANT_DEV): the mu part of the unit deviance times w -- the full unit
// deviance for the Gaussian family, 2 w [D/2 - c(y)] for Poisson and NB
// (HALF: divided by dev_unit<FAM>(), which the caller applies to its sum:
// 2 for Poisson, 2 ln 2 for NB, whose entries are then in base-2 units).
template <int FAM>
__host__ __device__ constexpr double dev_unit() {
  return FAM == kGaussian ? 1.0 : (FAM == kNegBin ? 2.0 * 0.6931471805599453 : 2.0);
}

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
    const float t = ec * 1.4426950408889634f;                      // eta log2(e)
    const float mu = __builtin_amdgcn_exp2f(t);
    if constexpr (FAM == kPoisson) {
      const float wp = w * c.phi_inv;
      d1 = wp * (mu - y);
      d2 = wp * mu;
      if constexpr (WANT_DEV) {
        dev = (HALF ? 1.f : 2.f) * w * fmaf(-y, ec, mu);
      }
    } else {
      const float inv = __builtin_amdgcn_rcpf(c.a + mu);
      const float wa = w * c.a_phi * inv;
      d2 = wa * mu;
      d1 = fmaf(-wa, y, d2);
      if constexpr (WANT_DEV) {
        const float l2 = __builtin_amdgcn_logf(fmaf(mu, c.inv_a, 1.0f));   // log2(1 + mu/a)
        const float dh2 = fmaf(y + c.a, l2, -y * t);   // the mu part / ln 2
        if constexpr (HALF) dev = w * dh2;
        else dev = (2.0f * 0.6931471805599453f) * w * dh2;
      }
    }
  }
}

// family_entry<FAM, WANT_DEV, true> with the entry's deviance added to `acc`
// instead of returned: for NB without weights the two terms of the mu part go
// into the sum by two fused multiply-adds, one operation less per entry.
template <int FAM, bool WANT_DEV, bool HAS_W>
__device__ __forceinline__ void family_entry_acc(float eta, float y, float w, const FamilyConst& c,
                                                 float& d1, float& d2, float& acc) {
  if constexpr (FAM == kNegBin && WANT_DEV && !HAS_W) {
    const float ec = __builtin_amdgcn_fmed3f(eta, c.lo, c.hi);
    const float t = ec * 1.4426950408889634f;
    const float mu = __builtin_amdgcn_exp2f(t);
    const float inv = __builtin_amdgcn_rcpf(c.a + mu);
    const float wa = c.a_phi * inv;
    d2 = wa * mu;
    d1 = fmaf(-wa, y, d2);
    const float l2 = __builtin_amdgcn_logf(fmaf(mu, c.inv_a, 1.0f));
    acc = fmaf(-y, t, fmaf(y + c.a, l2, acc));
  } else {
    float dv = 0.f;
    family_entry<FAM, WANT_DEV, true>(eta, y, w, c, d1, d2, dv);
    if constexpr (WANT_DEV) acc += dv;
  }
}

}  // namespace gmf
