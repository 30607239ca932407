// Matrix-core wrappers, bfloat16 conversions and the adaptive step shared by
// the step kernels (step.hip) and the projection kernel (project.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace gmf {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// D(16x16) += A(16x4) B(4x16), float32: lane (i = lane % 16, k = lane / 16)
// holds A[i][k] and B[k][i]; the result lane (j = lane % 16, g = lane / 16)
// holds rows 4g .. 4g+3 of column j.
__device__ __forceinline__ floatx4 mfma_f32(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// D(16x16) += A(16x32) B(32x16), bfloat16 operands, float32 accumulation: lane
// (i, g) holds A[i][8g .. 8g+7] and B[8g .. 8g+7][i].
__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 to_bf16(floatx8 x) { return __builtin_convertvector(x, bf16x8); }
// low part of a split: bf16(x - hi), where x - hi is exact in float32
__device__ __forceinline__ bf16x8 lo_bf16(floatx8 x, bf16x8 hi) {
  return to_bf16(x - __builtin_convertvector(hi, floatx8));
}
__device__ __forceinline__ __bf16 lo_bf16(float x, __bf16 hi) { return (__bf16)(x - (float)hi); }

// Split BF16 uses split operands in eta and the gradient sums D1 [Z,V],
// D1^T [X,U], and, with kSplitCurvature, also in the curvature sums
// D2 [Z^2,V^2], D2^T [X^2,U^2].  The curvature only scales the step (the
// diagonal of eq. 13-14); with single bfloat16 products there the steps run
// 5-10 % faster, but a 20-epoch Poisson fit (1000 x 500, d = 5) ends 8e-5
// from the float64 deviance instead of 1e-6, so the sums are split.
constexpr bool kSplitCurvature = true;

// EMA of the gradient and curvature (eq. 12) and the step
// theta -= stepsize * Gbar / (Hbar + damping) (eq. 13-14) for one parameter;
// returns false if the result is not finite.
// ema_apply takes the current theta, Gbar, Hbar as values (loaded ahead by
// the caller); ema_step loads them itself.
__device__ __forceinline__ bool ema_apply(float* th, double* gm, double* hm, float th0, double g0,
                                          double h0, double G, double H, double a1, double a2,
                                          double damping, double stepsize) {
  const double gbar = (1.0 - a1) * g0 + a1 * G;
  const double hbar = (1.0 - a2) * h0 + a2 * H;
  *gm = gbar;
  *hm = hbar;
  const float nv = (float)((double)th0 - stepsize * gbar / (hbar + damping));
  *th = nv;
  return isfinite(nv);
}
__device__ __forceinline__ bool ema_step(float* th, double* gm, double* hm, double G, double H,
                                         double a1, double a2, double damping, double stepsize) {
  return ema_apply(th, gm, hm, *th, *gm, *hm, G, H, a1, a2, damping, stepsize);
}

}  // namespace gmf
