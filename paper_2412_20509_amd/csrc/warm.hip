// Starting values of the row projection (the warm-start pipeline).
//
//  * row_intercept_kernel: the row intercept gamma_i0 of a new row given the
//    frozen column side, from matching the row total: with U = 0 and the first
//    column of Z the intercept (z_j0 = 1),
//      log link:      sum_j exp(x_i' beta_j + gamma_i0) = sum_j y_ij + 1/2
//                     -> gamma_i0 = log(sum_j y_ij + 1/2) - log sum_j exp(x_i' beta_j),
//      identity link: sum_j (x_i' beta_j + gamma_i0)    = sum_j y_ij
//                     -> gamma_i0 = mean_j (y_ij - x_i' beta_j);
//    the other columns of Gamma start at 0.
//  * row_select_kernel: per row, the deviance sum_j D(y_ij, mu_ij) of the
//    candidate scores u_i (e.g. an encoder's output) and of u_i = 0, both with
//    the row's covariate and Gamma terms; the row starts from the candidate when
//    its deviance is lower, else from 0 (a fallback, counted).
// One wavefront per row; each lane walks the columns j = lane, lane + 64, ...
// in the caller's original column order (the frozen column panel is stored in
// the fit's permuted order and is addressed through the column tables); the
// per-lane sums are combined by a fixed butterfly, so results are
// reproducible.
#include <hip/hip_runtime.h>

#include "family.hpp"
#include "gmf_kernels.hpp"

namespace gmf {

namespace {

constexpr int kRowsPerWG = 4;   // one wavefront per row, 256 threads

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <bool Y_INT>
__device__ __forceinline__ float y_at(const void* Y, int64_t idx) {
  if constexpr (Y_INT) return (float)static_cast<const int*>(Y)[idx];
  else return static_cast<const float*>(Y)[idx];
}

template <bool Y_INT, bool LOG_LINK>
__global__ __launch_bounds__(256) void row_intercept_kernel(WarmArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * kRowsPerWG + (threadIdx.x >> 6);
  if (i >= a.n) return;
  float* prow = a.Prow + i * a.KP;
  double sy = 0.0, s2 = 0.0;
  for (int j = lane; j < a.m; j += 64) {
    const int jp = a.co[a.colblk[j]] + a.colloc[j];
    const float* pc = a.Pcol + (int64_t)jp * a.KP;
    float ex = 0.f;
    for (int k = 0; k < a.p; ++k) ex += prow[k] * pc[k];
    const float y = y_at<Y_INT>(a.Y, i * a.m + j);
    sy += (double)y;
    if constexpr (LOG_LINK) s2 += (double)fast_exp(fminf(fmaxf(ex, a.f.eta_lo), a.f.eta_hi));
    else s2 += (double)ex;
  }
  sy = wave_sum(sy);
  s2 = wave_sum(s2);
  if (lane < a.q) {
    float g = 0.f;
    if (lane == 0) {
      if constexpr (LOG_LINK) g = (float)(log(sy + 0.5) - log(s2));
      else g = (float)((sy - s2) / (double)a.m);
    }
    prow[a.p + lane] = g;
  }
}

template <bool Y_INT, int FAM>
__global__ __launch_bounds__(256) void row_select_kernel(WarmArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * kRowsPerWG + (threadIdx.x >> 6);
  if (i >= a.n) return;
  const FamilyConst fc = family_const(a.f);
  float* prow = a.Prow + i * a.KP;
  const float* uw = a.Ucand + i * a.d;
  const int pq = a.p + a.q;
  float dw = 0.f, dc = 0.f;
  for (int j = lane; j < a.m; j += 64) {
    const int jp = a.co[a.colblk[j]] + a.colloc[j];
    const float* pc = a.Pcol + (int64_t)jp * a.KP;
    float base = 0.f;
    for (int k = 0; k < pq; ++k) base += prow[k] * pc[k];
    float lat = 0.f;
    for (int k = 0; k < a.d; ++k) lat += uw[k] * pc[pq + k];
    const float y = y_at<Y_INT>(a.Y, i * a.m + j);
    float x1, x2, dv;
    family_entry<FAM, true>(base + lat, y, 1.f, fc, x1, x2, dv);
    dw += dv;
    family_entry<FAM, true>(base, y, 1.f, fc, x1, x2, dv);
    dc += dv;
  }
  const double sw = wave_sum((double)dw);
  const double sc = wave_sum((double)dc);
  const bool warm = sw < sc;
  if (a.dev_out && lane == 0) {
    a.dev_out[2 * i] = sw;
    a.dev_out[2 * i + 1] = sc;
  }
  if (lane < a.d) prow[pq + lane] = warm ? uw[lane] : 0.f;
  if (!warm && lane == 0) atomicAdd(a.fallback, 1ULL);
}

template <int FAM>
hipError_t select_fam(const WarmArgs& a, bool y_int, dim3 grid, hipStream_t s) {
  if (y_int) hipLaunchKernelGGL((row_select_kernel<true, FAM>), grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((row_select_kernel<false, FAM>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_row_intercept(const WarmArgs& a, bool y_int, bool log_link, hipStream_t s) {
  if (a.n <= 0 || a.q <= 0) return hipSuccess;
  const dim3 grid((unsigned)((a.n + kRowsPerWG - 1) / kRowsPerWG));
  if (y_int) {
    if (log_link) hipLaunchKernelGGL((row_intercept_kernel<true, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((row_intercept_kernel<true, false>), grid, dim3(256), 0, s, a);
  } else {
    if (log_link) hipLaunchKernelGGL((row_intercept_kernel<false, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((row_intercept_kernel<false, false>), grid, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_row_select(const WarmArgs& a, int fam, bool y_int, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((a.n + kRowsPerWG - 1) / kRowsPerWG));
  switch (fam) {
    case kPoisson: return select_fam<kPoisson>(a, y_int, grid, s);
    case kNegBin: return select_fam<kNegBin>(a, y_int, grid, s);
    case kGaussian: return select_fam<kGaussian>(a, y_int, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gmf
