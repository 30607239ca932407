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
// A workgroup takes 16 rows; thread t walks the columns j = t, t + 256, ... in
// the caller's original column order (a copy of the frozen column panel in that
// order), so the count loads of consecutive threads are consecutive and every
// column's panel row is read once per 16 rows.  Per-row sums are combined in a
// fixed order (butterfly within a wavefront, then the four wavefronts), so
// results are reproducible.
#include <hip/hip_runtime.h>

#include "family.hpp"
#include "gmf_kernels.hpp"

namespace gmf {

namespace {

constexpr int kTileRows = 16;   // rows per workgroup
constexpr int kThreads = 256;
constexpr int kMaxK = 64;       // p + q + d <= 64

template <bool Y_INT>
__device__ __forceinline__ float y_at(const void* Y, int64_t idx) {
  if constexpr (Y_INT) return (float)static_cast<const int*>(Y)[idx];
  else return static_cast<const float*>(Y)[idx];
}

// Sums of kTileRows per-thread values over the workgroup, in a fixed order:
// a butterfly inside each wavefront, then the four wavefront totals in order;
// the totals land in tot[] (LDS).
__device__ __forceinline__ void tile_sums(const float (&v)[kTileRows], double (*red)[kTileRows],
                                          double* tot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = 0; r < kTileRows; ++r) {
    double x = (double)v[r];
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[wave][r] = x;
  }
  __syncthreads();
  if (threadIdx.x < kTileRows) {
    const int r = threadIdx.x;
    tot[r] = ((red[0][r] + red[1][r]) + red[2][r]) + red[3][r];
  }
  __syncthreads();
}

// Stage the tile's panel rows (Prow, first `cols` values) into LDS.
__device__ __forceinline__ void stage_rows(const WarmArgs& a, int64_t r0, int nr, int cols,
                                           float (*sP)[kMaxK + 1]) {
  for (int idx = threadIdx.x; idx < kTileRows * cols; idx += kThreads) {
    const int r = idx / cols, k = idx % cols;
    sP[r][k] = (r < nr) ? a.Prow[(r0 + r) * a.KP + k] : 0.f;
  }
}

template <bool Y_INT, bool LOG_LINK>
__global__ __launch_bounds__(kThreads) void row_intercept_kernel(WarmArgs a) {
  __shared__ float sP[kTileRows][kMaxK + 1];
  __shared__ double red[4][kTileRows];
  const int64_t r0 = (int64_t)blockIdx.x * kTileRows;
  const int nr = (int)min<int64_t>(kTileRows, a.n - r0);
  stage_rows(a, r0, nr, a.p, sP);
  __syncthreads();
  float sy[kTileRows], s2[kTileRows];
  for (int r = 0; r < kTileRows; ++r) sy[r] = s2[r] = 0.f;
  for (int j = threadIdx.x; j < a.m; j += kThreads) {
    const float* pc = a.Pcol_orig + (int64_t)j * a.KP;
    float ex[kTileRows];
    for (int r = 0; r < kTileRows; ++r) ex[r] = 0.f;
    for (int k = 0; k < a.p; ++k) {
      const float b = pc[k];
      for (int r = 0; r < kTileRows; ++r) ex[r] = fmaf(sP[r][k], b, ex[r]);
    }
    for (int r = 0; r < kTileRows; ++r) {
      if (r < nr) {
        sy[r] += y_at<Y_INT>(a.Y, (r0 + r) * a.m + j);
        if constexpr (LOG_LINK) s2[r] += fast_exp(fminf(fmaxf(ex[r], a.f.eta_lo), a.f.eta_hi));
        else s2[r] += ex[r];
      }
    }
  }
  __shared__ double ty[kTileRows], t2[kTileRows];
  tile_sums(sy, red, ty);
  tile_sums(s2, red, t2);
  // index r * q + c: column c of Gamma for row r
  for (int t = threadIdx.x; t < kTileRows * a.q; t += kThreads) {
    const int r = t / a.q, c = t % a.q;
    if (r < nr) {
      float g = 0.f;
      if (c == 0) {
        const double yr = ty[r], xr = t2[r];
        if constexpr (LOG_LINK) g = (float)(log(yr + 0.5) - log(xr));
        else g = (float)((yr - xr) / (double)a.m);
      }
      a.Prow[(r0 + r) * a.KP + a.p + c] = g;
    }
  }
}

template <bool Y_INT, int FAM>
__global__ __launch_bounds__(kThreads) void row_select_kernel(WarmArgs a) {
  __shared__ float sP[kTileRows][kMaxK + 1];
  __shared__ double red[4][kTileRows];
  const int64_t r0 = (int64_t)blockIdx.x * kTileRows;
  const int nr = (int)min<int64_t>(kTileRows, a.n - r0);
  const int pq = a.p + a.q;
  const int kk = pq + a.d;
  // panel rows with the candidate scores in the U columns
  for (int idx = threadIdx.x; idx < kTileRows * kk; idx += kThreads) {
    const int r = idx / kk, k = idx % kk;
    float v = 0.f;
    if (r < nr) v = (k < pq) ? a.Prow[(r0 + r) * a.KP + k] : a.Ucand[(r0 + r) * a.d + (k - pq)];
    sP[r][k] = v;
  }
  __syncthreads();
  const FamilyConst fc = family_const(a.f);
  float dw[kTileRows], dz[kTileRows];
  for (int r = 0; r < kTileRows; ++r) dw[r] = dz[r] = 0.f;
  for (int j = threadIdx.x; j < a.m; j += kThreads) {
    const float* pc = a.Pcol_orig + (int64_t)j * a.KP;
    float base[kTileRows], lat[kTileRows];
    for (int r = 0; r < kTileRows; ++r) base[r] = lat[r] = 0.f;
    for (int k = 0; k < pq; ++k) {
      const float b = pc[k];
      for (int r = 0; r < kTileRows; ++r) base[r] = fmaf(sP[r][k], b, base[r]);
    }
    for (int k = pq; k < kk; ++k) {
      const float b = pc[k];
      for (int r = 0; r < kTileRows; ++r) lat[r] = fmaf(sP[r][k], b, lat[r]);
    }
    for (int r = 0; r < kTileRows; ++r) {
      if (r < nr) {
        const float y = y_at<Y_INT>(a.Y, (r0 + r) * a.m + j);
        float x1, x2, dv;
        family_entry<FAM, true>(base[r] + lat[r], y, 1.f, fc, x1, x2, dv);
        dw[r] += dv;
        family_entry<FAM, true>(base[r], y, 1.f, fc, x1, x2, dv);
        dz[r] += dv;
      }
    }
  }
  __shared__ double tw[kTileRows], tz[kTileRows];
  tile_sums(dw, red, tw);
  tile_sums(dz, red, tz);
  // index r * d + c: score c of row r
  for (int t = threadIdx.x; t < kTileRows * a.d; t += kThreads) {
    const int r = t / a.d, c = t % a.d;
    if (r < nr) {
      const double wr = tw[r], zr = tz[r];
      const bool warm = wr < zr;
      a.Prow[(r0 + r) * a.KP + pq + c] = warm ? sP[r][pq + c] : 0.f;
      if (c == 0) {
        if (a.dev_out) {
          a.dev_out[2 * (r0 + r)] = wr;
          a.dev_out[2 * (r0 + r) + 1] = zr;
        }
        if (!warm) atomicAdd(a.fallback, 1ULL);
      }
    }
  }
}

template <int FAM>
hipError_t select_fam(const WarmArgs& a, bool y_int, dim3 grid, hipStream_t s) {
  if (y_int) hipLaunchKernelGGL((row_select_kernel<true, FAM>), grid, dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL((row_select_kernel<false, FAM>), grid, dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_row_intercept(const WarmArgs& a, bool y_int, bool log_link, hipStream_t s) {
  if (a.n <= 0 || a.q <= 0) return hipSuccess;
  if (a.p + a.q + a.d > kMaxK) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((a.n + kTileRows - 1) / kTileRows));
  if (y_int) {
    if (log_link) hipLaunchKernelGGL((row_intercept_kernel<true, true>), grid, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((row_intercept_kernel<true, false>), grid, dim3(kThreads), 0, s, a);
  } else {
    if (log_link) hipLaunchKernelGGL((row_intercept_kernel<false, true>), grid, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((row_intercept_kernel<false, false>), grid, dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_row_select(const WarmArgs& a, int fam, bool y_int, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.p + a.q + a.d > kMaxK) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((a.n + kTileRows - 1) / kTileRows));
  switch (fam) {
    case kPoisson: return select_fam<kPoisson>(a, y_int, grid, s);
    case kNegBin: return select_fam<kNegBin>(a, y_int, grid, s);
    case kGaussian: return select_fam<kGaussian>(a, y_int, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gmf
