// Set-up, copy-out and monitoring kernels of libgmf (gfx950).
//
//  * permute_y_kernel: copies Y (and W) into the block-major permuted layout,
//    so that every block I_r x J_s is one dense rectangle (row stride padded to
//    a multiple of 4 floats).  Counts become float32 (exact below 2^24).
//  * pack/unpack panel kernels: [X|Gamma|U] and [B|Z|V] panels in permuted
//    order <-> caller arrays in original order.
//  * deviance_kernel: full deviance sum_ij w D(y, mu) of the current iterate
//    (definition after eq. 2; Supplementary Table 1; Appendix B for NB), eta on
//    the float32 matrix cores, per-entry deviance (its mu part) in float32,
//    float64 accumulation in a fixed order (per-tile partials, then one
//    ordered sum).
//  * count_sum_kernel: per deviance tile, sum w c(y) of the count-only part
//    of the deviance in float64 (constant during a fit).
//  * row_deviance_kernel: the deviance of every row, sum_j w D(y, mu), in the
//    caller's row order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "family.hpp"
#include "gmf_kernels.hpp"
#include "mfma.hpp"

namespace gmf {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ permute Y ----
struct PermuteTables {
  const int* row_block;        // original row i -> block r
  const int* row_local;        // original row i -> row inside the block
  const int* col_block;        // original col j -> block s
  const int* col_local;        // original col j -> col inside the block
  const int64_t* blk_row_base; // r -> offset of the first element of row block r
  const int* blk_nrows;        // r -> |I_r|
  const int64_t* blk_col_off;  // s -> padded column offset of J_s
  const int* blk_ld;           // s -> padded width of J_s
};

// Validation of y per family code (check = code + 1; 0 = none): counts (Poisson,
// NB) integer-valued >= 0, Gamma and inverse Gaussian > 0, Bernoulli 0 or 1,
// Gaussian finite.  With allow_missing a negative int32 or a NaN float32 is a
// missing entry, stored as NaN.
__device__ __forceinline__ bool valid_response(int check, float y) {
  switch (check - 1) {
    case kCodePoisson:
    case kCodeNegBin: return y >= 0.f && y == floorf(y);
    case kCodeGamma:
    case kCodeInvGauss: return y > 0.f;
    case kCodeBernoulli: return y == 0.f || y == 1.f;
    default: return true;
  }
}

__global__ void permute_y_kernel(const void* Y, int y_is_int, const float* W,
                                 int64_t n, int64_t m, PermuteTables t,
                                 float* Yb, float* Wb, int* err_flag, int allow_missing,
                                 int check) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int64_t i = idx / m;
  const int64_t j = idx % m;
  float y;
  if (y_is_int) {
    const int v = static_cast<const int*>(Y)[idx];
    if (v < 0 && allow_missing) {
      y = __builtin_nanf("");
    } else {
      if (v < 0 || v >= (1 << 24)) atomicOr(err_flag, 2);
      y = (float)v;
    }
  } else {
    y = static_cast<const float*>(Y)[idx];
    if (!(y == y) && allow_missing) {
      y = __builtin_nanf("");
    } else if (!isfinite(y)) {
      atomicOr(err_flag, 2);
    }
  }
  if (y == y && !valid_response(check, y)) atomicOr(err_flag, 2);
  const int r = t.row_block[i];
  const int s = t.col_block[j];
  const int64_t dst = t.blk_row_base[r] + (int64_t)t.blk_nrows[r] * t.blk_col_off[s] +
                      (int64_t)t.row_local[i] * t.blk_ld[s] + t.col_local[j];
  Yb[dst] = y;
  if (W) {
    const float w = W[idx];
    if (!(w > 0.f) || !isfinite(w)) atomicOr(err_flag, 2);
    Wb[dst] = w;
  }
}

hipError_t launch_permute_y(const void* Y, int y_is_int, const float* W, int64_t n,
                            int64_t m, const int* row_block, const int* row_local,
                            const int* col_block, const int* col_local,
                            const int64_t* blk_row_base, const int* blk_nrows,
                            const int64_t* blk_col_off, const int* blk_ld, float* Yb,
                            float* Wb, int* err_flag, hipStream_t s, int allow_missing,
                            int check) {
  PermuteTables t{row_block, row_local, col_block, col_local,
                  blk_row_base, blk_nrows, blk_col_off, blk_ld};
  const int64_t tot = n * m;
  const int64_t grid = (tot + 255) / 256;
  hipLaunchKernelGGL(permute_y_kernel, dim3((unsigned)grid), dim3(256), 0, s, Y,
                     y_is_int, W, n, m, t, Yb, Wb, err_flag, allow_missing, check);
  return hipGetLastError();
}

__global__ void iota_kernel(int* p, int64_t count) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) p[idx] = (int)idx;
}
hipError_t launch_iota(int* p, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

// ------------------------------------------------------- 16-bit counts ----
__global__ void compact_counts_kernel(const float* Yb, int64_t count, uint16_t* Yc, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float y = Yb[i];
  const bool ok = y >= 0.f && y <= 65535.f && y == floorf(y);   // false for NaN
  Yc[i] = ok ? (uint16_t)y : (uint16_t)0;
  if (!ok) atomicOr(flag, 1);
}
hipError_t launch_compact_counts(const float* Yb, int64_t count, uint16_t* Yc, int* flag,
                                 hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(compact_counts_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                     Yb, count, Yc, flag);
  return hipGetLastError();
}

// --------------------------------------------------------- panels ---------
__global__ void pack_panel_kernel(const float* M0, int c0, const float* M1, int c1,
                                  const float* M2, int c2, const int* perm,
                                  int64_t rows, int KP, float* P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * KP) return;
  const int64_t ip = idx / KP;
  const int c = (int)(idx % KP);
  const int64_t io = perm[ip];
  float v = 0.f;
  if (c < c0) v = M0[io * c0 + c];
  else if (c < c0 + c1) v = M1[io * c1 + (c - c0)];
  else if (c < c0 + c1 + c2) v = M2[io * c2 + (c - c0 - c1)];
  P[idx] = v;
}

hipError_t launch_pack_panel(const float* M0, int c0, const float* M1, int c1,
                             const float* M2, int c2, const int* perm, int64_t rows,
                             int KP, float* P, hipStream_t s) {
  const int64_t tot = rows * KP;
  hipLaunchKernelGGL(pack_panel_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256),
                     0, s, M0, c0, M1, c1, M2, c2, perm, rows, KP, P);
  return hipGetLastError();
}

__global__ void unpack_panel_kernel(const float* P, int KP, const int* perm,
                                    int64_t rows, int col0, int ncols, float* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * ncols) return;
  const int64_t ip = idx / ncols;
  const int c = (int)(idx % ncols);
  out[(int64_t)perm[ip] * ncols + c] = P[ip * KP + col0 + c];
}

hipError_t launch_unpack_panel(const float* P, int KP, const int* perm, int64_t rows,
                               int col0, int ncols, float* out, hipStream_t s) {
  if (ncols <= 0 || rows <= 0 || !out) return hipSuccess;
  const int64_t tot = rows * ncols;
  hipLaunchKernelGGL(unpack_panel_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256),
                     0, s, P, KP, perm, rows, col0, ncols, out);
  return hipGetLastError();
}

__global__ void unpack_moments_kernel(const double* M, int K, const int* perm,
                                      int64_t rows, double* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * K) return;
  const int64_t ip = idx / K;
  const int c = (int)(idx % K);
  out[(int64_t)perm[ip] * K + c] = M[idx];
}

hipError_t launch_unpack_moments(const double* M, int K, const int* perm, int64_t rows,
                                 double* out, hipStream_t s) {
  if (K <= 0 || rows <= 0 || !out) return hipSuccess;
  const int64_t tot = rows * K;
  hipLaunchKernelGGL(unpack_moments_kernel, dim3((unsigned)((tot + 255) / 256)),
                     dim3(256), 0, s, M, K, perm, rows, out);
  return hipGetLastError();
}

__global__ void fill_f64_kernel(double* p, int64_t count, double v) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) p[idx] = v;
}
__global__ void fill_i32_kernel(int* p, int64_t count, int v) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) p[idx] = v;
}
hipError_t launch_fill_f64(double* p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256),
                     0, s, p, count, v);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int* p, int64_t count, int v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256),
                     0, s, p, count, v);
  return hipGetLastError();
}

// Sum of squares of columns [col0, col0+ncols) of a panel: per-block partials.
__global__ void sumsq_kernel(const float* P, int KP, int64_t rows, int col0, int ncols,
                             double* partial) {
  __shared__ double red[256];
  double s = 0.0;
  const int64_t tot = rows * ncols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / ncols;
    const int c = (int)(idx % ncols);
    const double x = (double)P[r * KP + col0 + c];
    s += x * x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

hipError_t launch_sumsq(const float* P, int KP, int64_t rows, int col0, int ncols,
                        double* partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(nblocks), dim3(256), 0, s, P, KP, rows, col0,
                     ncols, partial);
  return hipGetLastError();
}

// Squared Frobenius norms of B, Gamma, U, V (eq. 6 penalty) in one pass:
// partial[k * gridDim.x + block] for k = 0..3 (fixed assignment and tree).
__global__ void norms_kernel(const float* Prow, const float* Pcol, int KP, int64_t n, int64_t m,
                             int p, int q, int d, double* partial) {
  __shared__ double red[4][256];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t idx = start; idx < n * (q + d); idx += stride) {   // Gamma, U
    const int64_t r = idx / (q + d);
    const int c = (int)(idx % (q + d));
    const double x = (double)Prow[r * KP + p + c];
    acc[c < q ? 1 : 2] += x * x;
  }
  for (int64_t idx = start; idx < m * (p + d); idx += stride) {   // B, V
    const int64_t r = idx / (p + d);
    const int c = (int)(idx % (p + d));
    const double x = (double)Pcol[r * KP + (c < p ? c : c + q)];
    acc[c < p ? 0 : 3] += x * x;
  }
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 4) partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_norms(const float* Prow, const float* Pcol, int KP, int64_t n, int64_t m,
                        int p, int q, int d, double* partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(norms_kernel, dim3(nblocks), dim3(256), 0, s, Prow, Pcol, KP, n, m, p, q, d,
                     partial);
  return hipGetLastError();
}

// out[0] = sum of dev[0..ndev), out[1+k] = sum of norm[k*nnorm .. (k+1)*nnorm).
__global__ void finalize_kernel(const double* dev, int ndev, const double* norm, int nnorm,
                                const int* flag, double* out) {
  __shared__ double red[5][256];
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  // unrolled so that several loads are in flight; the additions keep their order
#pragma unroll 8
  for (int i = threadIdx.x; i < ndev; i += 256) acc[0] += dev[i];
  if (norm)
    for (int k = 0; k < 4; ++k)
#pragma unroll 8
      for (int i = threadIdx.x; i < nnorm; i += 256) acc[1 + k] += norm[k * nnorm + i];
  for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 5) out[threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == 5) out[5] = flag ? (double)*flag : 0.0;
}

hipError_t launch_finalize(const double* dev, int ndev, const double* norm, int nnorm,
                           const int* flag, double* out, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, dev, ndev, norm, nnorm, flag, out);
  return hipGetLastError();
}

// Ordered sum of `count` doubles by one workgroup (fixed assignment and tree).
__global__ void sum_partials_kernel(const double* partial, int count, double* out) {
  __shared__ double red[256];
  double s = 0.0;
#pragma unroll 8
  for (int i = threadIdx.x; i < count; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_sum_partials(const double* partial, int count, double* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partial, count, out);
  return hipGetLastError();
}

// --------------------------------------------------------------- deviance --
// LDS of a deviance workgroup: the group's row panel, float32 (float32
// products) or as high and low bfloat16 parts (split products: panel
// strides 16, 32 and 64).
template <int KP>
struct DevLds {
  static constexpr bool SPL = KP == 16 || KP % 32 == 0;
  alignas(16) float sP[SPL ? 1 : kRowGroup][SPL ? 4 : KP + 4];
  alignas(16) __bf16 sPh[SPL ? kRowGroup : 1][SPL ? KP + 8 : 8];
  alignas(16) __bf16 sPl[SPL ? kRowGroup : 1][SPL ? KP + 8 : 8];
  double sDev[kTileWaves];
};

// One workgroup per (block, range of up to 256 rows, strip of 128 columns);
// each wavefront owns 32 columns and walks the rows in groups of 32 with the
// next group's counts and panel rows prefetched.  Same 32x32 pieces and MFMA
// operand layout as the step kernel.  eta on the matrix cores: at panel
// strides 16, 32 and 64 as split bfloat16 products (each operand x = hi +
// lo, both bfloat16; hi hi + hi lo + lo hi, float32 accumulation, the
// products of the split-BF16 step: 16x16x16 at stride 16, 16x16x32 above),
// at stride 48 as float32 products.  Rows
// past the range and columns past the block read the last valid ones
// (clamped addresses) and are masked out of the sum; groups with none of them
// skip the mask.
template <int FAM, int KP, bool HAS_W, bool CY>
__device__ __forceinline__ void deviance_tile(const DevArgs& a, int tile, DevLds<KP>& L) {
  constexpr bool SPL = DevLds<KP>::SPL;
  constexpr bool K16 = KP == 16;   // 16x16x16 bfloat16 products
  using YRaw = typename std::conditional<CY, uint2, float4>::type;   // 4 counts as stored
  const FamilyConst fc = family_const(a.f);
  const int blk = a.tile_block[tile];
  const int local = tile - a.tile_first[blk];
  const int n_b = a.blk_nb[blk], m_b = a.blk_mb[blk];
  const int ldy = a.blk_ldy[blk];
  const int n_ct = a.blk_nct[blk];
  const int rpw = a.blk_rpw[blk];
  const float* Y = a.Y + a.blk_yoff[blk];
  const uint16_t* Yc = CY ? a.Yc + a.blk_yoff[blk] : nullptr;
  const float* W = HAS_W ? a.W + a.blk_yoff[blk] : nullptr;
  const float* Prow = a.Prow + (int64_t)a.blk_row0[blk] * KP;
  const float* Pcol = a.Pcol + (int64_t)a.blk_col0[blk] * KP;
  const int ct = local % n_ct, rr = local / n_ct;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int row0 = rr * rpw, row_end = min(n_b, row0 + rpw);
  const int colw = ct * kTileCols + wave * kWaveCols;
  const int colw_u = __builtin_amdgcn_readfirstlane(colw);   // the same in every lane

  constexpr int PF = (kRowGroup * (KP / 4) + kTileThreads - 1) / kTileThreads;
  auto load_p = [&](int rg, float4 (&pf)[PF]) {
    for (int u = 0; u < PF; ++u) {
      const int idx = tid + u * kTileThreads;
      pf[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (idx < kRowGroup * (KP / 4)) {
        const int r = idx / (KP / 4), c4 = idx % (KP / 4);
        if (rg + r < row_end) pf[u] = reinterpret_cast<const float4*>(Prow + (int64_t)(rg + r) * KP)[c4];
      }
    }
  };
  auto y_offset = [&](int row, int C) {
    return (int64_t)min(row, row_end - 1) * ldy + min(colw + 16 * C + 4 * g, ldy - 4);
  };
  auto load_y = [&](int rg, YRaw (&y)[2][2]) {
    for (int R = 0; R < 2; ++R)
      for (int C = 0; C < 2; ++C) {
        const int64_t off = y_offset(rg + 2 * l16 + R, C);
        if constexpr (CY) y[R][C] = *reinterpret_cast<const uint2*>(Yc + off);
        else y[R][C] = *reinterpret_cast<const float4*>(Y + off);
      }
  };
  float4 pnext[PF];
  YRaw ynext[2][2], yalt[2][2];
  load_p(row0, pnext);
  load_y(row0, ynext);
  // column operands, fixed over the tile: float32 entries 4kk + g, or the
  // bfloat16 parts of entries 32kk + 8g .. +7, of column colw + 16c + l16
  float pa[2][SPL ? 1 : KP / 4];
  bf16x8 pah[2][(SPL && !K16) ? KP / 32 : 1], pal[2][(SPL && !K16) ? KP / 32 : 1];
  bf16x4 kah[2], kal[2];   // stride 16: entries 4g .. 4g+3
  for (int c = 0; c < 2; ++c) {
    const int col = colw + 16 * c + l16;
    if constexpr (K16) {
      floatx4 x = {0.f, 0.f, 0.f, 0.f};
      if (col < m_b) {
        const float4 u = *reinterpret_cast<const float4*>(Pcol + (int64_t)col * KP + 4 * g);
        x = floatx4{u.x, u.y, u.z, u.w};
      }
      kah[c] = __builtin_convertvector(x, bf16x4);
      kal[c] = __builtin_convertvector(x - __builtin_convertvector(kah[c], floatx4), bf16x4);
    } else if constexpr (SPL) {
      for (int kk = 0; kk < KP / 32; ++kk) {
        floatx8 x = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (col < m_b) {
          const float4 u = *reinterpret_cast<const float4*>(Pcol + (int64_t)col * KP + 32 * kk + 8 * g);
          const float4 w = *reinterpret_cast<const float4*>(Pcol + (int64_t)col * KP + 32 * kk + 8 * g + 4);
          x = floatx8{u.x, u.y, u.z, u.w, w.x, w.y, w.z, w.w};
        }
        pah[c][kk] = to_bf16(x);
        pal[c][kk] = lo_bf16(x, pah[c][kk]);
      }
    } else {
      for (int kk = 0; kk < KP / 4; ++kk)
        pa[c][kk] = (col < m_b) ? Pcol[(int64_t)col * KP + 4 * kk + g] : 0.f;
    }
  }
  double acc = 0.0;
  // one 32-row group; the count registers alternate between groups
  auto group = [&](const int rg, const YRaw (&ycur)[2][2], YRaw (&ynxt)[2][2]) {
    __syncthreads();
    for (int u = 0; u < PF; ++u) {
      const int idx = tid + u * kTileThreads;
      if (idx < kRowGroup * (KP / 4)) {
        const int r = idx / (KP / 4), c0 = 4 * (idx % (KP / 4));
        if constexpr (SPL) {
          const floatx4 x = {pnext[u].x, pnext[u].y, pnext[u].z, pnext[u].w};
          const bf16x4 h = __builtin_convertvector(x, bf16x4);
          const bf16x4 l = __builtin_convertvector(x - __builtin_convertvector(h, floatx4), bf16x4);
          *reinterpret_cast<bf16x4*>(&L.sPh[r][c0]) = h;
          *reinterpret_cast<bf16x4*>(&L.sPl[r][c0]) = l;
        } else {
          *reinterpret_cast<float4*>(&L.sP[r][c0]) = pnext[u];
        }
      }
    }
    if (rg + kRowGroup < row_end) {
      load_p(rg + kRowGroup, pnext);
      load_y(rg + kRowGroup, ynxt);
    }
    __syncthreads();
    const bool full = rg + kRowGroup <= row_end && colw_u + kWaveCols <= m_b;
    float grp = 0.f;
    for (int R = 0; R < 2; ++R) {
      const int lrow = 2 * l16 + R;
      const int row = rg + lrow;
      for (int C = 0; C < 2; ++C) {
        floatx4 e = {0.f, 0.f, 0.f, 0.f};
        if constexpr (K16) {   // the small products first
          const bf16x4 bh = *reinterpret_cast<const bf16x4*>(&L.sPh[lrow][4 * g]);
          const bf16x4 bl = *reinterpret_cast<const bf16x4*>(&L.sPl[lrow][4 * g]);
          e = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(kal[C], bh, e, 0, 0, 0);
          e = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(kah[C], bl, e, 0, 0, 0);
          e = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(kah[C], bh, e, 0, 0, 0);
        } else if constexpr (SPL) {
          for (int kk = 0; kk < KP / 32; ++kk) {   // the small products first
            const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&L.sPh[lrow][32 * kk + 8 * g]);
            const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&L.sPl[lrow][32 * kk + 8 * g]);
            e = mfma_bf16(pal[C][kk], bh, e);
            e = mfma_bf16(pah[C][kk], bl, e);
            e = mfma_bf16(pah[C][kk], bh, e);
          }
        } else {
          for (int kk = 0; kk < KP / 4; ++kk)
            e = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[C][kk], L.sP[lrow][4 * kk + g], e, 0, 0, 0);
        }
        const int colb = colw + 16 * C + 4 * g;
        float4 w4 = make_float4(1.f, 1.f, 1.f, 1.f);   // a literal 1 without weights
        if constexpr (HAS_W) w4 = *reinterpret_cast<const float4*>(W + y_offset(row, C));
        const float4 y4 = counts_f4(ycur[R][C]);
        const float ys[4] = {y4.x, y4.y, y4.z, y4.w};
        const float ws[4] = {w4.x, w4.y, w4.z, w4.w};
        // entries in the units of the HALF epilogues (the tile scales its sum)
        auto entries = [&](auto masked) {
          for (int v = 0; v < 4; ++v) {
            float x1, x2, dv = 0.f;
            if constexpr (FAM == kGeneric) {
              const float av = column_alpha(fc, a.blk_col0[blk] + min(colb + v, m_b - 1));
              family_entry_generic<true, true>(e[v], ys[v], ws[v], av, fc, x1, x2, dv);
            } else if constexpr (!decltype(masked)::value) {
              family_entry_acc<FAM, true, HAS_W>(e[v], ys[v], ws[v], fc, x1, x2, grp);
              continue;
            } else {
              family_entry<FAM, true, true>(e[v], ys[v], ws[v], fc, x1, x2, dv);
            }
            if constexpr (decltype(masked)::value) grp += (row < row_end && colb + v < m_b) ? dv : 0.f;
            else grp += dv;
          }
        };
        if (full) entries(std::false_type{});
        else entries(std::true_type{});
      }
    }
    acc += (double)grp;
  };
  for (int rg = row0; rg < row_end; rg += 2 * kRowGroup) {
    group(rg, ynext, yalt);
    if (rg + kRowGroup >= row_end) break;
    group(rg + kRowGroup, yalt, ynext);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) L.sDev[wave] = acc;
  __syncthreads();
  if (tid == 0) a.partial[tile] = dev_unit<FAM>() * (((L.sDev[0] + L.sDev[1]) + L.sDev[2]) + L.sDev[3]);
}

// One workgroup per tile, or (grid_cap) fewer workgroups walking the tiles:
// a capped grid leaves compute units to work running beside it.
template <int FAM, int KP, bool HAS_W, bool CY>
__global__ __launch_bounds__(kTileThreads) void deviance_kernel(DevArgs a) {
  __shared__ DevLds<KP> L;
  for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    // the strips of a row range on one XCD (with a grid of a multiple of 8)
    deviance_tile<FAM, KP, HAS_W, CY>(a, xcd_tile(tile, a.n_tiles), L);
    __syncthreads();   // the LDS is reused by the next tile
  }
}

template <int FAM, int KP, bool HAS_W>
static void launch_dev_y(const DevArgs& a, dim3 grid, dim3 block, hipStream_t s) {
  if constexpr (FAM == kPoisson || FAM == kNegBin)
    if (a.Yc) {
      hipLaunchKernelGGL((deviance_kernel<FAM, KP, HAS_W, true>), grid, block, 0, s, a);
      return;
    }
  hipLaunchKernelGGL((deviance_kernel<FAM, KP, HAS_W, false>), grid, block, 0, s, a);
}

template <int FAM, int KP>
static void launch_dev_w(const DevArgs& a, dim3 grid, dim3 block, hipStream_t s) {
  if (a.W) launch_dev_y<FAM, KP, true>(a, grid, block, s);
  else launch_dev_y<FAM, KP, false>(a, grid, block, s);
}

template <int FAM>
static hipError_t launch_dev_kp(int KP, const DevArgs& a, hipStream_t s) {
  if (a.n_tiles <= 0) return hipSuccess;
  const dim3 grid(a.grid_cap > 0 ? std::min(a.n_tiles, a.grid_cap) : a.n_tiles), block(kTileThreads);
  switch (KP) {
    case 16: launch_dev_w<FAM, 16>(a, grid, block, s); break;
    case 32: launch_dev_w<FAM, 32>(a, grid, block, s); break;
    case 48: launch_dev_w<FAM, 48>(a, grid, block, s); break;
    case 64: launch_dev_w<FAM, 64>(a, grid, block, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------ count-only part --
// c(y) for the integer counts below kTileThreads comes from a table formed by
// the workgroup (one float64 evaluation per thread, the same function, so the
// values are identical); other counts are evaluated directly.
template <int FAM>
__global__ __launch_bounds__(kTileThreads) void count_sum_kernel(DevArgs a) {
  __shared__ double red[kTileThreads];
  __shared__ double ctab[kTileThreads];
  const int tile = blockIdx.x;
  const int blk = a.tile_block[tile];
  const int local = tile - a.tile_first[blk];
  const int n_b = a.blk_nb[blk], m_b = a.blk_mb[blk];
  const int ldy = a.blk_ldy[blk];
  const int n_ct = a.blk_nct[blk];
  const int rpw = a.blk_rpw[blk];
  const float* Y = a.Y + a.blk_yoff[blk];
  const float* W = a.W ? a.W + a.blk_yoff[blk] : nullptr;
  const int ct = local % n_ct, rr = local / n_ct;
  const int row0 = rr * rpw, row_end = min(n_b, row0 + rpw);
  const int col0 = ct * kTileCols, col_end = min(m_b, col0 + kTileCols);
  const double alpha = a.f.est ? a.f.est[1] : (double)a.f.nb_alpha;
  if constexpr (FAM != kGeneric) ctab[threadIdx.x] = count_part<FAM>((double)threadIdx.x, alpha);
  __syncthreads();
  double acc = 0.0;
  // thread t: column col0 + t % 128 of rows row0 + t / 128, row0 + t / 128 + 2, ...
  const int c = col0 + (int)(threadIdx.x % kTileCols);
  if (c < col_end)
    for (int r = row0 + (int)(threadIdx.x / kTileCols); r < row_end; r += kTileThreads / kTileCols) {
      const int64_t idx = (int64_t)r * ldy + c;
      const double w = W ? (double)W[idx] : 1.0;
      const float y = Y[idx];
      double cy;
      if constexpr (FAM == kGeneric) {
        const double ac = a.f.alpha_col ? (double)a.f.alpha_col[a.blk_col0[blk] + c] : alpha;
        cy = count_part_generic(a.f.code, (double)y, ac);
      } else {
        const int yi = (int)y;
        cy = (yi >= 0 && yi < kTileThreads && (float)yi == y) ? ctab[yi]
                                                              : count_part<FAM>((double)y, alpha);
      }
      acc += w * cy;
    }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kTileThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[tile] = red[0];
}

hipError_t launch_count_sum(int fam, const DevArgs& a, hipStream_t s) {
  if (a.n_tiles <= 0) return hipSuccess;
  switch (fam) {
    case kPoisson:
      hipLaunchKernelGGL((count_sum_kernel<kPoisson>), dim3(a.n_tiles), dim3(kTileThreads), 0, s, a);
      break;
    case kNegBin:
      hipLaunchKernelGGL((count_sum_kernel<kNegBin>), dim3(a.n_tiles), dim3(kTileThreads), 0, s, a);
      break;
    case kGeneric:
      hipLaunchKernelGGL((count_sum_kernel<kGeneric>), dim3(a.n_tiles), dim3(kTileThreads), 0, s, a);
      break;
    default:
      return hipSuccess;   // Gaussian: no count-only part
  }
  return hipGetLastError();
}

// ---------------------------------------------------------- per-row deviance --
// One workgroup per 16 rows (caller's order): the rows' panel entries in LDS;
// thread t walks the columns j = t, t + 256, ... of every column block, loads
// the column's panel row once for the 16 rows, forms eta in float32, the mu part
// of the unit deviance in float32 (as the full deviance) and adds the count-only
// part c(y) in float64 (a per-workgroup table below 256); the 16 row sums are
// float64, combined in a fixed order.
constexpr int kRowDevRows = 16;

template <int FAM, int KP, bool HAS_W>
__global__ __launch_bounds__(kTileThreads) void row_deviance_kernel(RowDevArgs a) {
  __shared__ float sP[kRowDevRows][KP + 1];
  __shared__ double ctab[kTileThreads];
  __shared__ double red[kTileWaves][kRowDevRows];
  __shared__ int64_t rbase[kRowDevRows];
  __shared__ int rnb[kRowDevRows], rli[kRowDevRows];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * kRowDevRows;
  const int nr = (int)min<int64_t>(kRowDevRows, a.n - i0);
  const double alpha = a.f.est ? a.f.est[1] : (double)a.f.nb_alpha;
  if constexpr (FAM != kGeneric) ctab[tid] = count_part<FAM>((double)tid, alpha);
  if (tid < kRowDevRows) {
    int rb = 0, li = 0;
    if (tid < nr) { rb = a.rowblk[i0 + tid]; li = a.rowloc[i0 + tid]; }
    rbase[tid] = a.rowbase[rb];
    rnb[tid] = a.nrows[rb];
    rli[tid] = li;
  }
  for (int idx = tid; idx < kRowDevRows * KP; idx += kTileThreads) {
    const int r = idx / KP, k = idx % KP;
    float v = 0.f;
    if (r < nr) {
      const int pr = a.ro[a.rowblk[i0 + r]] + a.rowloc[i0 + r];
      v = a.Prow[(int64_t)pr * KP + k];
    }
    sP[r][k] = v;
  }
  __syncthreads();
  const FamilyConst fc = family_const(a.f);
  double acc[kRowDevRows];
  for (int r = 0; r < kRowDevRows; ++r) acc[r] = 0.0;
  for (int s = 0; s < a.S; ++s) {
    const int mb = a.mcols[s], c0 = a.co[s], ld = a.ld[s];
    const int64_t coff = a.coloff[s];
    for (int j = tid; j < mb; j += kTileThreads) {
      float pc[KP];
      const float4* src = reinterpret_cast<const float4*>(a.Pcol + (int64_t)(c0 + j) * KP);
      for (int q = 0; q < KP / 4; ++q) {
        const float4 x = src[q];
        pc[4 * q] = x.x; pc[4 * q + 1] = x.y; pc[4 * q + 2] = x.z; pc[4 * q + 3] = x.w;
      }
      for (int r = 0; r < kRowDevRows; ++r) {
        if (r >= nr) break;
        float eta = 0.f;
        for (int k = 0; k < KP; ++k) eta = fmaf(sP[r][k], pc[k], eta);
        const int64_t at = rbase[r] + (int64_t)rnb[r] * coff + (int64_t)rli[r] * ld + j;
        const float y = a.Yb[at];
        const float w = HAS_W ? a.Wb[at] : 1.f;
        float d1, d2, dv;
        double cy;
        if constexpr (FAM == kGeneric) {
          const float av = column_alpha(fc, c0 + j);
          family_entry_generic<true>(eta, y, w, av, fc, d1, d2, dv);
          cy = count_part_generic(fc.code, (double)y, (double)av);
        } else {
          family_entry<FAM, true>(eta, y, w, fc, d1, d2, dv);
          const int yi = (int)y;
          cy = (yi >= 0 && yi < kTileThreads && (float)yi == y) ? ctab[yi]
                                                                : count_part<FAM>((double)y, alpha);
        }
        acc[r] += (double)dv + 2.0 * (double)w * cy;
      }
    }
  }
  for (int r = 0; r < kRowDevRows; ++r) {
    double x = acc[r];
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) red[wave][r] = x;
  }
  __syncthreads();
  if (tid < nr) a.out[i0 + tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
}

template <int FAM, bool HAS_W>
static hipError_t launch_row_dev_kp(int KP, const RowDevArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.n + kRowDevRows - 1) / kRowDevRows)), block(kTileThreads);
  switch (KP) {
    case 16: hipLaunchKernelGGL((row_deviance_kernel<FAM, 16, HAS_W>), grid, block, 0, s, a); break;
    case 32: hipLaunchKernelGGL((row_deviance_kernel<FAM, 32, HAS_W>), grid, block, 0, s, a); break;
    case 48: hipLaunchKernelGGL((row_deviance_kernel<FAM, 48, HAS_W>), grid, block, 0, s, a); break;
    case 64: hipLaunchKernelGGL((row_deviance_kernel<FAM, 64, HAS_W>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int FAM>
static hipError_t launch_row_dev_w(int KP, const RowDevArgs& a, hipStream_t s) {
  return a.Wb ? launch_row_dev_kp<FAM, true>(KP, a, s) : launch_row_dev_kp<FAM, false>(KP, a, s);
}

hipError_t launch_row_deviance(int fam, int KP, const RowDevArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  switch (fam) {
    case kPoisson: return launch_row_dev_w<kPoisson>(KP, a, s);
    case kNegBin: return launch_row_dev_w<kNegBin>(KP, a, s);
    case kGaussian: return launch_row_dev_w<kGaussian>(KP, a, s);
    case kGeneric: return launch_row_dev_w<kGeneric>(KP, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_deviance(int fam, int KP, const DevArgs& a, hipStream_t s) {
  switch (fam) {
    case kPoisson: return launch_dev_kp<kPoisson>(KP, a, s);
    case kNegBin: return launch_dev_kp<kNegBin>(KP, a, s);
    case kGaussian: return launch_dev_kp<kGaussian>(KP, a, s);
    case kGeneric: return launch_dev_kp<kGeneric>(KP, a, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------ dispersion estimation --
constexpr int kStatRows = 16;

int block_stats_workgroups(int n_b) { return (n_b + kStatRows - 1) / kStatRows; }

__global__ __launch_bounds__(kTileThreads) void block_stats_kernel(BlockStatsArgs a) {
  __shared__ float sP[kStatRows][65];
  __shared__ double red[3][kTileThreads];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * kStatRows;
  const int nr = min(kStatRows, a.n_b - r0);
  for (int idx = tid; idx < kStatRows * a.KP; idx += kTileThreads) {
    const int r = idx / a.KP, k = idx % a.KP;
    sP[r][k] = r < nr ? a.Prow[(int64_t)(r0 + r) * a.KP + k] : 0.f;
  }
  __syncthreads();
  const FamilyConst fc = family_const(a.f);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int j = tid; j < a.m_b; j += kTileThreads) {
    const float* pc = a.Pcol + (int64_t)j * a.KP;
    const float alpha = column_alpha(fc, a.col0 + j);
    for (int r = 0; r < nr; ++r) {
      const int64_t at = (int64_t)(r0 + r) * a.ldy + j;
      const float y = a.Y[at];
      if (!(y == y)) continue;   // missing
      float eta = 0.f;
      for (int k = 0; k < a.KP; ++k) eta = fmaf(sP[r][k], pc[k], eta);
      const float mu = inverse_link_code(fc.link, eta, fc.lo, fc.hi);
      const double w = a.W ? (double)a.W[at] : 1.0;
      const double res = (double)y - (double)mu;
      s0 += w * res * res / (double)variance_code(fc.code, mu, alpha);
      s1 += w * (double)mu * (double)mu;
      s2 += w * (res * res - (double)mu);
    }
  }
  red[0][tid] = s0;
  red[1][tid] = s1;
  red[2][tid] = s2;
  __syncthreads();
  for (int off = kTileThreads / 2; off > 0; off >>= 1) {
    if (tid < off)
      for (int q = 0; q < 3; ++q) red[q][tid] += red[q][tid + off];
    __syncthreads();
  }
  if (tid < 3) a.partial[3 * (int64_t)blockIdx.x + tid] = red[tid][0];
}

hipError_t launch_block_stats(const BlockStatsArgs& a, hipStream_t s) {
  const int nwg = block_stats_workgroups(a.n_b);
  if (nwg <= 0) return hipSuccess;
  if (a.KP > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(block_stats_kernel, dim3(nwg), dim3(kTileThreads), 0, s, a);
  return hipGetLastError();
}

__global__ void est_update_kernel(const double* partial, int nwg, double* est, double scale_phi,
                                  double rho, double eps, int est_phi, int est_alpha) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int i = 0; i < nwg; ++i) {
    s0 += partial[3 * i];
    s1 += partial[3 * i + 1];
    s2 += partial[3 * i + 2];
  }
  if (est_phi) est[0] = (1.0 - rho) * est[0] + rho * (scale_phi * s0);
  if (est_alpha) est[1] = (1.0 - rho) * est[1] + rho * fmax(eps, s1 / s2);
}

hipError_t launch_est_update(const double* partial, int nwg, double* est, double scale_phi,
                             double rho, double eps, int est_phi, int est_alpha, hipStream_t s) {
  hipLaunchKernelGGL(est_update_kernel, dim3(1), dim3(64), 0, s, partial, nwg, est, scale_phi, rho,
                     eps, est_phi, est_alpha);
  return hipGetLastError();
}

// ------------------------------------------------- held-out metrics --
__global__ __launch_bounds__(kTileThreads) void observed_sum_kernel(DevArgs a, double* partial) {
  __shared__ double red[2][kTileThreads];
  const int tile = blockIdx.x;
  const int blk = a.tile_block[tile];
  const int local = tile - a.tile_first[blk];
  const int n_b = a.blk_nb[blk], m_b = a.blk_mb[blk];
  const int ldy = a.blk_ldy[blk];
  const int n_ct = a.blk_nct[blk];
  const int rpw = a.blk_rpw[blk];
  const float* Y = a.Y + a.blk_yoff[blk];
  const int ct = local % n_ct, rr = local / n_ct;
  const int row0 = rr * rpw, row_end = min(n_b, row0 + rpw);
  const int col0 = ct * kTileCols, col_end = min(m_b, col0 + kTileCols);
  double sy = 0.0, cnt = 0.0;
  const int c = col0 + (int)(threadIdx.x % kTileCols);
  if (c < col_end)
    for (int r = row0 + (int)(threadIdx.x / kTileCols); r < row_end; r += kTileThreads / kTileCols) {
      const float y = Y[(int64_t)r * ldy + c];
      if (y == y) {
        sy += (double)y;
        cnt += 1.0;
      }
    }
  red[0][threadIdx.x] = sy;
  red[1][threadIdx.x] = cnt;
  __syncthreads();
  for (int off = kTileThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x < 2) partial[2 * (int64_t)tile + threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_observed_sum(const DevArgs& a, double* partial, hipStream_t s) {
  if (a.n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(observed_sum_kernel, dim3(a.n_tiles), dim3(kTileThreads), 0, s, a, partial);
  return hipGetLastError();
}

int heldout_workgroups(int64_t n) { return (int)((n + kStatRows - 1) / kStatRows); }

__global__ __launch_bounds__(kTileThreads) void heldout_kernel(HeldoutArgs a) {
  __shared__ float sP[kStatRows][65];
  __shared__ int64_t orow[kStatRows];
  __shared__ double red[7][kTileThreads];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kStatRows;
  const int nr = (int)min<int64_t>(kStatRows, a.n - r0);
  for (int idx = tid; idx < kStatRows * a.KP; idx += kTileThreads) {
    const int r = idx / a.KP, k = idx % a.KP;
    sP[r][k] = r < nr ? a.Prow[(r0 + r) * a.KP + k] : 0.f;
  }
  if (tid < kStatRows) orow[tid] = tid < nr ? (int64_t)a.row_perm[r0 + tid] : 0;
  __syncthreads();
  const FamilyConst fc = family_const(a.f);
  const float ybar = (float)a.ybar;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t jp = tid; jp < a.m; jp += kTileThreads) {
    const float* pc = a.Pcol + jp * a.KP;
    const int64_t jo = a.col_perm[jp];
    const float alpha = column_alpha(fc, jp);
    for (int r = 0; r < nr; ++r) {
      const int64_t at = orow[r] * a.m + jo;
      float y;
      if (a.y_int) {
        const int v = static_cast<const int*>(a.Ytest)[at];
        if (v < 0) continue;
        y = (float)v;
      } else {
        y = static_cast<const float*>(a.Ytest)[at];
        if (!(y == y)) continue;
      }
      float eta = 0.f;
      for (int k = 0; k < a.KP; ++k) eta = fmaf(sP[r][k], pc[k], eta);
      const float mu = inverse_link_code(fc.link, eta, fc.lo, fc.hi);
      const double l1 = (double)logf((1.f + y) / (1.f + mu));
      const double l0 = (double)logf((1.f + y) / (1.f + ybar));
      acc[0] += l1 * l1;
      acc[1] += l0 * l0;
      acc[2] += (double)unit_deviance_code(kCodePoisson, y, mu, alpha);
      acc[3] += (double)unit_deviance_code(kCodePoisson, y, ybar, alpha);
      acc[4] += (double)unit_deviance_code(fc.code, y, mu, alpha);
      acc[5] += (double)unit_deviance_code(fc.code, y, ybar, alpha);
      acc[6] += 1.0;
    }
  }
  for (int q = 0; q < 7; ++q) red[q][tid] = acc[q];
  __syncthreads();
  for (int off = kTileThreads / 2; off > 0; off >>= 1) {
    if (tid < off)
      for (int q = 0; q < 7; ++q) red[q][tid] += red[q][tid + off];
    __syncthreads();
  }
  if (tid < 7) a.partial[8 * (int64_t)blockIdx.x + tid] = red[tid][0];
}

hipError_t launch_heldout(const HeldoutArgs& a, hipStream_t s) {
  const int nwg = heldout_workgroups(a.n);
  if (nwg <= 0) return hipSuccess;
  if (a.KP > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(heldout_kernel, dim3(nwg), dim3(kTileThreads), 0, s, a);
  return hipGetLastError();
}

__global__ void check_positive_kernel(const float* x, int64_t count, int* err_flag) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count && !(x[idx] > 0.f && isfinite(x[idx]))) atomicOr(err_flag, 2);
}

hipError_t launch_check_positive(const float* x, int64_t count, int* err_flag, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_positive_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                     x, count, err_flag);
  return hipGetLastError();
}

}  // namespace gmf
