// Kernels of the parameter initialization (Section 4.1, "Parameter
// initialization", least-squares form) on gfx950.
//
// The initialization never forms the n x m matrices it works with.  Every
// pass over Y computes, entry by entry from the block-major counts and the
// current panels, one of
//   mode 0  L = g(y + c)                          (link-transformed response)
//   mode 1  L - eta,  eta = [X|Gamma] [B|Z]'      (link-scale residual)
//   mode 2  (y - mu) sqrt(w / nu(mu))             (Pearson residual)
//   mode 3  sign(y - mu) sqrt(w D(y, mu))         (deviance residual)
//   mode 4  1 for an observed entry, 0 for a missing one
// with mu = g^-1(eta) clamped like the fit's mean, and contracts it with a
// dense operand in the same pass:
//   row pass     out_s[i, :] = sum_{j in J_s} E_ij Om[j, :]   (E Om, per column block s)
//   column pass  out_c[j, :] = sum_{i in chunk c} E_ij Q[i, :]  (E' Q, per row chunk c)
// Partial results (float32 sums over 64-entry tiles, one set per column block
// or row chunk) are summed in float64 in a fixed order by sum_parts_kernel, so
// the results do not depend on scheduling.  A missing entry (NaN in the
// block-major Y) contributes its imputed value: in mode 0 the column's value
// given in colfill (the current prediction of the column), else 0 (y <- mu).
//
// The small dense algebra of the randomized range finder and of the normal
// equations (Gram matrices of tall operands, products with k x k matrices)
// runs in float64: gram_kernel, apply_kernel.
#include <hip/hip_runtime.h>

#include "family.hpp"
#include "gmf_kernels.hpp"

namespace gmf {

namespace {

constexpr int kT = 64;        // tile edge (rows and columns)
constexpr int kThreads = 256;

struct EntryConst {
  int fam, link;
  float c_off, alpha, lo, hi;
  const float* alpha_col;   // NB shape per permuted column, or null
};

// L = g(y + c): log(y + c), y + c, or for the logit link logit((y + c)/(1 + 2c)).
__device__ __forceinline__ float link_transform(float y, const EntryConst& c) {
  if (c.link == kLinkLog) return logf(y + c.c_off);
  if (c.link == kLinkLogit) {
    const float q = (y + c.c_off) / (1.f + 2.f * c.c_off);
    return logf(q / (1.f - q));
  }
  return y + c.c_off;
}

template <int MODE>
__device__ __forceinline__ float init_entry(float y, float w, float eta, float fill, float alpha,
                                            const EntryConst& c) {
  if (y != y) return MODE == 0 ? fill : 0.f;          // missing: imputed value
  if constexpr (MODE == 4) {
    return 1.f;                                       // observed indicator
  } else if constexpr (MODE == 0) {
    return link_transform(y, c);
  } else if constexpr (MODE == 1) {
    return link_transform(y, c) - eta;
  } else {
    const float mu = inverse_link_code(c.link, eta, c.lo, c.hi);
    if constexpr (MODE == 2) {
      return (y - mu) * sqrtf(w / variance_code(c.fam, mu, alpha));
    } else {
      const float r = sqrtf(w * fmaxf(unit_deviance_code(c.fam, y, mu, alpha), 0.f));
      return y > mu ? r : (y < mu ? -r : 0.f);
    }
  }
}

// Loads the first ke panel columns of `rows` panel rows starting at row0 into
// s[row][k] (zero past `rows`).
__device__ __forceinline__ void load_panel_rows(const float* P, int KP, int64_t row0, int rows,
                                                int ke, float (*s)[33]) {
  for (int idx = threadIdx.x; idx < kT * ke; idx += kThreads) {
    const int r = idx / ke, k = idx % ke;
    s[r][k] = r < rows ? P[(row0 + r) * KP + k] : 0.f;
  }
}

// Loads `rows` rows of a dense operand (ld kq) starting at row0 into s (kq
// columns, zero past `rows`).
__device__ __forceinline__ void load_dense_rows(const float* Q, int kq, int64_t row0, int rows,
                                                float (*s)[kT]) {
  for (int idx = threadIdx.x; idx < kT * kq; idx += kThreads) {
    const int r = idx / kq, k = idx % kq;
    s[r][k] = r < rows ? Q[(row0 + r) * kq + k] : 0.f;
  }
}

// The 64 x 64 tile of E at rows [li0, li0 + nr) of row block r and columns
// [lj0, lj0 + nc) of column block s into sE (zero outside).  sA: the rows'
// panel entries, sB: the columns' (k-major, sB[k][col]).
template <int MODE>
__device__ __forceinline__ void entry_tile(const InitPassArgs& a, int r, int s, int li0, int nr,
                                           int lj0, int nc, float (*sA)[33], float (*sBt)[kT],
                                           float (*sE)[kT + 1], const EntryConst& c) {
  const int col = threadIdx.x & (kT - 1);
  const int ldy = a.ldy[s];
  const int64_t base = (int64_t)a.ro[r] * a.LDtot + (int64_t)a.nrows[r] * a.coP[s];
  const float fill = (MODE == 0 && a.colfill && col < nc) ? a.colfill[a.co[s] + lj0 + col] : 0.f;
  for (int row = threadIdx.x >> 6; row < kT; row += kThreads / kT) {
    float e = 0.f;
    if (row < nr && col < nc) {
      const int64_t off = base + (int64_t)(li0 + row) * ldy + lj0 + col;
      const float y = a.Yb[off];
      const float w = a.Wb ? a.Wb[off] : 1.f;
      float eta = 0.f;
      if constexpr (MODE == 1 || MODE == 2 || MODE == 3)
        for (int k = 0; k < a.ke; ++k) eta = fmaf(sA[row][k], sBt[k][col], eta);
      const float alpha = c.alpha_col ? c.alpha_col[a.co[s] + lj0 + col] : c.alpha;
      e = init_entry<MODE>(y, w, eta, fill, alpha, c);
    }
    sE[row][col] = e;
  }
}

EntryConst entry_const(const InitPassArgs& a) {
  EntryConst c;
  c.fam = a.f.code;
  c.link = a.f.link;
  c.c_off = a.c_off;
  c.alpha = a.f.nb_alpha;
  c.lo = a.f.eta_lo;
  c.hi = a.f.eta_hi;
  c.alpha_col = a.f.alpha_col;
  return c;
}

}  // namespace

// Row pass: workgroup (x = row tile from the table, y = column block s).
template <int MODE>
__global__ __launch_bounds__(kThreads) void init_row_pass_kernel(InitPassArgs a, EntryConst c) {
  __shared__ float sA[kT][33];
  __shared__ float sBt[32][kT];
  __shared__ float sE[kT][kT + 1];
  __shared__ float sO[kT][kT];
  const int r = a.tiles[2 * blockIdx.x], li0 = a.tiles[2 * blockIdx.x + 1];
  const int s = blockIdx.y;
  const int nr = min(kT, a.nrows[r] - li0);
  const int ms = a.mcols[s];
  const int64_t prow0 = (int64_t)a.ro[r] + li0;
  if (MODE >= 1 && MODE <= 3) load_panel_rows(a.Prow, a.KP, prow0, nr, a.ke, sA);
  const int row = threadIdx.x >> 2, g = threadIdx.x & 3;
  const int per = (a.kq + 3) / 4;   // outputs per thread, contiguous
  float acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = 0.f;
  for (int lj0 = 0; lj0 < ms; lj0 += kT) {
    const int nc = min(kT, ms - lj0);
    const int64_t pcol0 = (int64_t)a.co[s] + lj0;
    __syncthreads();
    if (MODE >= 1 && MODE <= 3)
      for (int idx = threadIdx.x; idx < kT * a.ke; idx += kThreads) {
        const int cc = idx / a.ke, k = idx % a.ke;
        sBt[k][cc] = cc < nc ? a.Pcol[(pcol0 + cc) * a.KP + k] : 0.f;
      }
    load_dense_rows(a.Q, a.kq, pcol0, nc, sO);
    __syncthreads();
    entry_tile<MODE>(a, r, s, li0, nr, lj0, nc, sA, sBt, sE, c);
    __syncthreads();
    for (int cc = 0; cc < nc; ++cc) {
      const float e = sE[row][cc];
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (t < per && g * per + t < a.kq) acc[t] = fmaf(e, sO[cc][g * per + t], acc[t]);
    }
  }
  if (row < nr) {
    float* out = a.part + ((int64_t)s * a.nout + prow0 + row) * a.kq;
#pragma unroll
    for (int t = 0; t < 16; ++t)
      if (t < per && g * per + t < a.kq) out[g * per + t] = acc[t];
  }
}

// Column pass: workgroup (x = column tile from the table, y = row chunk from
// the chunk table: row block, first row, rows).
template <int MODE>
__global__ __launch_bounds__(kThreads) void init_col_pass_kernel(InitPassArgs a, EntryConst c) {
  __shared__ float sA[kT][33];
  __shared__ float sBt[32][kT];
  __shared__ float sE[kT][kT + 1];
  __shared__ float sQ[kT][kT];
  const int s = a.tiles[2 * blockIdx.x], lj0 = a.tiles[2 * blockIdx.x + 1];
  const int r = a.chunks[3 * blockIdx.y], ci0 = a.chunks[3 * blockIdx.y + 1];
  const int crows = a.chunks[3 * blockIdx.y + 2];
  const int nc = min(kT, a.mcols[s] - lj0);
  const int64_t pcol0 = (int64_t)a.co[s] + lj0;
  if (MODE >= 1 && MODE <= 3)
    for (int idx = threadIdx.x; idx < kT * a.ke; idx += kThreads) {
      const int cc = idx / a.ke, k = idx % a.ke;
      sBt[k][cc] = cc < nc ? a.Pcol[(pcol0 + cc) * a.KP + k] : 0.f;
    }
  const int col = threadIdx.x >> 2, g = threadIdx.x & 3;
  const int per = (a.kq + 3) / 4;
  float acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = 0.f;
  for (int li0 = ci0; li0 < ci0 + crows; li0 += kT) {
    const int nr = min(kT, ci0 + crows - li0);
    const int64_t prow0 = (int64_t)a.ro[r] + li0;
    __syncthreads();
    if (MODE >= 1 && MODE <= 3) load_panel_rows(a.Prow, a.KP, prow0, nr, a.ke, sA);
    load_dense_rows(a.Q, a.kq, prow0, nr, sQ);
    __syncthreads();
    entry_tile<MODE>(a, r, s, li0, nr, lj0, nc, sA, sBt, sE, c);
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      const float e = sE[rr][col];
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (t < per && g * per + t < a.kq) acc[t] = fmaf(e, sQ[rr][g * per + t], acc[t]);
    }
  }
  if (col < nc) {
    float* out = a.part + ((int64_t)blockIdx.y * a.nout + pcol0 + col) * a.kq;
#pragma unroll
    for (int t = 0; t < 16; ++t)
      if (t < per && g * per + t < a.kq) out[g * per + t] = acc[t];
  }
}

hipError_t launch_init_pass(const InitPassArgs& a, bool row_pass, int grid_x, int grid_y,
                            hipStream_t st) {
  if (grid_x <= 0 || grid_y <= 0) return hipSuccess;
  if (a.kq < 1 || a.kq > 64 || a.ke < 0 || a.ke > 32) return hipErrorInvalidValue;
  const EntryConst c = entry_const(a);
  const dim3 grid(grid_x, grid_y), block(kThreads);
#define GMF_INIT_CASE(M)                                                                  \
  case M:                                                                                 \
    if (row_pass) hipLaunchKernelGGL(init_row_pass_kernel<M>, grid, block, 0, st, a, c); \
    else hipLaunchKernelGGL(init_col_pass_kernel<M>, grid, block, 0, st, a, c);          \
    break;
  switch (a.mode) {
    GMF_INIT_CASE(0)
    GMF_INIT_CASE(1)
    GMF_INIT_CASE(2)
    GMF_INIT_CASE(3)
    GMF_INIT_CASE(4)
    default: return hipErrorInvalidValue;
  }
#undef GMF_INIT_CASE
  return hipGetLastError();
}

// out[x] = sum_{c < nparts} part[c * stride + x] in float64, c ascending.
__global__ void sum_parts_kernel(const float* part, int nparts, int64_t stride, int64_t count,
                                 double* out64, float* out32) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= count) return;
  double s = 0.0;
  for (int c = 0; c < nparts; ++c) s += (double)part[(int64_t)c * stride + x];
  if (out64) out64[x] = s;
  if (out32) out32[x] = (float)s;
}

hipError_t launch_sum_parts(const float* part, int nparts, int64_t stride, int64_t count,
                            double* out64, float* out32, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                     part, nparts, stride, count, out64, out32);
  return hipGetLastError();
}

// Gram matrix of a tall float64 operand A (rows x k, ld k): workgroup b sums
// rows [b*rows_per, (b+1)*rows_per) into part[b] (k x k); the partials are
// then summed in order by sum_gram_kernel.
__global__ __launch_bounds__(256) void gram_kernel(const double* A, int64_t rows, int k,
                                                   int64_t rows_per, double* part) {
  __shared__ double sR[32][65];
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = min(rows, r0 + rows_per);
  double acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = 0.0;
  for (int64_t c0 = r0; c0 < r1; c0 += 32) {
    const int nr = (int)min<int64_t>(32, r1 - c0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < 32 * k; idx += 256) {
      const int rr = idx / k, cc = idx % k;
      sR[rr][cc] = rr < nr ? A[(c0 + rr) * k + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int pair = threadIdx.x + 256 * t;
      if (pair < k * k) {
        const int a = pair / k, b = pair % k;
        double sacc = acc[t];
        for (int rr = 0; rr < nr; ++rr) sacc = fma(sR[rr][a], sR[rr][b], sacc);
        acc[t] = sacc;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int pair = threadIdx.x + 256 * t;
    if (pair < k * k) part[(int64_t)blockIdx.x * k * k + pair] = acc[t];
  }
}

__global__ void sum_gram_kernel(const double* part, int nparts, int kk, double* out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= kk) return;
  double s = 0.0;
  for (int c = 0; c < nparts; ++c) s += part[(int64_t)c * kk + x];
  out[x] = s;
}

hipError_t launch_gram(const double* A, int64_t rows, int k, double* part, int nparts, double* out,
                       hipStream_t st) {
  if (k < 1 || k > 64) return hipErrorInvalidValue;
  const int64_t rows_per = (rows + nparts - 1) / nparts;
  hipLaunchKernelGGL(gram_kernel, dim3(nparts), dim3(256), 0, st, A, rows, k, rows_per, part);
  hipLaunchKernelGGL(sum_gram_kernel, dim3((k * k + 255) / 256), dim3(256), 0, st, part, nparts,
                     k * k, out);
  return hipGetLastError();
}

// out = A M (A rows x ka float64, M ka x kb float64 on the device), written as
// float64 (out64, ld kb), float32 (out32, ld kb) and/or into panel columns
// [col0, col0 + kb) of a panel with stride KP, column j times scale[j].
__global__ __launch_bounds__(256) void apply_kernel(const double* A, int64_t rows, int ka, int kb,
                                                    const double* M, const double* scale,
                                                    double* out64, float* out32, float* panel,
                                                    int KP, int col0) {
  __shared__ double sM[64 * 64];
  for (int idx = threadIdx.x; idx < ka * kb; idx += 256) sM[idx] = M[idx];
  __syncthreads();
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= rows * kb) return;
  const int64_t i = idx / kb;
  const int j = (int)(idx % kb);
  double s = 0.0;
  for (int k = 0; k < ka; ++k) s = fma(A[i * ka + k], sM[k * kb + j], s);
  if (scale) s *= scale[j];
  if (out64) out64[idx] = s;
  if (out32) out32[idx] = (float)s;
  if (panel) panel[i * KP + col0 + j] = (float)s;
}

hipError_t launch_apply(const double* A, int64_t rows, int ka, int kb, const double* M,
                        const double* scale, double* out64, float* out32, float* panel, int KP,
                        int col0, hipStream_t st) {
  if (ka < 1 || ka > 64 || kb < 1 || kb > 64) return hipErrorInvalidValue;
  const int64_t tot = rows * kb;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(apply_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, A, rows,
                     ka, kb, M, scale, out64, out32, panel, KP, col0);
  return hipGetLastError();
}

// Panel columns [col0, col0 + ncols) of `rows` panel rows: read into dense
// float64 / float32 arrays (ld ncols), or set to zero.
__global__ void panel_cols_kernel(float* P, int KP, int64_t rows, int col0, int ncols,
                                  double* out64, float* out32, int zero) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * ncols) return;
  const int64_t i = idx / ncols;
  const int c = (int)(idx % ncols);
  float* p = P + i * KP + col0 + c;
  if (zero) {
    *p = 0.f;
    return;
  }
  if (out64) out64[idx] = (double)*p;
  if (out32) out32[idx] = *p;
}

hipError_t launch_panel_cols(float* P, int KP, int64_t rows, int col0, int ncols, double* out64,
                             float* out32, int zero, hipStream_t st) {
  const int64_t tot = rows * ncols;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(panel_cols_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, P,
                     KP, rows, col0, ncols, out64, out32, zero);
  return hipGetLastError();
}

// out[x] = num[x] / den[x] (0 where den is 0), float32.
__global__ void ratio_kernel(const double* num, const double* den, int64_t count, float* out) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < count) out[x] = den[x] > 0.0 ? (float)(num[x] / den[x]) : 0.f;
}

hipError_t launch_ratio(const double* num, const double* den, int64_t count, float* out,
                        hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(ratio_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, num,
                     den, count, out);
  return hipGetLastError();
}

}  // namespace gmf
