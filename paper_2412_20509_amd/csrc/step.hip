// Fused block step of the adaptive SGD for GMF (Algorithm 1, steps 2-4, with
// the covariate extension of Appendix A) on gfx950.
//
// tile_kernel: one workgroup = 4 wavefronts = a range of block rows x a strip
// of 128 block columns (32 per wavefront).  For every 32x32 piece it
//   1. forms eta^T = [B|Z|V]_J [X|Gamma|U]_I^T on the matrix cores (MFMA
//      16x16, K = padded p+q+d), one 16x16 output per (col, row) sub-tile;
//   2. applies the fused epilogue: clamp, inverse link, D1, D2, deviance;
//   3. U side: sums over the wavefront's columns D1 [Z,V]_J and D2 [Z^2,V^2]_J
//      with MFMA (A = D1 straight from the eta registers);
//   4. V side: sums over rows D1^T [X,U]_I and D2^T [X^2,U^2]_I with MFMA
//      (A = D1^T, obtained by a transpose through LDS).
// U-side sums are reduced across the 4 wavefronts in a fixed order and written
// per (column strip, row); V-side sums are accumulated across the whole row
// range in registers and written per (row range, column).  Nothing of the
// n* x m* block (eta, mu, D1, D2) is written to memory.
//
// update_kernel: sums the partials in a fixed order, scales by m/m* or n/n*
// (eq. 15), adds the ridge terms, updates the float64 EMAs (eq. 12) and takes
// the bias-corrected diagonal quasi-Newton step (eq. 13-14).
#include <hip/hip_runtime.h>

#include "family.hpp"
#include "gmf_kernels.hpp"

namespace gmf {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ floatx4 mfma_f32(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Row stride (in elements) of the per-wavefront transpose buffers.
template <int PREC> struct TStride { static constexpr int v = (PREC == kF32) ? 36 : 40; };

template <int PREC>
using TElem = typename std::conditional<PREC == kF32, float, __bf16>::type;

template <int PREC, int FAM, int KP>
__global__ __launch_bounds__(kTileThreads) void tile_kernel(TileArgs a) {
  constexpr int NB = KP / 16;          // 16-wide output blocks of the contractions
  constexpr int TS = TStride<PREC>::v;
  using TE = TElem<PREC>;

  __shared__ float sP[kRowGroup][KP + 4];                 // staged row-panel rows
  __shared__ TE sT[kTileWaves][2][kWaveCols][TS];         // D1^T, D2^T per wavefront
  __shared__ float sU[kTileWaves][kRowGroup][2 * KP + 1]; // U-side sums per wavefront
  __shared__ double sDev[kTileWaves];

  const BlockView& B = a.b;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int g = lane >> 4;
  const int ct = blockIdx.x % B.n_ct;
  const int rr = blockIdx.x / B.n_ct;
  const int row0 = rr * B.rows_per_wg;
  const int row_end = min(B.n_b, row0 + B.rows_per_wg);
  const int colw = ct * kTileCols + wave * kWaveCols;   // first column of this wavefront
  const bool want_dev = a.want_dev != 0;

  // ---- column-panel operands of this wavefront (fixed for the whole range)
  // eta A operand: Pcol[col = colw + 16c + l16][k]
  float pa32[2][(PREC == kF32) ? KP / 4 : 1];
  bf16x8 pa16[2][(PREC == kBF16) ? KP / 32 : 1];
  // U-side B operands: Pcol[col][o] and its square
  float ub32[2][4][(PREC == kF32) ? NB : 1], ub32q[2][4][(PREC == kF32) ? NB : 1];
  bf16x8 ub16[(PREC == kBF16) ? NB : 1], ub16q[(PREC == kBF16) ? NB : 1];

  for (int c = 0; c < 2; ++c) {
    const int col = colw + 16 * c + l16;
    const bool ok = col < B.m_b;
    const float* pc = B.Pcol + (int64_t)col * KP;
    if constexpr (PREC == kF32) {
      for (int kk = 0; kk < KP / 4; ++kk) pa32[c][kk] = ok ? pc[4 * kk + g] : 0.f;
    } else {
      for (int kk = 0; kk < KP / 32; ++kk)
        for (int u = 0; u < 8; ++u)
          pa16[c][kk][u] = (__bf16)(ok ? pc[32 * kk + 8 * g + u] : 0.f);
    }
  }
  if constexpr (PREC == kF32) {
    for (int c = 0; c < 2; ++c)
      for (int v = 0; v < 4; ++v) {
        const int col = colw + 16 * c + 4 * g + v;
        const bool ok = col < B.m_b;
        for (int ob = 0; ob < NB; ++ob) {
          const float x = ok ? B.Pcol[(int64_t)col * KP + 16 * ob + l16] : 0.f;
          ub32[c][v][ob] = x;
          ub32q[c][v][ob] = x * x;
        }
      }
  } else {
    for (int ob = 0; ob < NB; ++ob)
      for (int u = 0; u < 8; ++u) {
        const int col = colw + (u < 4 ? 4 * g + u : 16 + 4 * g + (u - 4));
        const bool ok = col < B.m_b;
        const float x = ok ? B.Pcol[(int64_t)col * KP + 16 * ob + l16] : 0.f;
        ub16[ob][u] = (__bf16)x;
        ub16q[ob][u] = (__bf16)(x * x);
      }
  }

  floatx4 vacc[2][NB][2];     // V side: [col sub-tile][out block][G/H]
  for (int c = 0; c < 2; ++c)
    for (int ob = 0; ob < NB; ++ob)
      for (int h = 0; h < 2; ++h) vacc[c][ob][h] = floatx4{0.f, 0.f, 0.f, 0.f};
  double dev_acc = 0.0;

  for (int rg = row0; rg < row_end; rg += kRowGroup) {
    __syncthreads();   // previous group's readers of sP / sU are done
    // ---- stage rows rg..rg+31 of the row panel
    for (int idx = tid; idx < kRowGroup * (KP / 4); idx += kTileThreads) {
      const int r = idx / (KP / 4);
      const int c4 = idx % (KP / 4);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (rg + r < B.n_b)
        v = reinterpret_cast<const float4*>(B.Prow + (int64_t)(rg + r) * KP)[c4];
      sP[r][4 * c4 + 0] = v.x;
      sP[r][4 * c4 + 1] = v.y;
      sP[r][4 * c4 + 2] = v.z;
      sP[r][4 * c4 + 3] = v.w;
    }
    __syncthreads();

    // ---- eta, epilogue: lane holds cols 16C+4g+v, row 16R+l16 of the piece
    float d1[2][2][4], d2[2][2][4];
    for (int R = 0; R < 2; ++R) {
      const int row = rg + 16 * R + l16;
      const bool row_ok = row < B.n_b;
      for (int C = 0; C < 2; ++C) {
        floatx4 e = {0.f, 0.f, 0.f, 0.f};
        if constexpr (PREC == kF32) {
          for (int kk = 0; kk < KP / 4; ++kk)
            e = mfma_f32(pa32[C][kk], sP[16 * R + l16][4 * kk + g], e);
        } else {
          for (int kk = 0; kk < KP / 32; ++kk) {
            bf16x8 bb;
            for (int u = 0; u < 8; ++u) bb[u] = (__bf16)sP[16 * R + l16][32 * kk + 8 * g + u];
            e = mfma_bf16(pa16[C][kk], bb, e);
          }
        }
        const int colb = colw + 16 * C + 4 * g;
        float4 y4 = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 w4 = make_float4(1.f, 1.f, 1.f, 1.f);
        if (row_ok && colb < B.ldy) {
          y4 = *reinterpret_cast<const float4*>(B.Y + (int64_t)row * B.ldy + colb);
          if (B.W) w4 = *reinterpret_cast<const float4*>(B.W + (int64_t)row * B.ldy + colb);
        }
        const float ys[4] = {y4.x, y4.y, y4.z, y4.w};
        const float ws[4] = {w4.x, w4.y, w4.z, w4.w};
        for (int v = 0; v < 4; ++v) {
          float x1 = 0.f, x2 = 0.f, dv = 0.f;
          if (row_ok && colb + v < B.m_b) {
            family_entry<FAM>(e[v], ys[v], ws[v], a.f, want_dev, x1, x2, dv);
            if (want_dev) dev_acc += (double)dv;
          }
          d1[R][C][v] = x1;
          d2[R][C][v] = x2;
        }
      }
    }

    // ---- transpose D1, D2 into this wavefront's LDS buffers: sT[w][h][col][row]
    for (int R = 0; R < 2; ++R)
      for (int C = 0; C < 2; ++C)
        for (int v = 0; v < 4; ++v) {
          sT[wave][0][16 * C + 4 * g + v][16 * R + l16] = (TE)d1[R][C][v];
          sT[wave][1][16 * C + 4 * g + v][16 * R + l16] = (TE)d2[R][C][v];
        }
    __syncthreads();

    // ---- V side: G_V[col][o] += sum_row D1[row][col] P[row][o]
    for (int C = 0; C < 2; ++C) {
      if constexpr (PREC == kF32) {
        float t1[8], t2[8];
        for (int s = 0; s < 8; ++s) {
          t1[s] = sT[wave][0][16 * C + l16][8 * g + s];
          t2[s] = sT[wave][1][16 * C + l16][8 * g + s];
        }
        for (int s = 0; s < 8; ++s)
          for (int ob = 0; ob < NB; ++ob) {
            const float pb = sP[8 * g + s][16 * ob + l16];
            vacc[C][ob][0] = mfma_f32(t1[s], pb, vacc[C][ob][0]);
            vacc[C][ob][1] = mfma_f32(t2[s], pb * pb, vacc[C][ob][1]);
          }
      } else {
        bf16x8 t1, t2;
        for (int u = 0; u < 8; ++u) {
          t1[u] = sT[wave][0][16 * C + l16][8 * g + u];
          t2[u] = sT[wave][1][16 * C + l16][8 * g + u];
        }
        for (int ob = 0; ob < NB; ++ob) {
          bf16x8 pb, pq;
          for (int u = 0; u < 8; ++u) {
            const float x = sP[8 * g + u][16 * ob + l16];
            pb[u] = (__bf16)x;
            pq[u] = (__bf16)(x * x);
          }
          vacc[C][ob][0] = mfma_bf16(t1, pb, vacc[C][ob][0]);
          vacc[C][ob][1] = mfma_bf16(t2, pq, vacc[C][ob][1]);
        }
      }
    }

    // ---- U side: G_U[row][o] = sum_col D1[row][col] P[col][o] over this wavefront
    for (int R = 0; R < 2; ++R) {
      floatx4 ug[NB], uh[NB];
      for (int ob = 0; ob < NB; ++ob) {
        ug[ob] = floatx4{0.f, 0.f, 0.f, 0.f};
        uh[ob] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
      if constexpr (PREC == kF32) {
        for (int C = 0; C < 2; ++C)
          for (int v = 0; v < 4; ++v)
            for (int ob = 0; ob < NB; ++ob) {
              ug[ob] = mfma_f32(d1[R][C][v], ub32[C][v][ob], ug[ob]);
              uh[ob] = mfma_f32(d2[R][C][v], ub32q[C][v][ob], uh[ob]);
            }
      } else {
        bf16x8 x1, x2;
        for (int u = 0; u < 4; ++u) {
          x1[u] = (__bf16)d1[R][0][u];
          x1[4 + u] = (__bf16)d1[R][1][u];
          x2[u] = (__bf16)d2[R][0][u];
          x2[4 + u] = (__bf16)d2[R][1][u];
        }
        for (int ob = 0; ob < NB; ++ob) {
          ug[ob] = mfma_bf16(x1, ub16[ob], ug[ob]);
          uh[ob] = mfma_bf16(x2, ub16q[ob], uh[ob]);
        }
      }
      // D layout: lane holds rows 4g+v of sub-tile R, output o = 16ob + l16
      for (int ob = 0; ob < NB; ++ob)
        for (int v = 0; v < 4; ++v) {
          sU[wave][16 * R + 4 * g + v][16 * ob + l16] = ug[ob][v];
          sU[wave][16 * R + 4 * g + v][KP + 16 * ob + l16] = uh[ob][v];
        }
    }
    __syncthreads();

    // ---- reduce over the 4 wavefronts (fixed order) and store the strip partial
    const int KU = a.KU;
    for (int idx = tid; idx < kRowGroup * 2 * KU; idx += kTileThreads) {
      const int r = idx / (2 * KU);
      const int oo = idx % (2 * KU);
      const int row = rg + r;
      if (row >= B.n_b) continue;
      const int src = (oo < KU) ? (a.p + oo) : (KP + a.p + (oo - KU));
      const float s = ((sU[0][r][src] + sU[1][r][src]) + sU[2][r][src]) + sU[3][r][src];
      a.Upart[((int64_t)ct * B.n_b + row) * (2 * KU) + oo] = s;
    }
  }

  // ---- V-side partial of this row range: cols colw+16C+4g+v, outputs 16ob+l16
  const int KV = a.KV;
  for (int C = 0; C < 2; ++C)
    for (int v = 0; v < 4; ++v) {
      const int col = colw + 16 * C + 4 * g + v;
      if (col >= B.m_b) continue;
      float* dst = a.Vpart + ((int64_t)rr * B.m_b + col) * (2 * KV);
      for (int ob = 0; ob < NB; ++ob) {
        const int o = 16 * ob + l16;
        int oo = -1;
        if (o < a.p) oo = o;
        else if (o >= a.p + a.q && o < a.p + a.q + a.d) oo = o - a.q;
        if (oo >= 0) {
          dst[oo] = vacc[C][ob][0][v];
          dst[KV + oo] = vacc[C][ob][1][v];
        }
      }
    }

  // ---- block deviance partial of this tile (fixed reduction tree)
  if (want_dev) {
    for (int off = 32; off > 0; off >>= 1) dev_acc += __shfl_down(dev_acc, off, 64);
    if (lane == 0) sDev[wave] = dev_acc;
    __syncthreads();
    if (tid == 0) a.devpart[blockIdx.x] = ((sDev[0] + sDev[1]) + sDev[2]) + sDev[3];
  }
}

// ------------------------------------------------------------------ update --
__global__ __launch_bounds__(256) void update_kernel(UpdateArgs a) {
  const int64_t nrow_items = (int64_t)a.n_b * a.KU;
  const int64_t ncol_items = (int64_t)a.m_b * a.KV;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < nrow_items) {
    const int i = (int)(idx / a.KU);
    const int o = (int)(idx % a.KU);
    double sg = 0.0, sh = 0.0;
    for (int c = 0; c < a.n_ct; ++c) {
      const float* src = a.Upart + ((int64_t)c * a.n_b + i) * (2 * a.KU);
      sg += (double)src[o];
      sh += (double)src[a.KU + o];
    }
    float* th = a.Prow + (int64_t)i * a.KP + a.p + o;
    const double theta = (double)*th;
    const double lam = (o < a.q) ? a.lam_A : a.lam_U;
    const double G = a.scale_m * sg + lam * theta;
    const double H = a.scale_m * sh + lam;
    double* gm = a.Grow + (int64_t)i * a.KU + o;
    double* hm = a.Hrow + (int64_t)i * a.KU + o;
    const double gbar = (1.0 - a.a1) * (*gm) + a.a1 * G;
    const double hbar = (1.0 - a.a2) * (*hm) + a.a2 * H;
    *gm = gbar;
    *hm = hbar;
    const float nv = (float)(theta - a.stepsize * gbar / (hbar + a.damping));
    if (!isfinite(nv)) atomicOr(a.err_flag, 1);
    *th = nv;
  } else if (idx < nrow_items + ncol_items) {
    const int64_t k = idx - nrow_items;
    const int j = (int)(k / a.KV);
    const int o = (int)(k % a.KV);
    double sg = 0.0, sh = 0.0;
    for (int r = 0; r < a.n_rr; ++r) {
      const float* src = a.Vpart + ((int64_t)r * a.m_b + j) * (2 * a.KV);
      sg += (double)src[o];
      sh += (double)src[a.KV + o];
    }
    const int pc = (o < a.p) ? o : (o + a.q);
    float* th = a.Pcol + (int64_t)j * a.KP + pc;
    const double theta = (double)*th;
    const double lam = (o < a.p) ? a.lam_B : a.lam_V;
    const double G = a.scale_n * sg + lam * theta;
    const double H = a.scale_n * sh + lam;
    double* gm = a.Gcol + (int64_t)j * a.KV + o;
    double* hm = a.Hcol + (int64_t)j * a.KV + o;
    const double gbar = (1.0 - a.a1) * (*gm) + a.a1 * G;
    const double hbar = (1.0 - a.a2) * (*hm) + a.a2 * H;
    *gm = gbar;
    *hm = hbar;
    const float nv = (float)(theta - a.stepsize * gbar / (hbar + a.damping));
    if (!isfinite(nv)) atomicOr(a.err_flag, 1);
    *th = nv;
  } else if (idx == nrow_items + ncol_items && a.want_dev) {
    double s = 0.0;
    for (int t = 0; t < a.n_tiles; ++t) s += a.devpart[t];
    *a.dev_out = s;
  }
}

// ---------------------------------------------------------------- launchers --
template <int PREC, int FAM, int KP>
static hipError_t launch_tile_t(const TileArgs& a, hipStream_t s) {
  const int grid = a.b.n_rr * a.b.n_ct;
  hipLaunchKernelGGL((tile_kernel<PREC, FAM, KP>), dim3(grid), dim3(kTileThreads), 0, s, a);
  return hipGetLastError();
}

template <int PREC, int FAM>
static hipError_t launch_tile_kp(int KP, const TileArgs& a, hipStream_t s) {
  switch (KP) {
    case 16: if constexpr (PREC == kF32) return launch_tile_t<PREC, FAM, 16>(a, s);
             else return hipErrorInvalidValue;
    case 32: return launch_tile_t<PREC, FAM, 32>(a, s);
    case 48: if constexpr (PREC == kF32) return launch_tile_t<PREC, FAM, 48>(a, s);
             else return hipErrorInvalidValue;
    case 64: return launch_tile_t<PREC, FAM, 64>(a, s);
  }
  return hipErrorInvalidValue;
}

template <int PREC>
static hipError_t launch_tile_fam(int fam, int KP, const TileArgs& a, hipStream_t s) {
  switch (fam) {
    case kPoisson: return launch_tile_kp<PREC, kPoisson>(KP, a, s);
    case kNegBin: return launch_tile_kp<PREC, kNegBin>(KP, a, s);
    case kGaussian: return launch_tile_kp<PREC, kGaussian>(KP, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_tile(int prec, int fam, int KP, const TileArgs& a, hipStream_t s) {
  if (a.b.n_rr <= 0 || a.b.n_ct <= 0) return hipSuccess;
  if (prec == kF32) return launch_tile_fam<kF32>(fam, KP, a, s);
  return launch_tile_fam<kBF16>(fam, KP, a, s);
}

hipError_t launch_update(const UpdateArgs& a, hipStream_t s) {
  const int64_t items = (int64_t)a.n_b * a.KU + (int64_t)a.m_b * a.KV + 1;
  const int64_t grid = (items + 255) / 256;
  hipLaunchKernelGGL(update_kernel, dim3((unsigned)grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace gmf
