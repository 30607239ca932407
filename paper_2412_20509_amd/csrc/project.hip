// Row-only steps of the projection of new rows: Algorithm 1, steps 2-4, for
// the rows of the new samples only, with the column side (B, Z, V) frozen
// (the projection of Section 4 that scores unseen samples on a fitted model).
//
// With the column side fixed, the rows are independent problems, so a step on
// column block J_s needs no communication between rows: one wavefront owns RT
// tiles of 16 rows and walks all columns of J_s in chunks of 32, keeping its
// gradient and curvature sums
//   G[i][o] = sum_j D1[i][j] [Z,V][j][o],   H[i][o] = sum_j D2[i][j] [Z^2,V^2][j][o]
// in MFMA accumulators, then applies the scaled sums, the ridge term, the EMAs
// (eq. 12) and the step (eq. 13-14) to its own rows.  No partial sums leave
// the wavefront, there is no update launch and no LDS or barrier.  Per chunk:
//   1. eta^T (16 rows x 32 columns per row tile) on the matrix cores, A = the
//      chunk's column panel rows (loaded once for all row tiles), B = the
//      wavefront's row panel (loaded once per step, the pre-step values);
//   2. the family epilogue (clamp, inverse link, D1, D2) in registers;
//   3. G and H with A = D1 (D2) straight from the eta accumulators and
//      B = the chunk's column panel (squared for H).
// The next chunk's counts and column panel rows are loaded before the current
// chunk is computed.  The precisions are those of the fit steps: float32
// products, bfloat16 operands, or split bfloat16 (high and low parts, three
// products per contraction), with 16x16x32 bfloat16 products, or 16x16x16 at
// panel stride 16.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "family.hpp"
#include "gmf_kernels.hpp"
#include "mfma.hpp"

namespace gmf {

namespace {

constexpr int kWaves = 4;      // wavefronts per workgroup
constexpr int kChunk = 32;     // columns per chunk

// D(16x16) += A(16x16) B(16x16), bfloat16 operands, float32 accumulation: lane
// (i, g) holds A[i][4g .. 4g+3] and B[4g .. 4g+3][i] (the bfloat16 products
// at panel stride 16).
__device__ __forceinline__ floatx4 mfma_bf16_k16(bf16x4 a, bf16x4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x4 to_bf16x4(floatx4 x) { return __builtin_convertvector(x, bf16x4); }
__device__ __forceinline__ bf16x4 lo_bf16x4(floatx4 x, bf16x4 hi) {
  return to_bf16x4(x - __builtin_convertvector(hi, floatx4));
}

// One chunk's loads: column panel rows and counts (float32, or 16-bit
// integers with CY, converted when used).
template <int PREC, int KP, int RT, bool CY>
struct Chunk {
  static constexpr int NB = KP / 16;
  // eta's A operand: column c0 + 16C + l16, panel entries k (FP32: 4kk + g;
  // bfloat16: 32kk + 8g .. +7; bfloat16 at stride 16: 4g .. 4g+3)
  float pa[2][KP / 4];
  // U side B operand: column c0 + 16C + 4g + v, panel entry 16ob + l16
  float ub[2][4][NB];
  // row r0 + 16 rt + l16, columns c0 + 16C + 4g .. +3
  typename std::conditional<CY, uint2, float4>::type y[RT][2];
};

template <int PREC, int KP, int RT, bool CY>
__device__ __forceinline__ void load_chunk(const ProjStepArgs& a, int c0, int64_t r0,
                                           int l16, int g, Chunk<PREC, KP, RT, CY>& ch) {
  constexpr int NB = KP / 16;
  for (int C = 0; C < 2; ++C) {
    const int col = c0 + 16 * C + l16;
    const bool ok = col < a.m_b;
    const float* pc = a.Pcol + (int64_t)col * KP;
    if constexpr (PREC == kF32) {
      for (int kk = 0; kk < KP / 4; ++kk) ch.pa[C][kk] = ok ? pc[4 * kk + g] : 0.f;
    } else if constexpr (KP == 16) {
      const float4 u = ok ? *reinterpret_cast<const float4*>(pc + 4 * g) : make_float4(0.f, 0.f, 0.f, 0.f);
      ch.pa[C][0] = u.x; ch.pa[C][1] = u.y; ch.pa[C][2] = u.z; ch.pa[C][3] = u.w;
    } else {
      for (int kk = 0; kk < KP / 32; ++kk) {
        float4 u = make_float4(0.f, 0.f, 0.f, 0.f), w = u;
        if (ok) {
          u = *reinterpret_cast<const float4*>(pc + 32 * kk + 8 * g);
          w = *reinterpret_cast<const float4*>(pc + 32 * kk + 8 * g + 4);
        }
        float* d = &ch.pa[C][8 * kk];
        d[0] = u.x; d[1] = u.y; d[2] = u.z; d[3] = u.w;
        d[4] = w.x; d[5] = w.y; d[6] = w.z; d[7] = w.w;
      }
    }
    for (int v = 0; v < 4; ++v) {
      const int cu = c0 + 16 * C + 4 * g + v;
      const bool oku = cu < a.m_b;
      for (int ob = 0; ob < NB; ++ob)
        ch.ub[C][v][ob] = oku ? a.Pcol[(int64_t)cu * KP + 16 * ob + l16] : 0.f;
    }
    const int colb = c0 + 16 * C + 4 * g;
    for (int rt = 0; rt < RT; ++rt) {
      const int64_t row = r0 + 16 * rt + l16;
      if constexpr (CY) {
        ch.y[rt][C] = make_uint2(0u, 0u);
        if (row < a.n && colb < a.ldy)
          ch.y[rt][C] = *reinterpret_cast<const uint2*>(a.Yc + row * a.ldy + colb);
      } else {
        ch.y[rt][C] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < a.n && colb < a.ldy)
          ch.y[rt][C] = *reinterpret_cast<const float4*>(a.Y + row * a.ldy + colb);
      }
    }
  }
}

template <int PREC, int FAM, int KP, int RT, bool CY>
__global__ __launch_bounds__(kWave * kWaves, 2) void project_step_kernel(ProjStepArgs a) {
  constexpr int kRows = 16 * RT;   // rows per wavefront
  constexpr int NB = KP / 16;
  constexpr bool BF = PREC != kF32;
  constexpr bool SPLIT = PREC == kBF16X3;
  constexpr bool SPLIT_H = SPLIT && kSplitCurvature;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int64_t r0 = ((int64_t)blockIdx.x * kWaves + wave) * kRows;
  if (r0 >= a.n) return;   // uniform over the wavefront

  // eta's B operand: the row panel of row r0 + 16 rt + l16, pre-step values
  constexpr bool K16 = BF && KP == 16;   // bfloat16 products of K = 16
  float pb32[RT][(PREC == kF32) ? KP / 4 : 1];
  bf16x8 pb16[RT][(BF && !K16) ? KP / 32 : 1], pb16l[RT][(SPLIT && !K16) ? KP / 32 : 1];
  bf16x4 pk[RT], pkl[RT];
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t row = r0 + 16 * rt + l16;
    const bool row_ok = row < a.n;
    const float* pr = a.Prow + row * KP;
    if constexpr (PREC == kF32) {
      for (int kk = 0; kk < KP / 4; ++kk) pb32[rt][kk] = row_ok ? pr[4 * kk + g] : 0.f;
    } else if constexpr (K16) {
      const float4 u = row_ok ? *reinterpret_cast<const float4*>(pr + 4 * g) : make_float4(0.f, 0.f, 0.f, 0.f);
      const floatx4 x = {u.x, u.y, u.z, u.w};
      pk[rt] = to_bf16x4(x);
      if constexpr (SPLIT) pkl[rt] = lo_bf16x4(x, pk[rt]);
    } else {
      for (int kk = 0; kk < KP / 32; ++kk) {
        float4 u = make_float4(0.f, 0.f, 0.f, 0.f), w = u;
        if (row_ok) {
          u = *reinterpret_cast<const float4*>(pr + 32 * kk + 8 * g);
          w = *reinterpret_cast<const float4*>(pr + 32 * kk + 8 * g + 4);
        }
        const floatx8 x = {u.x, u.y, u.z, u.w, w.x, w.y, w.z, w.w};
        pb16[rt][kk] = to_bf16(x);
        if constexpr (SPLIT) pb16l[rt][kk] = lo_bf16(x, pb16[rt][kk]);
      }
    }
  }

  const FamilyConst fc = family_const(a.f);
  floatx4 ug[RT][NB], uh[RT][NB];
  for (int rt = 0; rt < RT; ++rt)
    for (int ob = 0; ob < NB; ++ob) ug[rt][ob] = uh[rt][ob] = floatx4{0.f, 0.f, 0.f, 0.f};

  Chunk<PREC, KP, RT, CY> cur, nxt{};
  load_chunk<PREC, KP, RT, CY>(a, 0, r0, l16, g, cur);
  for (int c0 = 0; c0 < a.m_b; c0 += kChunk) {
    if (c0 + kChunk < a.m_b) load_chunk<PREC, KP, RT, CY>(a, c0 + kChunk, r0, l16, g, nxt);
    // the chunk's column operands, converted once for all row tiles
    bf16x8 ah[2][(BF && !K16) ? KP / 32 : 1], al[2][(SPLIT && !K16) ? KP / 32 : 1];
    bf16x8 bh[(BF && !K16) ? NB : 1], bq[(BF && !K16) ? NB : 1], bhl[(SPLIT && !K16) ? NB : 1],
        bql[(SPLIT_H && !K16) ? NB : 1];
    // stride 16: per 16 columns C, A = the panel entries 4g .. 4g+3 of column
    // c0 + 16C + l16 (eta), B = entry l16 of columns c0 + 16C + 4g .. +3 (G, H)
    bf16x4 kah[2], kal[2], kbh[2], kbl[2], kqh[2], kql[2];
    if constexpr (K16) {
      for (int C = 0; C < 2; ++C) {
        const floatx4 x = {cur.pa[C][0], cur.pa[C][1], cur.pa[C][2], cur.pa[C][3]};
        kah[C] = to_bf16x4(x);
        if constexpr (SPLIT) kal[C] = lo_bf16x4(x, kah[C]);
        const floatx4 b = {cur.ub[C][0][0], cur.ub[C][1][0], cur.ub[C][2][0], cur.ub[C][3][0]};
        const floatx4 bb = b * b;
        kbh[C] = to_bf16x4(b);
        kqh[C] = to_bf16x4(bb);
        if constexpr (SPLIT) kbl[C] = lo_bf16x4(b, kbh[C]);
        if constexpr (SPLIT_H) kql[C] = lo_bf16x4(bb, kqh[C]);
      }
    } else if constexpr (BF) {
      for (int C = 0; C < 2; ++C)
        for (int kk = 0; kk < KP / 32; ++kk) {
          const float* s = &cur.pa[C][8 * kk];
          const floatx8 x = {s[0], s[1], s[2], s[3], s[4], s[5], s[6], s[7]};
          ah[C][kk] = to_bf16(x);
          if constexpr (SPLIT) al[C][kk] = lo_bf16(x, ah[C][kk]);
        }
      // k = 8g + u <-> column c0 + 16 (u / 4) + 4g + u % 4
      for (int ob = 0; ob < NB; ++ob) {
        const floatx8 x = {cur.ub[0][0][ob], cur.ub[0][1][ob], cur.ub[0][2][ob], cur.ub[0][3][ob],
                           cur.ub[1][0][ob], cur.ub[1][1][ob], cur.ub[1][2][ob], cur.ub[1][3][ob]};
        const floatx8 xq = x * x;
        bh[ob] = to_bf16(x);
        bq[ob] = to_bf16(xq);
        if constexpr (SPLIT) bhl[ob] = lo_bf16(x, bh[ob]);
        if constexpr (SPLIT_H) bql[ob] = lo_bf16(xq, bq[ob]);
      }
    }
    for (int rt = 0; rt < RT; ++rt) {
      // ---- eta^T: e[v] = eta(row r0 + 16 rt + l16, column c0 + 16C + 4g + v)
      float d1[2][4], d2[2][4];
      for (int C = 0; C < 2; ++C) {
        floatx4 e = {0.f, 0.f, 0.f, 0.f};
        if constexpr (PREC == kF32) {
          for (int kk = 0; kk < KP / 4; ++kk) e = mfma_f32(cur.pa[C][kk], pb32[rt][kk], e);
        } else if constexpr (K16) {
          if constexpr (SPLIT) {   // the small products first
            e = mfma_bf16_k16(kal[C], pk[rt], e);
            e = mfma_bf16_k16(kah[C], pkl[rt], e);
          }
          e = mfma_bf16_k16(kah[C], pk[rt], e);
        } else {
          for (int kk = 0; kk < KP / 32; ++kk) {
            if constexpr (SPLIT) {   // the small products first
              e = mfma_bf16(al[C][kk], pb16[rt][kk], e);
              e = mfma_bf16(ah[C][kk], pb16l[rt][kk], e);
            }
            e = mfma_bf16(ah[C][kk], pb16[rt][kk], e);
          }
        }
        const float4 y4 = counts_f4(cur.y[rt][C]);
        const float ys[4] = {y4.x, y4.y, y4.z, y4.w};
        for (int v = 0; v < 4; ++v) {
          float dv;
          family_entry<FAM, false>(e[v], ys[v], 1.f, fc, d1[C][v], d2[C][v], dv);
        }
      }
      // ---- G, H over the chunk's 32 columns
      if constexpr (PREC == kF32) {
        for (int C = 0; C < 2; ++C)
          for (int v = 0; v < 4; ++v)
            for (int ob = 0; ob < NB; ++ob) {
              const float b = cur.ub[C][v][ob];
              ug[rt][ob] = mfma_f32(d1[C][v], b, ug[rt][ob]);
              uh[rt][ob] = mfma_f32(d2[C][v], b * b, uh[rt][ob]);
            }
      } else if constexpr (K16) {
        // A = D1 (D2) of row l16, columns c0 + 16C + 4g .. +3 from the accumulators
        for (int C = 0; C < 2; ++C) {
          const floatx4 f1 = {d1[C][0], d1[C][1], d1[C][2], d1[C][3]};
          const floatx4 f2 = {d2[C][0], d2[C][1], d2[C][2], d2[C][3]};
          const bf16x4 b1 = to_bf16x4(f1), b2 = to_bf16x4(f2);
          if constexpr (SPLIT) {
            ug[rt][0] = mfma_bf16_k16(lo_bf16x4(f1, b1), kbh[C], ug[rt][0]);
            ug[rt][0] = mfma_bf16_k16(b1, kbl[C], ug[rt][0]);
          }
          if constexpr (SPLIT_H) {
            uh[rt][0] = mfma_bf16_k16(lo_bf16x4(f2, b2), kqh[C], uh[rt][0]);
            uh[rt][0] = mfma_bf16_k16(b2, kql[C], uh[rt][0]);
          }
          ug[rt][0] = mfma_bf16_k16(b1, kbh[C], ug[rt][0]);
          uh[rt][0] = mfma_bf16_k16(b2, kqh[C], uh[rt][0]);
        }
      } else {
        const floatx8 f1 = {d1[0][0], d1[0][1], d1[0][2], d1[0][3], d1[1][0], d1[1][1], d1[1][2], d1[1][3]};
        const floatx8 f2 = {d2[0][0], d2[0][1], d2[0][2], d2[0][3], d2[1][0], d2[1][1], d2[1][2], d2[1][3]};
        const bf16x8 b1 = to_bf16(f1), b2 = to_bf16(f2);
        for (int ob = 0; ob < NB; ++ob) {
          if constexpr (SPLIT) {
            ug[rt][ob] = mfma_bf16(lo_bf16(f1, b1), bh[ob], ug[rt][ob]);
            ug[rt][ob] = mfma_bf16(b1, bhl[ob], ug[rt][ob]);
          }
          if constexpr (SPLIT_H) {
            uh[rt][ob] = mfma_bf16(lo_bf16(f2, b2), bq[ob], uh[rt][ob]);
            uh[rt][ob] = mfma_bf16(b2, bql[SPLIT_H ? ob : 0], uh[rt][ob]);
          }
          ug[rt][ob] = mfma_bf16(b1, bh[ob], ug[rt][ob]);
          uh[rt][ob] = mfma_bf16(b2, bq[ob], uh[rt][ob]);
        }
      }
    }
    cur = nxt;
  }

  // ---- update: lane (l16, g) holds G and H of rows r0 + 16 rt + 4g + v,
  // panel entry o = 16 ob + l16; the row parameters are the entries [p, p + q + d)
  bool ok = true;
  for (int ob = 0; ob < NB; ++ob) {
    const int o = 16 * ob + l16;
    const int oo = o - a.p;
    if (oo < 0 || oo >= a.KU) continue;
    const double lam = (oo < a.q) ? a.lam_A : a.lam_U;
    for (int rt = 0; rt < RT; ++rt)
      for (int v = 0; v < 4; ++v) {
        const int64_t rw = r0 + 16 * rt + 4 * g + v;
        if (rw >= a.n) continue;
        float* th = a.Prow + rw * KP + o;
        const double theta = (double)*th;
        ok = ema_step(th, a.Grow + rw * a.KU + oo, a.Hrow + rw * a.KU + oo,
                      a.scale_m * (double)ug[rt][ob][v] + lam * theta,
                      a.scale_m * (double)uh[rt][ob][v] + lam, a.a1, a.a2, a.damping, a.stepsize) && ok;
      }
  }
  if (!ok) atomicOr(a.err_flag, 1);
}

// Row tiles per wavefront: two for panel strides up to 32 (each chunk's column
// operands then serve 32 rows; 10-20 % faster per epoch than one tile on a
// 1,000,000 x 2000 projection), one for the larger strides (registers).
constexpr int rt_of(int prec, int KP) { return (KP <= 32) ? 2 : 1; }

// cy: the 16-bit counts (Poisson and NB only).
template <int PREC, int FAM, int KP>
const void* kernel_ptr(bool cy) {
  if constexpr (FAM == kPoisson || FAM == kNegBin)
    if (cy) return reinterpret_cast<const void*>(&project_step_kernel<PREC, FAM, KP, rt_of(PREC, KP), true>);
  return reinterpret_cast<const void*>(&project_step_kernel<PREC, FAM, KP, rt_of(PREC, KP), false>);
}

template <int PREC, int FAM>
const void* kernel_for_kp(int KP, bool cy) {
  switch (KP) {
    case 16: return kernel_ptr<PREC, FAM, 16>(cy);
    case 32: return kernel_ptr<PREC, FAM, 32>(cy);
    case 48: if constexpr (PREC == kF32) return kernel_ptr<PREC, FAM, 48>(cy); else break;
    case 64: return kernel_ptr<PREC, FAM, 64>(cy);
  }
  return nullptr;
}

template <int PREC>
const void* kernel_for_fam(int fam, int KP, bool cy) {
  switch (fam) {
    case kPoisson: return kernel_for_kp<PREC, kPoisson>(KP, cy);
    case kNegBin: return kernel_for_kp<PREC, kNegBin>(KP, cy);
    case kGaussian: return kernel_for_kp<PREC, kGaussian>(KP, cy);
  }
  return nullptr;
}

}  // namespace

hipError_t launch_project_step(int prec, int fam, int KP, const ProjStepArgs& a, hipStream_t s) {
  const void* k = nullptr;
  const bool cy = a.Yc != nullptr;
  if (prec == kF32) k = kernel_for_fam<kF32>(fam, KP, cy);
  else if (prec == kBF16) k = kernel_for_fam<kBF16>(fam, KP, cy);
  else if (prec == kBF16X3) k = kernel_for_fam<kBF16X3>(fam, KP, cy);
  if (!k) return hipErrorInvalidValue;
  if (a.n <= 0 || a.m_b <= 0) return hipSuccess;
  const int64_t rows_per_wg = (int64_t)16 * rt_of(prec, KP) * kWaves;
  const dim3 grid((unsigned)((a.n + rows_per_wg - 1) / rows_per_wg));
  void* args[] = {const_cast<ProjStepArgs*>(&a)};
  return hipLaunchKernel(k, grid, dim3(kWave * kWaves), args, 0, s);
}

}  // namespace gmf
