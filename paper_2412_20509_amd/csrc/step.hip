// Block steps of the adaptive SGD for GMF (Algorithm 1, steps 2-4, with the
// covariate extension of Appendix A) on gfx950, as one persistent launch.
//
// Work decomposition.  Step t uses the block I_r x J_s.  The block is cut into
// tiles: a range of `rpw` rows x a strip of 128 columns.  Tasks are the
// (step, tile) pairs in increasing step order; workgroups claim them from an
// atomic queue.  For every 32 x 32 piece of its tile a workgroup
//   1. forms eta^T = [B|Z|V]_J [X|Gamma|U]_I^T on the matrix cores (MFMA
//      16x16, K = padded p+q+d); sub-tile R of a 32-row group holds the rows
//      2j + R, so that a lane's two sub-tiles cover adjacent rows;
//   2. applies the fused epilogue: clamp, inverse link, D1, D2, deviance;
//   3. U side: D1 [Z,V]_J and D2 [Z^2,V^2]_J summed over its columns with MFMA
//      (A = D1 straight from the eta accumulators);
//   4. V side: D1^T [X,U]_I and D2^T [X^2,U^2]_I summed over its rows with MFMA
//      (A = D1^T after a transpose through LDS).
// Nothing of the block (eta, mu, D1, D2) is written to memory; the tile writes
// column-strip partial sums for its rows and row-range partial sums for its
// columns into a slot of partial buffers.
//
// Updates.  The last tile to finish a row range sums that range's partials over
// the column strips in a fixed order, scales by m/|J| (eq. 15), adds the ridge
// term, updates the float64 EMAs (eq. 12) and takes the step
// theta -= rho_t alpha_t Gbar/(Hbar + damping) (eq. 13-14) for [Gamma,U] of those
// rows; the last tile of a column strip does the same for [B,V] of its
// columns (scale n/|I|).  Both read only partials computed from the pre-step
// parameters, so the two halves of a step see the same iterate.
//
// Ordering.  A tile of step t waits until (a) every earlier step on row block r
// has updated the tile's row range, (b) every earlier step on column block s has
// updated its column strip, and (c) the previous user of its partial slot has
// finished.  All three are counters published by earlier steps only, so the
// lowest unfinished task can always run: the launch cannot deadlock, and steps
// on disjoint blocks overlap while the result equals sequential execution.
// Every wait is bounded; on expiry the launch aborts and reports an error.
#include <hip/hip_runtime.h>

#include "family.hpp"
#include "gmf_kernels.hpp"

namespace gmf {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ floatx4 mfma_f32(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 to_bf16(floatx8 x) { return __builtin_convertvector(x, bf16x8); }

template <int PREC> struct TStride { static constexpr int v = (PREC == kF32) ? 36 : 40; };
template <int PREC>
using TElem = typename std::conditional<PREC == kF32, float, __bf16>::type;

template <int PREC, int KP>
struct TileLds {
  static constexpr int TS = TStride<PREC>::v;
  static constexpr int T_BYTES = 2 * kWaveCols * TS * (int)sizeof(TElem<PREC>);
  static constexpr int U_BYTES = kRowGroup * (2 * KP + 1) * 4;
  static constexpr int WB = (T_BYTES > U_BYTES ? T_BYTES : U_BYTES);
  float sP[kRowGroup][KP + 4];
  alignas(16) char wave_buf[kTileWaves][WB];   // per wavefront: transpose, then U sums
  double sDev[kTileWaves];
  unsigned long long task;
  int flags[4];
};

// One tile's inputs.
struct TileView {
  const float* Y; const float* W;  // block base, row stride ldy
  const float* Prow;               // rows of I_r
  const float* Pcol;               // rows of J_s
  int ldy, n_b, m_b;
  int row0, row_end;               // row range of the tile
  int col0;                        // first column of the strip
  float* Upart;                    // this strip's partial rows: [n_b][2KU]
  float* Vpart;                    // this range's partial cols: [m_b][2KV]
};

template <int PREC, int FAM, int KP, bool WANT_DEV>
__device__ double compute_tile(const TileView& tv, const FamilyConst& fc, int p, int q, int d,
                               int KU, int KV, TileLds<PREC, KP>& L) {
  constexpr int NB = KP / 16;
  constexpr int TS = TStride<PREC>::v;
  using TE = TElem<PREC>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int g = lane >> 4;
  const int colw = tv.col0 + wave * kWaveCols;
  TE (*sT)[kWaveCols][TS] = reinterpret_cast<TE (*)[kWaveCols][TS]>(L.wave_buf[wave]);
  float (*sUw)[2 * KP + 1] = reinterpret_cast<float (*)[2 * KP + 1]>(L.wave_buf[wave]);
  const bool has_w = tv.W != nullptr;

  // ---- column-panel operands of this wavefront (fixed over the tile)
  float pa32[2][(PREC == kF32) ? KP / 4 : 1];
  bf16x8 pa16[2][(PREC == kBF16) ? KP / 32 : 1];
  float ub32[2][4][(PREC == kF32) ? NB : 1], ub32q[2][4][(PREC == kF32) ? NB : 1];
  bf16x8 ub16[(PREC == kBF16) ? NB : 1], ub16q[(PREC == kBF16) ? NB : 1];
  for (int c = 0; c < 2; ++c) {
    const int col = colw + 16 * c + l16;
    const bool ok = col < tv.m_b;
    const float* pc = tv.Pcol + (int64_t)col * KP;
    if constexpr (PREC == kF32) {
      for (int kk = 0; kk < KP / 4; ++kk) pa32[c][kk] = ok ? pc[4 * kk + g] : 0.f;
    } else {
      for (int kk = 0; kk < KP / 32; ++kk) {
        floatx8 x = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (ok) {
          const float4 a = *reinterpret_cast<const float4*>(pc + 32 * kk + 8 * g);
          const float4 b = *reinterpret_cast<const float4*>(pc + 32 * kk + 8 * g + 4);
          x = floatx8{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        }
        pa16[c][kk] = to_bf16(x);
      }
    }
  }
  if constexpr (PREC == kF32) {
    for (int c = 0; c < 2; ++c)
      for (int v = 0; v < 4; ++v) {
        const int col = colw + 16 * c + 4 * g + v;
        const bool ok = col < tv.m_b;
        for (int ob = 0; ob < NB; ++ob) {
          const float x = ok ? tv.Pcol[(int64_t)col * KP + 16 * ob + l16] : 0.f;
          ub32[c][v][ob] = x;
          ub32q[c][v][ob] = x * x;
        }
      }
  } else {
    for (int ob = 0; ob < NB; ++ob) {
      float xs[8];
      for (int u = 0; u < 8; ++u) {
        const int col = colw + (u < 4 ? 4 * g + u : 16 + 4 * g + (u - 4));
        xs[u] = (col < tv.m_b) ? tv.Pcol[(int64_t)col * KP + 16 * ob + l16] : 0.f;
      }
      const floatx8 x = {xs[0], xs[1], xs[2], xs[3], xs[4], xs[5], xs[6], xs[7]};
      ub16[ob] = to_bf16(x);
      ub16q[ob] = to_bf16(x * x);
    }
  }

  floatx4 vacc[2][NB][2];
  for (int c = 0; c < 2; ++c)
    for (int ob = 0; ob < NB; ++ob)
      for (int h = 0; h < 2; ++h) vacc[c][ob][h] = floatx4{0.f, 0.f, 0.f, 0.f};
  double dev_acc = 0.0;

  // Y of a row group: lane reads rows rg + 2 l16 + R, cols colw + 16C + 4g .. +3
  auto load_y = [&](int rg, float4 (&y)[2][2]) {
    for (int R = 0; R < 2; ++R) {
      const int row = rg + 2 * l16 + R;
      for (int C = 0; C < 2; ++C) {
        const int colb = colw + 16 * C + 4 * g;
        y[R][C] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < tv.row_end && colb < tv.ldy)
          y[R][C] = *reinterpret_cast<const float4*>(tv.Y + (int64_t)row * tv.ldy + colb);
      }
    }
  };
  float4 ynext[2][2];
  load_y(tv.row0, ynext);

  for (int rg = tv.row0; rg < tv.row_end; rg += kRowGroup) {
    float4 ycur[2][2];
    for (int R = 0; R < 2; ++R)
      for (int C = 0; C < 2; ++C) ycur[R][C] = ynext[R][C];
    __syncthreads();   // previous group's readers of sP and of the wave buffers are done
    for (int idx = tid; idx < kRowGroup * (KP / 4); idx += kTileThreads) {
      const int r = idx / (KP / 4);
      const int c4 = idx % (KP / 4);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (rg + r < tv.row_end) v = reinterpret_cast<const float4*>(tv.Prow + (int64_t)(rg + r) * KP)[c4];
      *reinterpret_cast<float4*>(&L.sP[r][4 * c4]) = v;
    }
    if (rg + kRowGroup < tv.row_end) load_y(rg + kRowGroup, ynext);   // prefetch
    __syncthreads();

    // ---- per 16-row sub-tile R: eta, epilogue, transpose store, U-side sums
    floatx4 ug[2][NB], uh[2][NB];
    for (int R = 0; R < 2; ++R) {
      const int lrow = 2 * l16 + R;
      const int row = rg + lrow;
      const bool row_ok = row < tv.row_end;
      float d1[2][4], d2[2][4];
      for (int C = 0; C < 2; ++C) {
        floatx4 e = {0.f, 0.f, 0.f, 0.f};
        if constexpr (PREC == kF32) {
          for (int kk = 0; kk < KP / 4; ++kk) e = mfma_f32(pa32[C][kk], L.sP[lrow][4 * kk + g], e);
        } else {
          for (int kk = 0; kk < KP / 32; ++kk) {
            const float4 a = *reinterpret_cast<const float4*>(&L.sP[lrow][32 * kk + 8 * g]);
            const float4 b = *reinterpret_cast<const float4*>(&L.sP[lrow][32 * kk + 8 * g + 4]);
            e = mfma_bf16(pa16[C][kk], to_bf16(floatx8{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w}), e);
          }
        }
        const int colb = colw + 16 * C + 4 * g;
        float4 w4 = make_float4(1.f, 1.f, 1.f, 1.f);
        if (has_w && row_ok && colb < tv.ldy)
          w4 = *reinterpret_cast<const float4*>(tv.W + (int64_t)row * tv.ldy + colb);
        const float ys[4] = {ycur[R][C].x, ycur[R][C].y, ycur[R][C].z, ycur[R][C].w};
        const float ws[4] = {w4.x, w4.y, w4.z, w4.w};
        for (int v = 0; v < 4; ++v) {
          float x1, x2, dv = 0.f;
          family_entry<FAM, WANT_DEV>(e[v], ys[v], ws[v], fc, x1, x2, dv);
          const bool ok = row_ok && (colb + v < tv.m_b);
          d1[C][v] = ok ? x1 : 0.f;
          d2[C][v] = ok ? x2 : 0.f;
          if constexpr (WANT_DEV) dev_acc += ok ? (double)dv : 0.0;
        }
      }
      // transposed copies for the V side: sT[h][col][row]
      for (int C = 0; C < 2; ++C)
        for (int v = 0; v < 4; ++v) {
          const int cc = 16 * C + 4 * g + v;
          sT[0][cc][lrow] = (TE)d1[C][v];
          sT[1][cc][lrow] = (TE)d2[C][v];
        }
      // U side: G_U[row][o] = sum over this wavefront's cols of D1[row][col] P[col][o]
      for (int ob = 0; ob < NB; ++ob) {
        ug[R][ob] = floatx4{0.f, 0.f, 0.f, 0.f};
        uh[R][ob] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
      if constexpr (PREC == kF32) {
        for (int C = 0; C < 2; ++C)
          for (int v = 0; v < 4; ++v)
            for (int ob = 0; ob < NB; ++ob) {
              ug[R][ob] = mfma_f32(d1[C][v], ub32[C][v][ob], ug[R][ob]);
              uh[R][ob] = mfma_f32(d2[C][v], ub32q[C][v][ob], uh[R][ob]);
            }
      } else {
        const bf16x8 b1 = to_bf16(floatx8{d1[0][0], d1[0][1], d1[0][2], d1[0][3],
                                          d1[1][0], d1[1][1], d1[1][2], d1[1][3]});
        const bf16x8 b2 = to_bf16(floatx8{d2[0][0], d2[0][1], d2[0][2], d2[0][3],
                                          d2[1][0], d2[1][1], d2[1][2], d2[1][3]});
        for (int ob = 0; ob < NB; ++ob) {
          ug[R][ob] = mfma_bf16(b1, ub16[ob], ug[R][ob]);
          uh[R][ob] = mfma_bf16(b2, ub16q[ob], uh[R][ob]);
        }
      }
    }
    __syncthreads();

    // ---- V side: G_V[col][o] += sum_row D1[row][col] P[row][o]
    for (int C = 0; C < 2; ++C) {
      if constexpr (PREC == kF32) {
        const float4 ta = *reinterpret_cast<const float4*>(&sT[0][16 * C + l16][8 * g]);
        const float4 tb = *reinterpret_cast<const float4*>(&sT[0][16 * C + l16][8 * g + 4]);
        const float4 qa = *reinterpret_cast<const float4*>(&sT[1][16 * C + l16][8 * g]);
        const float4 qb = *reinterpret_cast<const float4*>(&sT[1][16 * C + l16][8 * g + 4]);
        const float t1[8] = {ta.x, ta.y, ta.z, ta.w, tb.x, tb.y, tb.z, tb.w};
        const float t2[8] = {qa.x, qa.y, qa.z, qa.w, qb.x, qb.y, qb.z, qb.w};
        for (int s = 0; s < 8; ++s)
          for (int ob = 0; ob < NB; ++ob) {
            const float pb = L.sP[8 * g + s][16 * ob + l16];
            vacc[C][ob][0] = mfma_f32(t1[s], pb, vacc[C][ob][0]);
            vacc[C][ob][1] = mfma_f32(t2[s], pb * pb, vacc[C][ob][1]);
          }
      } else {
        const bf16x8 t1 = *reinterpret_cast<const bf16x8*>(&sT[0][16 * C + l16][8 * g]);
        const bf16x8 t2 = *reinterpret_cast<const bf16x8*>(&sT[1][16 * C + l16][8 * g]);
        for (int ob = 0; ob < NB; ++ob) {
          float xs[8];
          for (int u = 0; u < 8; ++u) xs[u] = L.sP[8 * g + u][16 * ob + l16];
          const floatx8 x = {xs[0], xs[1], xs[2], xs[3], xs[4], xs[5], xs[6], xs[7]};
          vacc[C][ob][0] = mfma_bf16(t1, to_bf16(x), vacc[C][ob][0]);
          vacc[C][ob][1] = mfma_bf16(t2, to_bf16(x * x), vacc[C][ob][1]);
        }
      }
    }
    // the wave buffer now takes the U sums: rows 2(4g+v)+R of the group, output 16ob+l16
    for (int R = 0; R < 2; ++R)
      for (int ob = 0; ob < NB; ++ob)
        for (int v = 0; v < 4; ++v) {
          sUw[2 * (4 * g + v) + R][16 * ob + l16] = ug[R][ob][v];
          sUw[2 * (4 * g + v) + R][KP + 16 * ob + l16] = uh[R][ob][v];
        }
    __syncthreads();

    // ---- sum over the 4 wavefronts (fixed order) and store the strip partial
    for (int idx = tid; idx < kRowGroup * 2 * KU; idx += kTileThreads) {
      const int r = idx / (2 * KU);
      const int oo = idx % (2 * KU);
      const int row = rg + r;
      if (row < tv.row_end) {
        const int src = (oo < KU) ? (p + oo) : (KP + p + (oo - KU));
        float s = 0.f;
        for (int w = 0; w < kTileWaves; ++w)
          s += reinterpret_cast<float (*)[2 * KP + 1]>(L.wave_buf[w])[r][src];
        tv.Upart[(int64_t)row * (2 * KU) + oo] = s;
      }
    }
  }

  // ---- V-side partial of this row range
  for (int C = 0; C < 2; ++C)
    for (int v = 0; v < 4; ++v) {
      const int col = colw + 16 * C + 4 * g + v;
      if (col < tv.m_b) {
        float* dst = tv.Vpart + (int64_t)col * (2 * KV);
        for (int ob = 0; ob < NB; ++ob) {
          const int o = 16 * ob + l16;
          int oo = -1;
          if (o < p) oo = o;
          else if (o >= p + q && o < p + q + d) oo = o - q;
          if (oo >= 0) {
            dst[oo] = vacc[C][ob][0][v];
            dst[KV + oo] = vacc[C][ob][1][v];
          }
        }
      }
    }

  // ---- tile deviance (fixed reduction tree), result valid in thread 0
  double total = 0.0;
  if constexpr (WANT_DEV) {
    for (int off = 32; off > 0; off >>= 1) dev_acc += __shfl_down(dev_acc, off, 64);
    if (lane == 0) L.sDev[wave] = dev_acc;
    __syncthreads();
    total = ((L.sDev[0] + L.sDev[1]) + L.sDev[2]) + L.sDev[3];
  }
  return total;
}

// ------------------------------------------------------------- updates ----
// EMA + step for one parameter; returns false if the result is not finite.
__device__ __forceinline__ bool ema_step(float* th, double* gm, double* hm, double G, double H,
                                         const StepKernelArgs& a, double stepsize) {
  const double gbar = (1.0 - a.a1) * (*gm) + a.a1 * G;
  const double hbar = (1.0 - a.a2) * (*hm) + a.a2 * H;
  *gm = gbar;
  *hm = hbar;
  const float nv = (float)((double)*th - stepsize * gbar / (hbar + a.damping));
  *th = nv;
  return isfinite(nv);
}

// Row range [row0, row_end) of block r: sum the n_ct strip partials.
__device__ void update_rows(const StepKernelArgs& a, int row_first, int row0, int row_end,
                            int n_b, int n_ct, const float* Ubase, double scale_m,
                            double stepsize) {
  const int KU = a.KU;
  const int items = (row_end - row0) * KU;
  bool ok = true;
  for (int idx = threadIdx.x; idx < items; idx += blockDim.x) {
    const int i = row0 + idx / KU;
    const int o = idx % KU;
    double sg = 0.0, sh = 0.0;
    int c = 0;
    for (; c + 4 <= n_ct; c += 4) {
      float g4[4], h4[4];
      for (int u = 0; u < 4; ++u) {
        const float* src = Ubase + ((int64_t)(c + u) * n_b + i) * (2 * KU);
        g4[u] = src[o];
        h4[u] = src[KU + o];
      }
      for (int u = 0; u < 4; ++u) { sg += (double)g4[u]; sh += (double)h4[u]; }
    }
    for (; c < n_ct; ++c) {
      const float* src = Ubase + ((int64_t)c * n_b + i) * (2 * KU);
      sg += (double)src[o];
      sh += (double)src[KU + o];
    }
    const int64_t grow = (int64_t)row_first + i;
    float* th = a.Prow + grow * a.KP + a.p + o;
    const double lam = (o < a.q) ? a.lam_A : a.lam_U;
    const double theta = (double)*th;
    ok = ema_step(th, a.Grow + grow * KU + o, a.Hrow + grow * KU + o, scale_m * sg + lam * theta,
                  scale_m * sh + lam, a, stepsize) && ok;
  }
  if (!ok) atomicOr(a.err_flag, 1);
}

// Column strip [col0, col_end) of block s: sum the n_rr range partials.
__device__ void update_cols(const StepKernelArgs& a, int col_first, int col0, int col_end,
                            int m_b, int n_rr, const float* Vbase, double scale_n,
                            double stepsize) {
  const int KV = a.KV;
  const int items = (col_end - col0) * KV;
  bool ok = true;
  for (int idx = threadIdx.x; idx < items; idx += blockDim.x) {
    const int j = col0 + idx / KV;
    const int o = idx % KV;
    double sg = 0.0, sh = 0.0;
    int rr = 0;
    for (; rr + 8 <= n_rr; rr += 8) {
      float g8[8], h8[8];
      for (int u = 0; u < 8; ++u) {
        const float* src = Vbase + ((int64_t)(rr + u) * m_b + j) * (2 * KV);
        g8[u] = src[o];
        h8[u] = src[KV + o];
      }
      for (int u = 0; u < 8; ++u) { sg += (double)g8[u]; sh += (double)h8[u]; }
    }
    for (; rr < n_rr; ++rr) {
      const float* src = Vbase + ((int64_t)rr * m_b + j) * (2 * KV);
      sg += (double)src[o];
      sh += (double)src[KV + o];
    }
    const int64_t gcol = (int64_t)col_first + j;
    const int pc = (o < a.p) ? o : (o + a.q);
    float* th = a.Pcol + gcol * a.KP + pc;
    const double lam = (o < a.p) ? a.lam_B : a.lam_V;
    const double theta = (double)*th;
    ok = ema_step(th, a.Gcol + gcol * KV + o, a.Hcol + gcol * KV + o, scale_n * sg + lam * theta,
                  scale_n * sh + lam, a, stepsize) && ok;
  }
  if (!ok) atomicOr(a.err_flag, 1);
}

// --------------------------------------------------------------- waits ----
__device__ __forceinline__ int ld_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin until *p >= need (thread 0 only).  Returns false on abort / expiry.
__device__ bool wait_ge(const int* p, int need, const StepKernelArgs& a) {
  for (int it = 0;; ++it) {
    if (ld_agent(p) >= need) return true;
    if (ld_agent(a.abort_flag) != 0) return false;
    if (it >= a.spin_limit) {
      atomicOr(a.err_flag, 8);
      atomicExch(a.abort_flag, 1);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Count one finished phase of the step in `slot`; the last phase opens the slot.
__device__ void phase_done(const StepKernelArgs& a, int slot, int phases) {
  if (threadIdx.x == 0) {
    const int old = atomicAdd(a.phase + slot, 1);
    if (old == phases - 1) {
      atomicExch(a.phase + slot, 0);
      __threadfence();
      atomicAdd(a.slotgen + slot, 1);
    }
  }
}

// ------------------------------------------------------------- kernel -----
template <int PREC, int FAM, int KP, bool WANT_DEV>
__global__ __launch_bounds__(kTileThreads, 2) void steps_kernel(StepKernelArgs a) {
  __shared__ TileLds<PREC, KP> L;
  const FamilyConst fc = family_const(a.f);
  const int tid = threadIdx.x;
  const int T = a.rr_max * a.ct_max;
  const unsigned long long total = (unsigned long long)a.nsteps * T;

  for (;;) {
    if (tid == 0) L.task = atomicAdd(a.task_ctr, 1ull) - a.task_base;
    __syncthreads();
    const unsigned long long task = L.task;
    __syncthreads();
    if (task >= total) break;
    const int k = (int)(task / T);
    const int tile = (int)(task % T);
    const int64_t t = a.t_first + k;
    const StepDesc sd = a.desc[(t - 1) % a.desc_window];
    const int r = sd.r, s = sd.s;
    const int n_b = a.nrows[r], m_b = a.mcols[s];
    const int n_rr = a.nrr[r], n_ct = a.nct[s], rpw = a.rpw[r];
    const int rr = tile / a.ct_max, ct = tile % a.ct_max;
    if (rr >= n_rr || ct >= n_ct) continue;   // this block has fewer tiles

    // ---- dependencies
    if (tid == 0) {
      bool ok = wait_ge(a.rowver + r * a.rr_max + rr, sd.need_row, a);
      ok = ok && wait_ge(a.colver + s * a.ct_max + ct, sd.need_col, a);
      ok = ok && wait_ge(a.slotgen + sd.slot, sd.need_slot, a);
      L.flags[0] = ok ? 1 : 0;
    }
    __syncthreads();
    if (!L.flags[0]) continue;
    __threadfence();

    // ---- the tile
    float* Uslot = a.Upart + (int64_t)sd.slot * a.slot_u_elems;
    float* Vslot = a.Vpart + (int64_t)sd.slot * a.slot_v_elems;
    double* Dslot = a.devpart + (int64_t)sd.slot * a.slot_dev_elems;
    TileView tv;
    tv.ldy = a.ldy[s];
    tv.Y = a.Y + (int64_t)a.ro[r] * a.LDtot + (int64_t)n_b * a.coP[s];
    tv.W = a.W ? a.W + (int64_t)a.ro[r] * a.LDtot + (int64_t)n_b * a.coP[s] : nullptr;
    tv.Prow = a.Prow + (int64_t)a.ro[r] * a.KP;
    tv.Pcol = a.Pcol + (int64_t)a.co[s] * a.KP;
    tv.n_b = n_b;
    tv.m_b = m_b;
    tv.row0 = rr * rpw;
    tv.row_end = min(n_b, (rr + 1) * rpw);
    tv.col0 = ct * kTileCols;
    tv.Upart = Uslot + (int64_t)ct * n_b * (2 * a.KU);
    tv.Vpart = Vslot + (int64_t)rr * m_b * (2 * a.KV);
    const double dev = compute_tile<PREC, FAM, KP, WANT_DEV>(tv, fc, a.p, a.q, a.d, a.KU, a.KV, L);
    if (tid == 0) Dslot[rr * n_ct + ct] = dev;

    // ---- arrive
    __threadfence();
    __syncthreads();
    int* arr = a.arr + (int64_t)sd.slot * (a.rr_max + a.ct_max + 1);
    if (tid == 0) {
      L.flags[1] = (atomicAdd(arr + rr, 1) == n_ct - 1);
      L.flags[2] = (atomicAdd(arr + a.rr_max + ct, 1) == n_rr - 1);
      L.flags[3] = (atomicAdd(arr + a.rr_max + a.ct_max, 1) == n_rr * n_ct - 1);
    }
    __syncthreads();
    const int phases = n_rr + n_ct + 1;
    if (L.flags[1]) {   // last tile of this row range: update [Gamma, U] of its rows
      __threadfence();
      update_rows(a, a.ro[r], tv.row0, tv.row_end, n_b, n_ct, Uslot, (double)a.m / m_b,
                  sd.stepsize);
      __threadfence();
      __syncthreads();
      if (tid == 0) {
        atomicExch(arr + rr, 0);
        __threadfence();
        atomicAdd(a.rowver + r * a.rr_max + rr, 1);
      }
      phase_done(a, sd.slot, phases);
    }
    if (L.flags[2]) {   // last tile of this column strip: update [B, V] of its columns
      __threadfence();
      update_cols(a, a.co[s], tv.col0, min(m_b, tv.col0 + kTileCols), m_b, n_rr, Vslot,
                  (double)a.n / n_b, sd.stepsize);
      __threadfence();
      __syncthreads();
      if (tid == 0) {
        atomicExch(arr + a.rr_max + ct, 0);
        __threadfence();
        atomicAdd(a.colver + s * a.ct_max + ct, 1);
      }
      phase_done(a, sd.slot, phases);
    }
    if (L.flags[3]) {   // last tile of the step: block deviance in a fixed order
      __threadfence();
      if (tid == 0) {
        if (WANT_DEV) {
          double sum = 0.0;
          for (int i = 0; i < n_rr * n_ct; ++i) sum += Dslot[i];
          a.devring[(t - 1) % a.devring_len] = sum;
        }
        atomicExch(arr + a.rr_max + a.ct_max, 0);
        __threadfence();
      }
      phase_done(a, sd.slot, phases);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ launchers ----
template <int PREC, int FAM, int KP>
static const void* kernel_ptr(bool want_dev) {
  return want_dev ? reinterpret_cast<const void*>(&steps_kernel<PREC, FAM, KP, true>)
                  : reinterpret_cast<const void*>(&steps_kernel<PREC, FAM, KP, false>);
}

template <int PREC, int FAM>
static const void* kernel_ptr_kp(int KP, bool want_dev) {
  switch (KP) {
    case 16: if constexpr (PREC == kF32) return kernel_ptr<PREC, FAM, 16>(want_dev); else break;
    case 32: return kernel_ptr<PREC, FAM, 32>(want_dev);
    case 48: if constexpr (PREC == kF32) return kernel_ptr<PREC, FAM, 48>(want_dev); else break;
    case 64: return kernel_ptr<PREC, FAM, 64>(want_dev);
  }
  return nullptr;
}

const void* steps_kernel_for(int prec, int fam, int KP, bool want_dev) {
  if (prec == kF32) {
    switch (fam) {
      case kPoisson: return kernel_ptr_kp<kF32, kPoisson>(KP, want_dev);
      case kNegBin: return kernel_ptr_kp<kF32, kNegBin>(KP, want_dev);
      case kGaussian: return kernel_ptr_kp<kF32, kGaussian>(KP, want_dev);
    }
  } else {
    switch (fam) {
      case kPoisson: return kernel_ptr_kp<kBF16, kPoisson>(KP, want_dev);
      case kNegBin: return kernel_ptr_kp<kBF16, kNegBin>(KP, want_dev);
      case kGaussian: return kernel_ptr_kp<kBF16, kGaussian>(KP, want_dev);
    }
  }
  return nullptr;
}

hipError_t launch_steps(int prec, int fam, int KP, bool want_dev, const StepKernelArgs& a,
                        int grid, hipStream_t s) {
  const void* k = steps_kernel_for(prec, fam, KP, want_dev);
  if (!k) return hipErrorInvalidValue;
  void* args[] = {const_cast<StepKernelArgs*>(&a)};
  return hipLaunchKernel(k, dim3(grid), dim3(kTileThreads), args, 0, s);
}

int steps_occupancy(int prec, int fam, int KP, bool want_dev) {
  const void* k = steps_kernel_for(prec, fam, KP, want_dev);
  if (!k) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kTileThreads, 0) != hipSuccess) return 0;
  return nb;
}

}  // namespace gmf
