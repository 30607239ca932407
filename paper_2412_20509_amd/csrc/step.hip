// Block steps of the adaptive SGD for GMF (Algorithm 1, steps 2-4, with the
// covariate extension of Appendix B) on gfx950.
//
// Tiles.  Step t uses the block I_r x J_s, cut into tiles of `rpw` rows x 128
// columns.  For every 32 x 32 piece of its tile a workgroup
//   1. forms eta^T = [B|Z|V]_J [X|Gamma|U]_I^T on the matrix cores (MFMA
//      16x16, K = padded p+q+d); sub-tile R of a 32-row group holds the rows
//      2j + R;
//   2. applies the fused epilogue: clamp, inverse link, D1, D2, deviance;
//   3. U side: D1 [Z,V]_J and D2 [Z^2,V^2]_J summed over its columns with MFMA
//      (A = D1 straight from the eta accumulators);
//   4. V side: D1^T [X,U]_I and D2^T [X^2,U^2]_I summed over its rows with MFMA
//      (A = D1^T after a transpose through LDS).
// Nothing of the block (eta, mu, D1, D2) is written to memory; the tile writes
// column-strip partial sums for its rows and row-range partial sums for its
// columns into the step's slot of partial buffers.
//
// Updates.  Row-chunk workgroups sum a chunk's partials over the column strips
// in a fixed order, scale by m/|J| (eq. 15), add the ridge term, update the
// float64 EMAs (eq. 12) and take theta -= rho_t alpha_t Gbar/(Hbar + damping)
// (eq. 13-14) for [Gamma,U]; column-chunk workgroups do the same for [B,V]
// (scale n/|I|); one workgroup sums the block deviance.  Both halves read only
// partials computed from the pre-step parameters.
//
// Levels.  One launch runs the tiles of a set of steps ("level k") and the
// updates of the steps of level k-1.  The host places step t at level
// T(t) = 2 + max(T of the previous step on row block r, T of the previous step
// on column block s, T of the previous user of its partial slot), so every
// tile runs after the updates it depends on (earlier launch) and before any
// later update of its rows or columns: the launches reproduce sequential
// execution exactly while steps on disjoint blocks run side by side.  Kernel
// boundaries are the only synchronisation.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "family.hpp"
#include "gmf_kernels.hpp"
#include "mfma.hpp"

namespace gmf {

// D(16x16) += A(16x16) B(16x16), bfloat16 operands, float32 accumulation:
// lane (i, g) holds A[i][4g .. 4g+3] and B[4g .. 4g+3][i] (the bfloat16
// products at panel stride 16).
__device__ __forceinline__ floatx4 mfma_bf16_k16(bf16x4 a, bf16x4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x4 to_bf16x4(floatx4 x) { return __builtin_convertvector(x, bf16x4); }
__device__ __forceinline__ bf16x4 lo_bf16x4(floatx4 x, bf16x4 hi) {
  return to_bf16x4(x - __builtin_convertvector(hi, floatx4));
}
__device__ __forceinline__ bf16x4 lds4(const __bf16* p) { return *reinterpret_cast<const bf16x4*>(p); }

template <int PREC> struct TStride { static constexpr int v = (PREC == kF32) ? 36 : 40; };
template <int PREC>
using TElem = typename std::conditional<PREC == kF32, float, __bf16>::type;

// LDS of a tile workgroup of NW wavefronts (4 or 8).  With 4, wavefront w
// owns columns [32w, 32w+32) and both 16-row sub-tiles of every 32-row group;
// with 8, wavefronts w and w + 4 share those columns and take sub-tile 0 and
// 1.  gbuf[c]: the transposed D1/D2 of column group c (read by the V side);
// with 4 wavefronts it then takes that wavefront's U sums (32 rows), with 8
// the U sums (16 rows per wavefront) go to ubuf.
template <int PREC, int KP, int NW>
struct TileLds {
  static constexpr int TS = TStride<PREC>::v;
  static constexpr int NTB = (PREC == kBF16X3) ? (kSplitCurvature ? 4 : 3) : 2;   // D1, D2 (+ low parts)
  static constexpr int T_BYTES = NTB * kWaveCols * TS * (int)sizeof(TElem<PREC>);
  static constexpr int U_ROWS = kRowGroup * 4 / NW;
  static constexpr int U_BYTES = U_ROWS * (2 * KP + 1) * 4;
  static constexpr int GB = (NW == 4 && U_BYTES > T_BYTES) ? U_BYTES : T_BYTES;
  // the group's row panel: float32 (the float32 tile's operands) or bfloat16
  // copies converted once per group: row-major (eta operand) and transposed,
  // plain and squared (V-side operand); with split operands also their low parts
  static constexpr int PB = (PREC != kF32) ? 1 : 0;
  float sP[PB ? 1 : kRowGroup][PB ? 4 : KP + 4];
  static constexpr int PL = (PREC == kBF16X3) ? 1 : 0;
  alignas(16) __bf16 sPb[PB ? kRowGroup : 1][PB ? KP + 8 : 8];
  alignas(16) __bf16 sPT[PB ? 2 : 1][PB ? KP : 1][PB ? kRowGroup + 8 : 8];
  alignas(16) __bf16 sPbl[PL ? kRowGroup : 1][PL ? KP + 8 : 8];
  alignas(16) __bf16 sPTl[PL ? (kSplitCurvature ? 2 : 1) : 1][PL ? KP : 1][PL ? kRowGroup + 8 : 8];
  alignas(16) char gbuf[4][GB];
  alignas(16) char ubuf[NW == 8 ? NW : 1][NW == 8 ? U_BYTES : 4];
  double sDev[NW];
  unsigned long long task;
  int flags[4];
};

// One tile's inputs.
struct TileView {
  const float* Y; const float* W;  // block base, row stride ldy
  const uint16_t* Yc;              // the counts as 16-bit integers (CY tiles), same layout
  const float* Prow;               // rows of I_r
  const float* Pcol;               // rows of J_s
  int ldy, n_b, m_b;
  int row0, row_end;               // row range of the tile
  int col0;                        // first column of the strip
  float* Upart;                    // this strip's partial rows: [n_b][2KU]
  float* Vpart;                    // this range's partial cols: [m_b][2KV]
  unsigned long long* stamps;      // optional: 3 timestamps (profiling), or null
  const float* alpha;              // generic path: NB shape of the block's columns, or null
};

template <int PREC, int FAM, int KP, bool WANT_DEV, int NW, bool HAS_W, bool CY>
__device__ double compute_tile(const TileView& tv, const FamilyConst& fc, int p, int q, int d,
                               int KU, int KV, TileLds<PREC, KP, NW>& L) {
  using YRaw = typename std::conditional<CY, uint2, float4>::type;   // 4 counts as stored
  constexpr int NB = KP / 16;
  constexpr int TS = TStride<PREC>::v;
  constexpr int NT = kWave * NW;          // threads
  constexpr int NR = (NW == 8) ? 1 : 2;   // 16-row sub-tiles per wavefront
  constexpr int NC = (NW == 8) ? 1 : 2;   // 16-column halves per wavefront on the V side
  constexpr bool BF = PREC != kF32;       // bfloat16 MFMA
  constexpr bool SPLIT = PREC == kBF16X3; // with high and low operand parts
  constexpr bool SPLIT_H = SPLIT && kSplitCurvature;
  constexpr bool K16 = BF && KP == 16;    // bfloat16 products of K = 16 (16x16x16)
  // bfloat16 transposed D1/D2 stored as row pairs: with 4 wavefronts a lane
  // holds rows 2 l16 and 2 l16 + 1 of its columns (sub-tiles 0 and 1), one
  // 32-bit store per pair, reusing the conversions of the U side (not with
  // the 16x16x16 products, where the packing cost more than it saved)
  constexpr bool PAIR_T = BF && NW == 4 && !K16;
  using TE = TElem<PREC>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int cg = wave & 3;                 // column group
  const int R0 = (NW == 8) ? (wave >> 2) : 0;
  const int l16 = lane & 15;
  const int g = lane >> 4;
  const int colw = tv.col0 + cg * kWaveCols;
  const int colw_u = __builtin_amdgcn_readfirstlane(colw);   // the same in every lane
  TE (*sT)[kWaveCols][TS] = reinterpret_cast<TE (*)[kWaveCols][TS]>(L.gbuf[cg]);
  float (*sUw)[2 * KP + 1] = (NW == 8)
      ? reinterpret_cast<float (*)[2 * KP + 1]>(L.ubuf[NW == 8 ? wave : 0])
      : reinterpret_cast<float (*)[2 * KP + 1]>(L.gbuf[cg]);
  // ---- column-panel operands of this wavefront (fixed over the tile)
  float pa32[2][(PREC == kF32) ? KP / 4 : 1];
  bf16x8 pa16[2][(BF && !K16) ? KP / 32 : 1], pa16l[2][(SPLIT && !K16) ? KP / 32 : 1];
  float ub32[2][4][(PREC == kF32) ? NB : 1], ub32q[2][4][(PREC == kF32) ? NB : 1];
  bf16x8 ub16[(BF && !K16) ? NB : 1], ub16q[(BF && !K16) ? NB : 1];
  bf16x8 ub16l[(SPLIT && !K16) ? NB : 1], ub16ql[(SPLIT_H && !K16) ? NB : 1];
  // stride 16: eta's A = entries 4g .. 4g+3 of column colw + 16c + l16; the U
  // side's B = entry l16 of columns colw + 16c + 4g .. +3 (plain and squared)
  bf16x4 ka[2], kal[2], kb[2], kbl[2], kq[2], kql[2];
  for (int c = 0; c < 2; ++c) {
    const int col = colw + 16 * c + l16;
    const bool ok = col < tv.m_b;
    const float* pc = tv.Pcol + (int64_t)col * KP;
    if constexpr (PREC == kF32) {
      for (int kk = 0; kk < KP / 4; ++kk) pa32[c][kk] = ok ? pc[4 * kk + g] : 0.f;
    } else if constexpr (K16) {
      const float4 u = ok ? *reinterpret_cast<const float4*>(pc + 4 * g) : make_float4(0.f, 0.f, 0.f, 0.f);
      const floatx4 x = {u.x, u.y, u.z, u.w};
      ka[c] = to_bf16x4(x);
      if constexpr (SPLIT) kal[c] = lo_bf16x4(x, ka[c]);
      float xs[4];
      for (int v = 0; v < 4; ++v) {
        const int cu = colw + 16 * c + 4 * g + v;
        xs[v] = (cu < tv.m_b) ? tv.Pcol[(int64_t)cu * KP + l16] : 0.f;
      }
      const floatx4 b = {xs[0], xs[1], xs[2], xs[3]};
      const floatx4 bb = b * b;
      kb[c] = to_bf16x4(b);
      kq[c] = to_bf16x4(bb);
      if constexpr (SPLIT) kbl[c] = lo_bf16x4(b, kb[c]);
      if constexpr (SPLIT_H) kql[c] = lo_bf16x4(bb, kq[c]);
    } else {
      for (int kk = 0; kk < KP / 32; ++kk) {
        floatx8 x = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (ok) {
          const float4 a = *reinterpret_cast<const float4*>(pc + 32 * kk + 8 * g);
          const float4 b = *reinterpret_cast<const float4*>(pc + 32 * kk + 8 * g + 4);
          x = floatx8{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        }
        pa16[c][kk] = to_bf16(x);
        if constexpr (SPLIT) pa16l[c][kk] = lo_bf16(x, pa16[c][kk]);
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
  } else if constexpr (!K16) {
    for (int ob = 0; ob < NB; ++ob) {
      float xs[8];
      for (int u = 0; u < 8; ++u) {
        const int col = colw + (u < 4 ? 4 * g + u : 16 + 4 * g + (u - 4));
        xs[u] = (col < tv.m_b) ? tv.Pcol[(int64_t)col * KP + 16 * ob + l16] : 0.f;
      }
      const floatx8 x = {xs[0], xs[1], xs[2], xs[3], xs[4], xs[5], xs[6], xs[7]};
      ub16[ob] = to_bf16(x);
      ub16q[ob] = to_bf16(x * x);
      if constexpr (SPLIT) {
        ub16l[ob] = lo_bf16(x, ub16[ob]);
        if constexpr (SPLIT_H) ub16ql[ob] = lo_bf16(x * x, ub16q[ob]);
      }
    }
  }

  floatx4 vacc[NC][NB][2];
  for (int c = 0; c < NC; ++c)
    for (int ob = 0; ob < NB; ++ob)
      for (int h = 0; h < 2; ++h) vacc[c][ob][h] = floatx4{0.f, 0.f, 0.f, 0.f};
  double dev_acc = 0.0;

  // Y of a row group: lane reads rows rg + 2 l16 + R, cols colw + 16C + 4g .. +3.
  // Rows past the tile end and columns past the padded row are clamped to the
  // last valid ones instead of zero-filled: those entries meet zero panel
  // operands in every contraction and are masked out of the deviance, so any
  // finite count serves.
  auto load_y = [&](int rg, YRaw (&y)[NR][2]) {
    for (int rr = 0; rr < NR; ++rr) {
      const int row = min(rg + 2 * l16 + R0 + rr, tv.row_end - 1);
      for (int C = 0; C < 2; ++C) {
        const int colb = min(colw + 16 * C + 4 * g, tv.ldy - 4);
        if constexpr (CY) y[rr][C] = *reinterpret_cast<const uint2*>(tv.Yc + (int64_t)row * tv.ldy + colb);
        else y[rr][C] = *reinterpret_cast<const float4*>(tv.Y + (int64_t)row * tv.ldy + colb);
      }
    }
  };
  // row-panel rows of a group, granules spread over the workgroup: float32
  // tiles 4 entries of a row; bfloat16 tiles 2 entries of a row pair (x, y of
  // row 2i, z, w of row 2i + 1), so that a thread writes both the row-major and
  // the transposed copies as 32-bit pairs
  constexpr int PF = (kRowGroup * (KP / 4) + NT - 1) / NT;
  auto load_p = [&](int rg, float4 (&pf)[PF]) {
    for (int u = 0; u < PF; ++u) {
      const int idx = tid + u * NT;
      pf[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (idx < kRowGroup * (KP / 4)) {
        if constexpr (BF) {
          const int r = 2 * (idx / (KP / 2)), c = 2 * (idx % (KP / 2));
          float2 a = make_float2(0.f, 0.f), b = make_float2(0.f, 0.f);
          if (rg + r < tv.row_end) a = *reinterpret_cast<const float2*>(tv.Prow + (int64_t)(rg + r) * KP + c);
          if (rg + r + 1 < tv.row_end)
            b = *reinterpret_cast<const float2*>(tv.Prow + (int64_t)(rg + r + 1) * KP + c);
          pf[u] = make_float4(a.x, a.y, b.x, b.y);
        } else {
          const int r = idx / (KP / 4), c4 = idx % (KP / 4);
          if (rg + r < tv.row_end)
            pf[u] = reinterpret_cast<const float4*>(tv.Prow + (int64_t)(rg + r) * KP)[c4];
        }
      }
    }
  };
  // strip partials: thread -> (output s_oo, rows s_r0, s_r0 + s_rows, ...),
  // fixed over the tile (2 KU <= 2 KP < NT, so every pass covers >= 2 rows)
  const int s_rows = NT / (2 * KU);
  const int s_r0 = tid / (2 * KU);
  const int s_oo = tid - s_r0 * (2 * KU);
  const bool s_on = s_r0 < s_rows;
  const int s_src = (s_oo < KU) ? (p + s_oo) : (KP + p + (s_oo - KU));
  // Where 2 KP divides the thread count, a thread instead takes one column f_o
  // of the padded U-sum rows (2 KP wide) and rows f_r0 + j RS: the passes and
  // the LDS offsets are compile-time constants, so the reads of all passes
  // issue together.  Columns outside the row side's parameters are read and
  // dropped (f_oo < 0).
  constexpr bool SFIX = NT % (2 * KP) == 0;
  constexpr int RS = SFIX ? NT / (2 * KP) : 1;
  constexpr int SJ = SFIX ? kRowGroup / RS : 1;
  const int f_o = tid % (2 * KP), f_r0 = tid / (2 * KP);
  const int f_c = (f_o < KP) ? f_o - p : f_o - KP - p;
  const int f_oo = (f_c >= 0 && f_c < KU) ? ((f_o < KP) ? f_c : KU + f_c) : -1;
  auto usum_row = [&](int c, int r) -> const float* {
    if constexpr (NW == 8)
      return reinterpret_cast<const float (*)[2 * KP + 1]>(L.ubuf[NW == 8 ? c + 4 * (r & 1) : 0])[r >> 1];
    else
      return reinterpret_cast<const float (*)[2 * KP + 1]>(L.gbuf[c])[r];
  };

  YRaw ynext[NR][2];
  float4 pnext[PF];
  load_p(tv.row0, pnext);
  load_y(tv.row0, ynext);
  if (tv.stamps && tid == 0) {
    // operands in registers: force the loads to complete before stamping
    float acc0 = 0.f;
    if constexpr (PREC == kF32) acc0 = pa32[0][0] + ub32[0][0][0];
    acc0 += counts_f4(ynext[0][0]).x + pnext[0].x;
    tv.stamps[0] = wall_clock64() + (acc0 == 12345.678f ? 1 : 0);
  }

  for (int rg = tv.row0; rg < tv.row_end; rg += kRowGroup) {
    YRaw ycur[NR][2];
    for (int rr = 0; rr < NR; ++rr)
      for (int C = 0; C < 2; ++C) ycur[rr][C] = ynext[rr][C];
    // No barrier before these stores: every reader of the row-panel buffers
    // (eta, the V side) of the previous group ran before that group's last
    // barrier, and after it the waves read only the U-sum buffers, which the
    // next writes of those (after the barrier below) cannot overtake.
    for (int u = 0; u < PF; ++u) {
      const int idx = tid + u * NT;
      if (idx < kRowGroup * (KP / 4)) {
        if constexpr (!BF) {
          const int r = idx / (KP / 4), c0 = 4 * (idx % (KP / 4));
          *reinterpret_cast<float4*>(&L.sP[r][c0]) = pnext[u];
        } else {
          // entries (r, c), (r, c + 1), (r + 1, c), (r + 1, c + 1)
          const int r = 2 * (idx / (KP / 2)), c = 2 * (idx % (KP / 2));
          const float x00 = pnext[u].x, x01 = pnext[u].y, x10 = pnext[u].z, x11 = pnext[u].w;
          auto pair = [](float a, float b) { return __builtin_convertvector(floatx2{a, b}, bf16x2); };
          auto st = [](__bf16* p, bf16x2 v) { *reinterpret_cast<bf16x2*>(p) = v; };
          st(&L.sPb[r][c], pair(x00, x01));
          st(&L.sPb[r + 1][c], pair(x10, x11));
          st(&L.sPT[0][c][r], pair(x00, x10));
          st(&L.sPT[0][c + 1][r], pair(x01, x11));
          const float q00 = x00 * x00, q01 = x01 * x01, q10 = x10 * x10, q11 = x11 * x11;
          st(&L.sPT[1][c][r], pair(q00, q10));
          st(&L.sPT[1][c + 1][r], pair(q01, q11));
          if constexpr (SPLIT) {
            auto lo = [](float a) { return a - (float)(__bf16)a; };
            st(&L.sPbl[r][c], pair(lo(x00), lo(x01)));
            st(&L.sPbl[r + 1][c], pair(lo(x10), lo(x11)));
            st(&L.sPTl[0][c][r], pair(lo(x00), lo(x10)));
            st(&L.sPTl[0][c + 1][r], pair(lo(x01), lo(x11)));
            if constexpr (kSplitCurvature) {
              st(&L.sPTl[kSplitCurvature ? 1 : 0][c][r], pair(lo(q00), lo(q10)));
              st(&L.sPTl[kSplitCurvature ? 1 : 0][c + 1][r], pair(lo(q01), lo(q11)));
            }
          }
        }
      }
    }
    if (rg + kRowGroup < tv.row_end) {   // prefetch the next group
      load_p(rg + kRowGroup, pnext);
      load_y(rg + kRowGroup, ynext);
    }
    __syncthreads();
    float dev_grp = 0.f;
    // every row and column of this wavefront's part of the group in the block
    const bool grp_full = rg + kRowGroup <= tv.row_end && colw_u + kWaveCols <= tv.m_b;

    // ---- per 16-row sub-tile R: eta, epilogue, transpose store, U-side sums
    floatx4 ug[NR][NB], uh[NR][NB];
    // bfloat16 D1, D2 (and their low parts) of columns colw + 16C + 4g + v,
    // element 4C + v, per sub-tile: the transposed stores of the row pairs
    bf16x8 th[PAIR_T ? NR : 1][SPLIT_H ? 4 : (SPLIT ? 3 : 2)];
    for (int rr = 0; rr < NR; ++rr) {
      const int R = R0 + rr;
      const int lrow = 2 * l16 + R;
      const int row = rg + lrow;
      const bool row_ok = row < tv.row_end;
      float d1[2][4], d2[2][4];
      for (int C = 0; C < 2; ++C) {
        floatx4 e = {0.f, 0.f, 0.f, 0.f};
        if constexpr (PREC == kF32) {
          for (int kk = 0; kk < KP / 4; ++kk) e = mfma_f32(pa32[C][kk], L.sP[lrow][4 * kk + g], e);
        } else if constexpr (K16) {
          const bf16x4 bh = lds4(&L.sPb[lrow][4 * g]);
          if constexpr (SPLIT) {   // the small products first
            e = mfma_bf16_k16(kal[C], bh, e);
            e = mfma_bf16_k16(ka[C], lds4(&L.sPbl[lrow][4 * g]), e);
          }
          e = mfma_bf16_k16(ka[C], bh, e);
        } else {
          for (int kk = 0; kk < KP / 32; ++kk) {
            const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&L.sPb[lrow][32 * kk + 8 * g]);
            if constexpr (SPLIT) {   // the small products first
              const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&L.sPbl[lrow][32 * kk + 8 * g]);
              e = mfma_bf16(pa16l[C][kk], bh, e);
              e = mfma_bf16(pa16[C][kk], bl, e);
            }
            e = mfma_bf16(pa16[C][kk], bh, e);
          }
        }
        const int colb = colw + 16 * C + 4 * g;
        float4 w4 = make_float4(1.f, 1.f, 1.f, 1.f);   // a literal 1 without weights
        if constexpr (HAS_W)   // clamped like the counts
          w4 = *reinterpret_cast<const float4*>(tv.W + (int64_t)min(row, tv.row_end - 1) * tv.ldy +
                                                min(colb, tv.ldy - 4));
        const float4 y4 = counts_f4(ycur[rr][C]);
        const float ys[4] = {y4.x, y4.y, y4.z, y4.w};
        const float ws[4] = {w4.x, w4.y, w4.z, w4.w};
        // Entries outside the block (rows past the tile end, padded columns)
        // need no masking in D1/D2: every contraction meets them with a zero
        // operand (zero-filled panel rows, zero column operands), and their
        // eta, mu, D1, D2 are finite.  Only the deviance sum is masked.
        // (the mask only where the wavefront's rows or columns reach past the
        // block: a branch uniform over the wavefront)
        auto entries = [&](auto masked) {
          for (int v = 0; v < 4; ++v) {
            float dv = 0.f;
            if constexpr (FAM == kGeneric) {
              const float av = tv.alpha ? tv.alpha[min(colb + v, tv.m_b - 1)] : fc.a;
              family_entry_generic<WANT_DEV, true>(e[v], ys[v], ws[v], av, fc, d1[C][v], d2[C][v], dv);
            } else if constexpr (!decltype(masked)::value) {
              family_entry_acc<FAM, WANT_DEV, HAS_W>(e[v], ys[v], ws[v], fc, d1[C][v], d2[C][v], dev_grp);
              continue;
            } else {
              family_entry<FAM, WANT_DEV, true>(e[v], ys[v], ws[v], fc, d1[C][v], d2[C][v], dv);
            }
            if constexpr (WANT_DEV) {
              if constexpr (decltype(masked)::value) dev_grp += (row_ok && colb + v < tv.m_b) ? dv : 0.f;
              else dev_grp += dv;
            }
          }
        };
        if (grp_full) entries(std::false_type{});
        else entries(std::true_type{});
      }
      // the deviance is formed here, not deferred past the contractions (the
      // per-entry values would stay live and cost registers)
      if constexpr (WANT_DEV) asm volatile("" ::"v"(dev_grp));
      // transposed copies for the V side: sT[h][col][row]
      if constexpr (!PAIR_T)
        for (int C = 0; C < 2; ++C)
          for (int v = 0; v < 4; ++v) {
            const int cc = 16 * C + 4 * g + v;
            const TE h1 = (TE)d1[C][v], h2 = (TE)d2[C][v];
            sT[0][cc][lrow] = h1;
            sT[1][cc][lrow] = h2;
            if constexpr (SPLIT) sT[2][cc][lrow] = lo_bf16(d1[C][v], h1);
            if constexpr (SPLIT_H) sT[SPLIT_H ? 3 : 2][cc][lrow] = lo_bf16(d2[C][v], h2);
          }
      // U side: G_U[row][o] = sum over this wavefront's cols of D1[row][col] P[col][o]
      for (int ob = 0; ob < NB; ++ob) {
        ug[rr][ob] = floatx4{0.f, 0.f, 0.f, 0.f};
        uh[rr][ob] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
      if constexpr (PREC == kF32) {
        for (int C = 0; C < 2; ++C)
          for (int v = 0; v < 4; ++v)
            for (int ob = 0; ob < NB; ++ob) {
              ug[rr][ob] = mfma_f32(d1[C][v], ub32[C][v][ob], ug[rr][ob]);
              uh[rr][ob] = mfma_f32(d2[C][v], ub32q[C][v][ob], uh[rr][ob]);
            }
      } else if constexpr (K16) {
        // A = D1 (D2) of row lrow, columns colw + 16C + 4g .. +3 from the accumulators
        bf16x4 k1[2], k2[2], k1l[2], k2l[2];
        for (int C = 0; C < 2; ++C) {
          const floatx4 f1 = {d1[C][0], d1[C][1], d1[C][2], d1[C][3]};
          const floatx4 f2 = {d2[C][0], d2[C][1], d2[C][2], d2[C][3]};
          const bf16x4 b1 = to_bf16x4(f1), b2 = to_bf16x4(f2);
          k1[C] = b1;
          k2[C] = b2;
          if constexpr (SPLIT) {
            k1l[C] = lo_bf16x4(f1, b1);
            ug[rr][0] = mfma_bf16_k16(k1l[C], kb[C], ug[rr][0]);
            ug[rr][0] = mfma_bf16_k16(b1, kbl[C], ug[rr][0]);
          }
          if constexpr (SPLIT_H) {
            k2l[C] = lo_bf16x4(f2, b2);
            uh[rr][0] = mfma_bf16_k16(k2l[C], kq[C], uh[rr][0]);
            uh[rr][0] = mfma_bf16_k16(b2, kql[C], uh[rr][0]);
          }
          ug[rr][0] = mfma_bf16_k16(b1, kb[C], ug[rr][0]);
          uh[rr][0] = mfma_bf16_k16(b2, kq[C], uh[rr][0]);
        }
        if constexpr (PAIR_T) {
          th[rr][0] = __builtin_shufflevector(k1[0], k1[1], 0, 1, 2, 3, 4, 5, 6, 7);
          th[rr][1] = __builtin_shufflevector(k2[0], k2[1], 0, 1, 2, 3, 4, 5, 6, 7);
          if constexpr (SPLIT) th[rr][2] = __builtin_shufflevector(k1l[0], k1l[1], 0, 1, 2, 3, 4, 5, 6, 7);
          if constexpr (SPLIT_H)
            th[rr][SPLIT_H ? 3 : 2] = __builtin_shufflevector(k2l[0], k2l[1], 0, 1, 2, 3, 4, 5, 6, 7);
        }
      } else {
        const floatx8 f1 = {d1[0][0], d1[0][1], d1[0][2], d1[0][3], d1[1][0], d1[1][1], d1[1][2], d1[1][3]};
        const floatx8 f2 = {d2[0][0], d2[0][1], d2[0][2], d2[0][3], d2[1][0], d2[1][1], d2[1][2], d2[1][3]};
        const bf16x8 b1 = to_bf16(f1), b2 = to_bf16(f2);
        bf16x8 b1l, b2l;
        if constexpr (SPLIT) b1l = lo_bf16(f1, b1);
        if constexpr (SPLIT_H) b2l = lo_bf16(f2, b2);
        for (int ob = 0; ob < NB; ++ob) {
          if constexpr (SPLIT) {
            ug[rr][ob] = mfma_bf16(b1l, ub16[ob], ug[rr][ob]);
            ug[rr][ob] = mfma_bf16(b1, ub16l[ob], ug[rr][ob]);
          }
          if constexpr (SPLIT_H) {
            uh[rr][ob] = mfma_bf16(b2l, ub16q[ob], uh[rr][ob]);
            uh[rr][ob] = mfma_bf16(b2, ub16ql[SPLIT_H ? ob : 0], uh[rr][ob]);
          }
          ug[rr][ob] = mfma_bf16(b1, ub16[ob], ug[rr][ob]);
          uh[rr][ob] = mfma_bf16(b2, ub16q[ob], uh[rr][ob]);
        }
        if constexpr (PAIR_T) {
          th[rr][0] = b1;
          th[rr][1] = b2;
          if constexpr (SPLIT) th[rr][2] = b1l;
          if constexpr (SPLIT_H) th[rr][SPLIT_H ? 3 : 2] = b2l;
        }
      }
    }
    if constexpr (PAIR_T) {
      // sT[h][col][2 l16 .. 2 l16 + 1] = (sub-tile 0, sub-tile 1)
      for (int h = 0; h < (SPLIT_H ? 4 : (SPLIT ? 3 : 2)); ++h)
        for (int C = 0; C < 2; ++C)
          for (int v = 0; v < 4; ++v) {
            const bf16x2 pr = {th[0][h][4 * C + v], th[NR - 1][h][4 * C + v]};
            *reinterpret_cast<bf16x2*>(&sT[h][16 * C + 4 * g + v][2 * l16]) = pr;
          }
    }
    // the column group's transposed rows are complete: with 4 wavefronts each
    // writes and reads only its own column group's rows (LDS operations of
    // one wavefront stay in order); with 8 the two halves of a group meet
    if constexpr (NW == 8) __syncthreads();

    // the Poisson and NB entries left out the deviance's factor 2 (NB: 2 ln 2,
    // its entries are in base-2 units)
    if constexpr (WANT_DEV) dev_acc += dev_unit<FAM>() * (double)dev_grp;
    if (tv.stamps && tid == 0 && rg == tv.row0) tv.stamps[1] = wall_clock64();
    // ---- V side: G_V[col][o] += sum_row D1[row][col] P[row][o]
    for (int cc = 0; cc < NC; ++cc) {
      const int C = (NW == 8) ? R0 : cc;
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
            vacc[cc][ob][0] = mfma_f32(t1[s], pb, vacc[cc][ob][0]);
            vacc[cc][ob][1] = mfma_f32(t2[s], pb * pb, vacc[cc][ob][1]);
          }
      } else if constexpr (K16) {
        // two K = 16 halves of the group's rows: A = D1^T of column 16C + l16,
        // rows 16h + 4g .. +3; B = the row panel entry l16 of those rows
        for (int h = 0; h < 2; ++h) {
          const int r4 = 16 * h + 4 * g;
          const bf16x4 t1 = lds4(&sT[0][16 * C + l16][r4]), t2 = lds4(&sT[1][16 * C + l16][r4]);
          const bf16x4 xb = lds4(&L.sPT[0][l16][r4]), xq = lds4(&L.sPT[1][l16][r4]);
          if constexpr (SPLIT) {
            vacc[cc][0][0] = mfma_bf16_k16(lds4(&sT[2][16 * C + l16][r4]), xb, vacc[cc][0][0]);
            vacc[cc][0][0] = mfma_bf16_k16(t1, lds4(&L.sPTl[0][l16][r4]), vacc[cc][0][0]);
          }
          if constexpr (SPLIT_H) {
            vacc[cc][0][1] = mfma_bf16_k16(lds4(&sT[SPLIT_H ? 3 : 2][16 * C + l16][r4]), xq, vacc[cc][0][1]);
            vacc[cc][0][1] = mfma_bf16_k16(t2, lds4(&L.sPTl[SPLIT_H ? 1 : 0][l16][r4]), vacc[cc][0][1]);
          }
          vacc[cc][0][0] = mfma_bf16_k16(t1, xb, vacc[cc][0][0]);
          vacc[cc][0][1] = mfma_bf16_k16(t2, xq, vacc[cc][0][1]);
        }
      } else {
        const bf16x8 t1 = *reinterpret_cast<const bf16x8*>(&sT[0][16 * C + l16][8 * g]);
        const bf16x8 t2 = *reinterpret_cast<const bf16x8*>(&sT[1][16 * C + l16][8 * g]);
        for (int ob = 0; ob < NB; ++ob) {
          const bf16x8 xb = *reinterpret_cast<const bf16x8*>(&L.sPT[0][16 * ob + l16][8 * g]);
          const bf16x8 xq = *reinterpret_cast<const bf16x8*>(&L.sPT[1][16 * ob + l16][8 * g]);
          if constexpr (SPLIT) {
            const bf16x8 t1l = *reinterpret_cast<const bf16x8*>(&sT[2][16 * C + l16][8 * g]);
            const bf16x8 xbl = *reinterpret_cast<const bf16x8*>(&L.sPTl[0][16 * ob + l16][8 * g]);
            vacc[cc][ob][0] = mfma_bf16(t1l, xb, vacc[cc][ob][0]);
            vacc[cc][ob][0] = mfma_bf16(t1, xbl, vacc[cc][ob][0]);
          }
          if constexpr (SPLIT_H) {
            const bf16x8 t2l = *reinterpret_cast<const bf16x8*>(&sT[SPLIT_H ? 3 : 2][16 * C + l16][8 * g]);
            const bf16x8 xql = *reinterpret_cast<const bf16x8*>(&L.sPTl[SPLIT_H ? 1 : 0][16 * ob + l16][8 * g]);
            vacc[cc][ob][1] = mfma_bf16(t2l, xq, vacc[cc][ob][1]);
            vacc[cc][ob][1] = mfma_bf16(t2, xql, vacc[cc][ob][1]);
          }
          vacc[cc][ob][0] = mfma_bf16(t1, xb, vacc[cc][ob][0]);
          vacc[cc][ob][1] = mfma_bf16(t2, xq, vacc[cc][ob][1]);
        }
      }
    }
    // U sums to LDS: row 4g+v of the wavefront's sub-tile rr (group row 2(4g+v)+R)
    for (int rr = 0; rr < NR; ++rr)
      for (int ob = 0; ob < NB; ++ob)
        for (int v = 0; v < 4; ++v) {
          const int ur = (NW == 8) ? (4 * g + v) : (2 * (4 * g + v) + rr);
          sUw[ur][16 * ob + l16] = ug[rr][ob][v];
          sUw[ur][KP + 16 * ob + l16] = uh[rr][ob][v];
        }
    __syncthreads();

    // ---- sum over the 4 column groups (fixed order) and store the strip partial
    if constexpr (SFIX) {
      auto strip = [&](auto ragged) {
        if (f_oo >= 0) {
          float* dst = tv.Upart + (int64_t)(rg + f_r0) * (2 * KU) + f_oo;
#pragma unroll
          for (int j = 0; j < SJ; ++j) {
            const int r = f_r0 + j * RS;
            float s = 0.f;
            for (int c = 0; c < 4; ++c) s += usum_row(c, r)[f_o];
            if (!decltype(ragged)::value || rg + r < tv.row_end) dst[(int64_t)j * RS * (2 * KU)] = s;
          }
        }
      };
      if (rg + kRowGroup <= tv.row_end) strip(std::false_type{});
      else strip(std::true_type{});
    } else if (s_on) {
      for (int r = s_r0; r < kRowGroup; r += s_rows) {
        const int row = rg + r;
        if (row < tv.row_end) {
          float s = 0.f;
          for (int c = 0; c < 4; ++c) s += usum_row(c, r)[s_src];
          tv.Upart[(int64_t)row * (2 * KU) + s_oo] = s;
        }
      }
    }
  }

  if (tv.stamps && tid == 0) tv.stamps[2] = wall_clock64();
  // ---- V-side partial of this row range
  for (int cc = 0; cc < NC; ++cc) {
    const int C = (NW == 8) ? R0 : cc;
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
            dst[oo] = vacc[cc][ob][0][v];
            dst[KV + oo] = vacc[cc][ob][1][v];
          }
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
    if constexpr (NW == 8) total += ((L.sDev[4] + L.sDev[5]) + L.sDev[6]) + L.sDev[7];
  }
  return total;
}

// ------------------------------------------------------------- updates ----
// Sum `nparts` partial segments (stride `part_stride` floats) element-wise in a
// fixed order into sums[0..seg), seg <= blockDim.x; float64 accumulation.
__device__ __forceinline__ void sum_segments(const float* base, int64_t part_stride, int nparts,
                                             int seg, double* sums) {
  const int i = threadIdx.x;
  if (i < seg) {
    double acc = 0.0;
    int k = 0;
    for (; k + 8 <= nparts; k += 8) {
      float v[8];
      for (int u = 0; u < 8; ++u) v[u] = base[(int64_t)(k + u) * part_stride + i];
      for (int u = 0; u < 8; ++u) acc += (double)v[u];
    }
    for (; k < nparts; ++k) acc += (double)base[(int64_t)k * part_stride + i];
    sums[i] = acc;
  }
}

template <int KP>
struct UpdLds {
  double sums[kTileThreads];
};

// Rows [row0, row1) of block r (block-local indices).
__device__ void update_rows(const LevelArgs& a, const LevelStep& st, int row0, int row1,
                            double* sums) {
  const int n_b = st.n_b, m_b = st.m_b;
  const int n_ct = st.n_ct;
  const int KU = a.KU;
  const float* U = a.Upart + (int64_t)st.slot * a.slot_u_elems;
  const int seg = (row1 - row0) * 2 * KU;
  const int cnt = (row1 - row0) * KU;
  // The thread's parameter, read before the partial sums so that both loads
  // are in flight together (a chunk has at most blockDim.x parameters; no
  // other workgroup of the launch writes these rows).
  const int idx = threadIdx.x;
  const int i = idx / KU, o = idx - i * KU;
  const int64_t grow = (int64_t)st.ro + row0 + i;
  float th0 = 0.f;
  double g0 = 0.0, h0 = 0.0;
  if (idx < cnt) {
    th0 = a.Prow[grow * a.KP + a.p + o];
    g0 = a.Grow[grow * KU + o];
    h0 = a.Hrow[grow * KU + o];
  }
  sum_segments(U + (int64_t)row0 * 2 * KU, (int64_t)n_b * 2 * KU, n_ct, seg, sums);
  __syncthreads();
  const double scale_m = (double)a.m / m_b;
  if (idx < cnt) {
    const double lam = (o < a.q) ? a.lam_A : a.lam_U;
    const bool ok = ema_apply(a.Prow + grow * a.KP + a.p + o, a.Grow + grow * KU + o,
                              a.Hrow + grow * KU + o, th0, g0, h0,
                              scale_m * sums[i * 2 * KU + o] + lam * (double)th0,
                              scale_m * sums[i * 2 * KU + KU + o] + lam, a.a1, a.a2, a.damping,
                              st.stepsize);
    if (!ok) atomicOr(a.err_flag, 1);
  }
}

// Columns [col0, col1) of block s (block-local indices).
__device__ void update_cols(const LevelArgs& a, const LevelStep& st, int col0, int col1,
                            double* sums) {
  const int n_b = st.n_b, m_b = st.m_b;
  const int n_rr = st.n_rr;
  const int KV = a.KV;
  const float* V = a.Vpart + (int64_t)st.slot * a.slot_v_elems;
  const int seg = (col1 - col0) * 2 * KV;
  const int cnt = (col1 - col0) * KV;
  // as in update_rows: the thread's parameter is read before the partial sums
  const int idx = threadIdx.x;
  const int j = idx / KV, o = idx - j * KV;
  const int64_t gcol = (int64_t)st.co + col0 + j;
  const int pc = (o < a.p) ? o : (o + a.q);
  float th0 = 0.f;
  double g0 = 0.0, h0 = 0.0;
  if (idx < cnt) {
    th0 = a.Pcol[gcol * a.KP + pc];
    g0 = a.Gcol[gcol * KV + o];
    h0 = a.Hcol[gcol * KV + o];
  }
  sum_segments(V + (int64_t)col0 * 2 * KV, (int64_t)m_b * 2 * KV, n_rr, seg, sums);
  __syncthreads();
  const double scale_n = (double)a.n / n_b;
  if (idx < cnt) {
    const double lam = (o < a.p) ? a.lam_B : a.lam_V;
    const bool ok = ema_apply(a.Pcol + gcol * a.KP + pc, a.Gcol + gcol * KV + o,
                              a.Hcol + gcol * KV + o, th0, g0, h0,
                              scale_n * sums[j * 2 * KV + o] + lam * (double)th0,
                              scale_n * sums[j * 2 * KV + KV + o] + lam, a.a1, a.a2, a.damping,
                              st.stepsize);
    if (!ok) atomicOr(a.err_flag, 1);
  }
}

// Block deviance of the step: fixed-order tree over the tile partials.
__device__ void sum_block_deviance(const LevelArgs& a, const LevelStep& st, double* sums) {
  const int ntiles = st.n_rr * st.n_ct;
  const double* D = a.devpart + (int64_t)st.slot * a.slot_dev_elems;
  double acc = 0.0;
  for (int i = threadIdx.x; i < ntiles; i += blockDim.x) acc += D[i];
  sums[threadIdx.x] = acc;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sums[threadIdx.x] += sums[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.devring[(st.t - 1) % a.devring_len] = sums[0];
}

// Update workgroup `local` of step `st`: a range of row chunks, of column
// chunks, or the block deviance.  Returns the task kind (1 row update, 2
// column update, 3 block deviance, -1 nothing to do).  sums: kTileThreads
// doubles of LDS; needs at least kTileThreads threads.
template <bool WANT_DEV>
__device__ __forceinline__ int run_update(const LevelArgs& a, const LevelStep& st, int local,
                                          double* sums) {
  int u = local;
  const int n_b = st.n_b, m_b = st.m_b;
  const int sub = a.upd_sub;
  const int rspan = a.row_chunk * sub, cspan = a.col_chunk * sub;
  const int nrw = (n_b + rspan - 1) / rspan;
  const int ncw = (m_b + cspan - 1) / cspan;
  if (u < nrw) {
    const int end = min(n_b, (u + 1) * rspan);
    for (int r0 = u * rspan; r0 < end; r0 += a.row_chunk) {
      update_rows(a, st, r0, min(end, r0 + a.row_chunk), sums);
      __syncthreads();   // sums is reused by the next chunk
    }
    return 1;
  }
  if ((u -= nrw) < ncw) {
    const int end = min(m_b, (u + 1) * cspan);
    for (int c0 = u * cspan; c0 < end; c0 += a.col_chunk) {
      update_cols(a, st, c0, min(end, c0 + a.col_chunk), sums);
      __syncthreads();
    }
    return 2;
  }
  if (u == ncw) {
    if (WANT_DEV) sum_block_deviance(a, st, sums);
    return 3;
  }
  return -1;
}

// ------------------------------------------------------------- kernel -----
template <int PREC, int KP, int NW>
union LevelLds {
  TileLds<PREC, KP, NW> tile;
  double sums[kWave * NW];
};

// One task of a level launch: tile `local` of step `st` (tile_task) or update
// workgroup `local` of step `st`.  Returns the task kind (0 tile, 1 row
// update, 2 column update, 3 block deviance, -1 nothing to do).
template <int PREC, int FAM, int KP, bool WANT_DEV, int NW, bool CY = false>
__device__ __forceinline__ int run_task(const LevelArgs& a, const LevelStep& st, bool tile_task,
                                        int local, LevelLds<PREC, KP, NW>& L,
                                        unsigned long long* stamps) {
  if (tile_task) {
    const int n_b = st.n_b, m_b = st.m_b;
    const int n_ct = st.n_ct, rpw = st.rpw;
    const int rr = local / a.ct_max, ct = local % a.ct_max;
    if (rr >= st.n_rr || ct >= n_ct) return -1;   // this block has fewer tiles
    TileView tv;
    tv.ldy = st.ldy;
    tv.Y = a.Y + st.yoff;
    tv.Yc = CY ? a.Yc + st.yoff : nullptr;
    tv.W = a.W ? a.W + st.yoff : nullptr;
    tv.Prow = a.Prow + (int64_t)st.ro * a.KP;
    tv.Pcol = a.Pcol + (int64_t)st.co * a.KP;
    tv.n_b = n_b;
    tv.m_b = m_b;
    tv.row0 = rr * rpw;
    tv.row_end = min(n_b, (rr + 1) * rpw);
    tv.col0 = ct * kTileCols;
    tv.Upart = a.Upart + (int64_t)st.slot * a.slot_u_elems + (int64_t)ct * n_b * (2 * a.KU);
    tv.Vpart = a.Vpart + (int64_t)st.slot * a.slot_v_elems + (int64_t)rr * m_b * (2 * a.KV);
    tv.stamps = stamps;
    tv.alpha = a.f.alpha_col ? a.f.alpha_col + st.co : nullptr;
    const FamilyConst fc = family_const(a.f);
    const double dev =
        tv.W ? compute_tile<PREC, FAM, KP, WANT_DEV, NW, true, CY>(tv, fc, a.p, a.q, a.d, a.KU, a.KV, L.tile)
             : compute_tile<PREC, FAM, KP, WANT_DEV, NW, false, CY>(tv, fc, a.p, a.q, a.d, a.KU, a.KV, L.tile);
    if (WANT_DEV && threadIdx.x == 0)
      a.devpart[(int64_t)st.slot * a.slot_dev_elems + rr * n_ct + ct] = dev;
    return 0;
  }
  return run_update<WANT_DEV>(a, st, local, L.sums);
}

// Occupancy: two 4-wavefront tiles per compute unit, three for the bfloat16
// tile at panel stride 32 (168 registers, a few spilled outside the row-group
// loop; 29.8 against 34.4 us per 10000 x 1000 step with two).  CY: the tiles
// read the 16-bit counts.
template <int PREC, int FAM, int KP, bool WANT_DEV, int NW, bool CY>
__global__ __launch_bounds__(kWave * NW, (NW == 8) ? 1 : ((PREC == kBF16 && KP == 32) ? 3 : 2)) void level_kernel(LevelArgs a) {
  __shared__ LevelLds<PREC, KP, NW> L;
  const unsigned long long tr0 = a.trace ? wall_clock64() : 0;
  __shared__ unsigned long long stamps[3];
  const int T = a.rr_max * a.ct_max;
  const int ntile_blocks = a.n_tile_steps * T;
  int b = blockIdx.x;
  int kind;
  if (b < ntile_blocks) {
    const int v = xcd_tile(b, ntile_blocks);   // the strips of a row range on one XCD
    kind = run_task<PREC, FAM, KP, WANT_DEV, NW, CY>(a, a.steps[v / T], true, v % T, L,
                                                     a.trace ? stamps : nullptr);
  } else {
    b -= ntile_blocks;
    const int k = b / a.upd_per_step;
    if (k >= a.n_upd_steps) return;
    kind = run_task<PREC, FAM, KP, WANT_DEV, NW, CY>(a, a.steps[a.n_tile_steps + k], false,
                                                     b % a.upd_per_step, L, nullptr);
  }
  if (kind < 0) return;
  if (a.trace && threadIdx.x == 0) {
    const long long gi = (long long)a.trace_base + blockIdx.x;
    if (gi < a.trace_cap) {
      unsigned long long* rec = a.trace + 8 * gi;
      rec[0] = a.launch_id;
      rec[1] = ((unsigned long long)blockIdx.x << 32) | (unsigned)kind;
      rec[2] = tr0;
      rec[3] = wall_clock64();
      rec[4] = __smid();
      rec[5] = kind == 0 ? stamps[0] : 0;
      rec[6] = kind == 0 ? stamps[1] : 0;
      rec[7] = kind == 0 ? stamps[2] : 0;
    }
  }
}

// A launch of updates only (no tiles): the same update tasks as level_kernel
// with only their own LDS (kTileThreads doubles), so that many more update
// workgroups share a compute unit than when they carry a tile's LDS.
template <bool WANT_DEV>
__global__ __launch_bounds__(kTileThreads) void update_kernel(LevelArgs a) {
  __shared__ double sums[kTileThreads];
  const unsigned long long tr0 = a.trace ? wall_clock64() : 0;
  const int b = blockIdx.x;
  const int k = b / a.upd_per_step;
  if (k >= a.n_upd_steps) return;
  const int kind = run_update<WANT_DEV>(a, a.steps[k], b % a.upd_per_step, sums);
  if (kind < 0) return;
  if (a.trace && threadIdx.x == 0) {
    const long long gi = (long long)a.trace_base + blockIdx.x;
    if (gi < a.trace_cap) {
      unsigned long long* rec = a.trace + 8 * gi;
      rec[0] = a.launch_id;
      rec[1] = ((unsigned long long)blockIdx.x << 32) | (unsigned)kind;
      rec[2] = tr0;
      rec[3] = wall_clock64();
      rec[4] = __smid();
      rec[5] = rec[6] = rec[7] = 0;
    }
  }
}

// Batched launches over many fits (see BatchArgs): the workgroup finds its
// segment by a binary search over the launch's segment starts, takes the fit's
// descriptor and the step from the device tables, and runs the task with the
// fit's family chosen at run time (uniform over the workgroup).
template <int PREC, int KP>
__global__ __launch_bounds__(kTileThreads, 2) void batch_kernel(BatchArgs ba) {
  __shared__ LevelLds<PREC, KP, 4> L;
  // tiles numbered per XCD: the strips of a row range of one fit's step on one XCD
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  int lo = 0, hi = ba.nsegs - 1;
  while (lo < hi) {   // last segment with start <= b
    const int mid = (lo + hi + 1) >> 1;
    if (ba.segs[mid].start <= b) lo = mid; else hi = mid - 1;
  }
  const BatchSeg sg = ba.segs[lo];
  const LevelArgs& a = ba.fits[sg.fit];
  const int64_t e = (int64_t)(*ba.cursor % ba.table_epochs);
  const LevelStep& st = ba.steps[e * ba.steps_per_epoch + sg.step_index];
  const bool tile_task = sg.kind == 0;
  const int local = b - sg.start;
  switch (a.fam) {
    case kPoisson: run_task<PREC, kPoisson, KP, false, 4>(a, st, tile_task, local, L, nullptr); break;
    case kNegBin: run_task<PREC, kNegBin, KP, false, 4>(a, st, tile_task, local, L, nullptr); break;
    case kGeneric:   // FP32 only (the host refuses other precisions for these fits)
      if constexpr (PREC == kF32) run_task<PREC, kGeneric, KP, false, 4>(a, st, tile_task, local, L, nullptr);
      break;
    default: run_task<PREC, kGaussian, KP, false, 4>(a, st, tile_task, local, L, nullptr); break;
  }
}

// A batched launch of update segments only: the same update tasks with only
// their own LDS (kTileThreads doubles), so that many more of them share a
// compute unit than when they carry a tile's LDS (as update_kernel for a
// single fit).  The update tasks do not depend on the precision, family or
// panel stride of the fit (read at run time), so one kernel serves every
// batch.
__global__ __launch_bounds__(kTileThreads) void batch_update_kernel(BatchArgs ba) {
  __shared__ double sums[kTileThreads];
  const int b = blockIdx.x;
  int lo = 0, hi = ba.nsegs - 1;
  while (lo < hi) {   // last segment with start <= b
    const int mid = (lo + hi + 1) >> 1;
    if (ba.segs[mid].start <= b) lo = mid; else hi = mid - 1;
  }
  const BatchSeg sg = ba.segs[lo];
  const LevelArgs& a = ba.fits[sg.fit];
  const int64_t e = (int64_t)(*ba.cursor % ba.table_epochs);
  const LevelStep& st = ba.steps[e * ba.steps_per_epoch + sg.step_index];
  run_update<false>(a, st, b - sg.start, sums);
}

__global__ void advance_cursor_kernel(int* cursor) {
  if (threadIdx.x == 0 && blockIdx.x == 0) cursor[0] = cursor[0] + 1;
}

// ------------------------------------------------------------ launchers ----
// 8-wavefront tiles exist for the smaller panel strides (FP32 16 and 32,
// BF16 and split BF16 32).
template <int PREC, int KP>
constexpr bool has_nw8() {
  return (PREC == kF32 && (KP == 16 || KP == 32)) || (PREC != kF32 && KP == 32);
}

// cy: the 16-bit counts (Poisson and NB, bfloat16 products, 4-wavefront
// tiles; the others read the float32 counts: the FP32 tile is bound by its
// float32 products, and the conversion of the counts cost it 1 %).
template <int PREC, int FAM, int KP>
static const void* kernel_ptr(bool want_dev, int nw, bool cy) {
  if constexpr (has_nw8<PREC, KP>())
    if (nw == 8)
      return want_dev ? reinterpret_cast<const void*>(&level_kernel<PREC, FAM, KP, true, 8, false>)
                      : reinterpret_cast<const void*>(&level_kernel<PREC, FAM, KP, false, 8, false>);
  if (nw != 4) return nullptr;
  if constexpr ((FAM == kPoisson || FAM == kNegBin) && PREC != kF32)
    if (cy)
      return want_dev ? reinterpret_cast<const void*>(&level_kernel<PREC, FAM, KP, true, 4, true>)
                      : reinterpret_cast<const void*>(&level_kernel<PREC, FAM, KP, false, 4, true>);
  return want_dev ? reinterpret_cast<const void*>(&level_kernel<PREC, FAM, KP, true, 4, false>)
                  : reinterpret_cast<const void*>(&level_kernel<PREC, FAM, KP, false, 4, false>);
}

template <int PREC, int FAM>
static const void* kernel_ptr_kp(int KP, bool want_dev, int nw, bool cy) {
  switch (KP) {
    case 16: return kernel_ptr<PREC, FAM, 16>(want_dev, nw, cy);
    case 32: return kernel_ptr<PREC, FAM, 32>(want_dev, nw, cy);
    case 48: if constexpr (PREC == kF32) return kernel_ptr<PREC, FAM, 48>(want_dev, nw, cy); else break;
    case 64: return kernel_ptr<PREC, FAM, 64>(want_dev, nw, cy);
  }
  return nullptr;
}

static const void* level_kernel_for(int prec, int fam, int KP, bool want_dev, int nw, bool cy) {
  if (prec == kF32) {
    switch (fam) {
      case kPoisson: return kernel_ptr_kp<kF32, kPoisson>(KP, want_dev, nw, cy);
      case kNegBin: return kernel_ptr_kp<kF32, kNegBin>(KP, want_dev, nw, cy);
      case kGaussian: return kernel_ptr_kp<kF32, kGaussian>(KP, want_dev, nw, cy);
      case kGeneric: return kernel_ptr_kp<kF32, kGeneric>(KP, want_dev, nw, cy);
    }
  } else if (prec == kBF16) {
    switch (fam) {
      case kPoisson: return kernel_ptr_kp<kBF16, kPoisson>(KP, want_dev, nw, cy);
      case kNegBin: return kernel_ptr_kp<kBF16, kNegBin>(KP, want_dev, nw, cy);
      case kGaussian: return kernel_ptr_kp<kBF16, kGaussian>(KP, want_dev, nw, cy);
    }
  } else if (prec == kBF16X3) {
    switch (fam) {
      case kPoisson: return kernel_ptr_kp<kBF16X3, kPoisson>(KP, want_dev, nw, cy);
      case kNegBin: return kernel_ptr_kp<kBF16X3, kNegBin>(KP, want_dev, nw, cy);
      case kGaussian: return kernel_ptr_kp<kBF16X3, kGaussian>(KP, want_dev, nw, cy);
    }
  }
  return nullptr;
}

bool level_supports_nw8(int prec, int KP) {
  return (prec == kF32 && (KP == 16 || KP == 32)) ||
         ((prec == kBF16 || prec == kBF16X3) && KP == 32);
}

hipError_t launch_level(int prec, int fam, int KP, bool want_dev, int nw, const LevelArgs& a,
                        int grid, hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop) {
  if (a.n_tile_steps == 0) {   // updates only: the small-LDS kernel, kTileThreads threads
    if (grid <= 0) return hipSuccess;
    const void* uk = want_dev ? reinterpret_cast<const void*>(&update_kernel<true>)
                              : reinterpret_cast<const void*>(&update_kernel<false>);
    void* uargs[] = {const_cast<LevelArgs*>(&a)};
    if (ev_start || ev_stop)
      return hipExtLaunchKernel(uk, dim3(grid), dim3(kTileThreads), uargs, 0, s, ev_start, ev_stop, 0);
    return hipLaunchKernel(uk, dim3(grid), dim3(kTileThreads), uargs, 0, s);
  }
  const void* k = level_kernel_for(prec, fam, KP, want_dev, nw, a.Yc != nullptr);
  if (!k) return hipErrorInvalidValue;
  if (grid <= 0) return hipSuccess;
  void* args[] = {const_cast<LevelArgs*>(&a)};
  const dim3 block(kWave * nw);
  if (ev_start || ev_stop)   // events stamped by the dispatch itself: kernel execution time only
    return hipExtLaunchKernel(k, dim3(grid), block, args, 0, s, ev_start, ev_stop, 0);
  return hipLaunchKernel(k, dim3(grid), block, args, 0, s);
}

hipError_t launch_batch(int prec, int KP, const BatchArgs& a, int grid, hipStream_t s,
                        bool updates_only) {
  if (grid <= 0) return hipSuccess;
  if (updates_only) {
    void* uargs[] = {const_cast<BatchArgs*>(&a)};
    return hipLaunchKernel(reinterpret_cast<const void*>(&batch_update_kernel), dim3(grid),
                           dim3(kTileThreads), uargs, 0, s);
  }
  const void* k = nullptr;
  if (prec == kF32) {
    switch (KP) {
      case 16: k = reinterpret_cast<const void*>(&batch_kernel<kF32, 16>); break;
      case 32: k = reinterpret_cast<const void*>(&batch_kernel<kF32, 32>); break;
      case 48: k = reinterpret_cast<const void*>(&batch_kernel<kF32, 48>); break;
      case 64: k = reinterpret_cast<const void*>(&batch_kernel<kF32, 64>); break;
    }
  } else if (prec == kBF16) {
    switch (KP) {
      case 16: k = reinterpret_cast<const void*>(&batch_kernel<kBF16, 16>); break;
      case 32: k = reinterpret_cast<const void*>(&batch_kernel<kBF16, 32>); break;
      case 64: k = reinterpret_cast<const void*>(&batch_kernel<kBF16, 64>); break;
    }
  } else if (prec == kBF16X3) {
    switch (KP) {
      case 16: k = reinterpret_cast<const void*>(&batch_kernel<kBF16X3, 16>); break;
      case 32: k = reinterpret_cast<const void*>(&batch_kernel<kBF16X3, 32>); break;
      case 64: k = reinterpret_cast<const void*>(&batch_kernel<kBF16X3, 64>); break;
    }
  }
  if (!k) return hipErrorInvalidValue;
  void* args[] = {const_cast<BatchArgs*>(&a)};
  return hipLaunchKernel(k, dim3(grid), dim3(kTileThreads), args, 0, s);
}

hipError_t launch_advance_cursor(int* cursor, hipStream_t s) {
  hipLaunchKernelGGL(advance_cursor_kernel, dim3(1), dim3(64), 0, s, cursor);
  return hipGetLastError();
}

}  // namespace gmf
